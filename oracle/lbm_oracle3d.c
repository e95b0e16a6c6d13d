/*
 * lbm_oracle3d.c -- plain, slow CPU oracle for the D3Q19 and D3Q27 BGK
 * lattice Boltzmann method with the Non-equilibrium Symmetry Boundary
 * Condition (NSBC) of Euser & Vuik (arXiv 2005.08674), carried from the
 * paper's D2Q9 setting (Secs. 3 and 5) to three dimensions.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite and the benchmark's CPU baseline use
 * it.  It shares no code, header, table or helper with the GPU library.
 *
 * Arithmetic type `real`: double, or x87 extended precision with
 * -DORC_LONG_DOUBLE.
 *
 * Lattices: D3Q19 is c_0 = 0 (w 1/3); the six axis directions (w 1/18) in
 * the order +x, -x, +y, -y, +z, -z; the twelve face diagonals (w 1/36) in
 * opposite pairs (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1),
 * (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).  D3Q27 is the
 * same 19 directions followed by the eight cube diagonals in opposite pairs
 * (1,1,1), (-1,-1,-1), (1,1,-1), (-1,-1,1), (1,-1,1), (-1,1,-1), (-1,1,1),
 * (1,-1,-1), with weights 8/27, 2/27, 1/54 and 1/216 by |c|^2 = 0, 1, 2, 3.
 * c_s^2 = 1/3 for both.  Each lattice carries its own q (19 or 27).
 *
 * State: the PRE-collision deviation g_i = f_i - w_i rho0, layout
 * g[i][z][y][x] (x fastest).  One step, in the paper's order:
 *   1. moments (rho, u) of every node                      (eqs. cf_0, cf_1)
 *   2. BGK collision of every node                          (eqs. lbe_1, feq_1)
 *   3. pull streaming; a population whose source lies outside the domain
 *      across a non-periodic face is unknown                (eq. lbe_0)
 *   4. NSBC on every node of an NSBC face (eqs. nes_0..nes_4): the node's
 *      outward normal is the normalised sum of the unit outward normals of
 *      the k faces it lies on (k = 1, 2, 3), so the normal derivative is
 *      (1/sqrt k) sum_j (m_b - m_{b - n_j}); m_p = m_b - gamma * that;
 *      m_c = (1 - beta) m_p + beta m0; an unknown population takes
 *      f^eq_i(m_c) + f_opp - f^eq_opp(m_c), or f^eq_i(m_c) when its opposite
 *      is unknown too; all populations are then shifted by
 *      w_i (drho + c_i . dj / c_s^2) so that the node carries m_c.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_LONG_DOUBLE
typedef long double real;
#else
typedef double real;
#endif

#define QMAX 27

static const int CX[QMAX] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                             1, -1, 1, -1, 1, -1, -1, 1};
static const int CY[QMAX] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                             1, -1, 1, -1, -1, 1, 1, -1};
static const int CZ[QMAX] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                             1, -1, -1, 1, 1, -1, 1, -1};

/* weight from |c|^2: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216 */
static real weight(int q, int i) {
    int c2 = CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i];
    if (q == 19) {
        if (c2 == 0) return (real)1 / (real)3;
        if (c2 == 1) return (real)1 / (real)18;
        return (real)1 / (real)36;
    }
    if (c2 == 0) return (real)8 / (real)27;
    if (c2 == 1) return (real)2 / (real)27;
    if (c2 == 2) return (real)1 / (real)54;
    return (real)1 / (real)216;
}

static int opposite(int q, int i) {
    for (int j = 0; j < q; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) return j;
    return -1;
}

typedef struct {
    int nx, ny, nz;
    double tau, rho0;
    int bc[6];            /* 0 periodic, 1 NSBC: [x=0, x=nx-1, y=0, y=ny-1, z=0, z=nz-1] */
    double gamma, beta;
    double m0[4];         /* far-field vector (rho, ux, uy, uz) */
    int q;                /* velocity set: 19 or 27 */
} orc3_params;

static const real CS2 = (real)1 / (real)3;

static void node_moments(int q, const real *g, real rho0, real m[4]) {
    real s = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < q; ++i) {
        s += g[i];
        j[0] += (real)CX[i] * g[i];
        j[1] += (real)CY[i] * g[i];
        j[2] += (real)CZ[i] * g[i];
    }
    real rho = rho0 + s;
    m[0] = s;
    for (int a = 0; a < 3; ++a) m[1 + a] = j[a] / rho;
}

/* eq. feq_1 minus w_i rho0 */
static void equilibrium(int q, real rho0, const real m[4], real *geq) {
    real rho = rho0 + m[0];
    real uu = m[1] * m[1] + m[2] * m[2] + m[3] * m[3];
    for (int i = 0; i < q; ++i) {
        real cu = (real)CX[i] * m[1] + (real)CY[i] * m[2] + (real)CZ[i] * m[3];
        geq[i] = weight(q, i) * (m[0] + rho * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2)));
    }
}

static void collide(int q, real tau, real rho0, const real *g, real *out) {
    real m[4], geq[QMAX];
    node_moments(q, g, rho0, m);
    equilibrium(q, rho0, m, geq);
    for (int i = 0; i < q; ++i) out[i] = g[i] - (g[i] - geq[i]) / tau;
}

static int check_params(const orc3_params *p) {
    if (!p || p->nx < 3 || p->ny < 3 || p->nz < 3) return -1;
    if (p->q != 19 && p->q != 27) return -1;
    if (!(p->tau > 0.5)) return -1;
    for (int f = 0; f < 6; ++f)
        if (p->bc[f] != 0 && p->bc[f] != 1) return -1;
    for (int a = 0; a < 3; ++a)
        if ((p->bc[2 * a] == 0) != (p->bc[2 * a + 1] == 0)) return -1;
    return 0;
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* ---------------------------------------------------------------- node API */

/* Node functions take the velocity set q (19 or 27) and arrays of q values. */
int orc3_lattice(int q, int *c, real *w, int *opp) {
    if (q != 19 && q != 27) return -1;
    for (int i = 0; i < q; ++i) {
        c[3 * i] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = weight(q, i);
        opp[i] = opposite(q, i);
    }
    return 0;
}

int orc3_feq(int q, double rho0, const double *m4, real *out) {
    if (q != 19 && q != 27) return -1;
    real m[4] = {(real)m4[0], (real)m4[1], (real)m4[2], (real)m4[3]};
    equilibrium(q, (real)rho0, m, out);
    return 0;
}

int orc3_collide_node(int q, double tau, double rho0, const real *g, real *out) {
    if (q != 19 && q != 27) return -1;
    collide(q, (real)tau, (real)rho0, g, out);
    return 0;
}

int orc3_moments_node(int q, double rho0, const real *g, real *out4) {
    if (q != 19 && q != 27) return -1;
    node_moments(q, g, (real)rho0, out4);
    return 0;
}

/* ------------------------------------------------------------- lattice API */

int orc3_init(const orc3_params *p, const double *drho, const double *ux, const double *uy, const double *uz,
              real *g) {
    if (check_params(p)) return -1;
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    for (size_t k = 0; k < n; ++k) {
        real m[4] = {(real)drho[k], (real)ux[k], (real)uy[k], (real)uz[k]}, geq[QMAX];
        equilibrium(p->q, (real)p->rho0, m, geq);
        for (int i = 0; i < p->q; ++i) g[(size_t)i * n + k] = geq[i];
    }
    return 0;
}

int orc3_moments(const orc3_params *p, const real *g, double *out /* [4][n] */) {
    if (check_params(p)) return -1;
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    for (size_t k = 0; k < n; ++k) {
        real gn[QMAX], m[4];
        for (int i = 0; i < p->q; ++i) gn[i] = g[(size_t)i * n + k];
        node_moments(p->q, gn, (real)p->rho0, m);
        for (int a = 0; a < 4; ++a) out[(size_t)a * n + k] = (double)m[a];
    }
    return 0;
}

/* Population i of node (x, y, z) is unknown when its source lies outside the
 * domain across a non-periodic face. */
static int is_unknown(const orc3_params *p, int x, int y, int z, int i) {
    int s[3] = {x - CX[i], y - CY[i], z - CZ[i]}, nn[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a)
        if ((s[a] < 0 || s[a] >= nn[a]) && p->bc[2 * a] != 0) return 1;
    return 0;
}

int orc3_step(const orc3_params *p, real *g, int nsteps) {
    if (check_params(p) || nsteps < 0) return -1;
    const int nx = p->nx, ny = p->ny, nz = p->nz, q = p->q;
    const size_t n = (size_t)nx * ny * nz;
    const real rho0 = (real)p->rho0, tau = (real)p->tau;
    const real gamma = (real)p->gamma, beta = (real)p->beta;
    const real m0[4] = {(real)p->m0[0] - rho0, (real)p->m0[1], (real)p->m0[2], (real)p->m0[3]};
    real *mom = malloc(4 * n * sizeof(real));
    real *post = malloc((size_t)q * n * sizeof(real));
    if (!mom || !post) {
        free(mom);
        free(post);
        return -2;
    }
    int opp[QMAX];
    for (int i = 0; i < q; ++i) opp[i] = opposite(q, i);

    for (int step = 0; step < nsteps; ++step) {
        /* 1 + 2: moments and collision */
#pragma omp parallel for schedule(static)
        for (size_t k = 0; k < n; ++k) {
            real gn[QMAX], gs[QMAX], m[4];
            for (int i = 0; i < q; ++i) gn[i] = g[(size_t)i * n + k];
            node_moments(q, gn, rho0, m);
            for (int a = 0; a < 4; ++a) mom[(size_t)a * n + k] = m[a];
            collide(q, tau, rho0, gn, gs);
            for (int i = 0; i < q; ++i) post[(size_t)i * n + k] = gs[i];
        }
        /* 3: pull streaming; unknown populations are NaN until the boundary step */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    size_t k = ((size_t)z * ny + y) * nx + x;
                    for (int i = 0; i < q; ++i) {
                        if (is_unknown(p, x, y, z, i)) {
                            g[(size_t)i * n + k] = (real)NAN;
                            continue;
                        }
                        int sx = wrap(x - CX[i], nx), sy = wrap(y - CY[i], ny), sz = wrap(z - CZ[i], nz);
                        g[(size_t)i * n + k] = post[(size_t)i * n + ((size_t)sz * ny + sy) * nx + sx];
                    }
                }
        /* 4: NSBC on the nodes of the NSBC faces */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    int c[3] = {x, y, z}, nn[3] = {nx, ny, nz};
                    int in[3][3], k = 0;
                    for (int a = 0; a < 3; ++a) {
                        if (p->bc[2 * a] != 1) continue;
                        int d = 0;
                        if (c[a] == 0) d = 1;             /* inward step from the low face */
                        else if (c[a] == nn[a] - 1) d = -1;
                        if (!d) continue;
                        in[k][0] = in[k][1] = in[k][2] = 0;
                        in[k][a] = d;
                        ++k;
                    }
                    if (!k) continue;
                    size_t kb = ((size_t)z * ny + y) * nx + x;
                    real fac = gamma / sqrtl((long double)k);
                    real mc[4];
                    for (int a = 0; a < 4; ++a) {
                        real mb = mom[(size_t)a * n + kb], d = 0;
                        for (int j = 0; j < k; ++j) {
                            size_t kn = ((size_t)(z + in[j][2]) * ny + (y + in[j][1])) * nx + (x + in[j][0]);
                            d += mb - mom[(size_t)a * n + kn];
                        }
                        real mp = mb - fac * d;                 /* eq. nes_2 */
                        mc[a] = (1 - beta) * mp + beta * m0[a]; /* eq. nes_3 */
                    }
                    real gn[QMAX], geq[QMAX];
                    int unk[QMAX];
                    for (int i = 0; i < q; ++i) {
                        gn[i] = g[(size_t)i * n + kb];
                        unk[i] = is_unknown(p, x, y, z, i);
                    }
                    equilibrium(q, rho0, mc, geq);
                    for (int i = 0; i < q; ++i) {
                        if (!unk[i]) continue;
                        int o = opp[i];
                        gn[i] = unk[o] ? geq[i] : geq[i] + (gn[o] - geq[o]); /* eqs. nes_0, nes_1 */
                    }
                    /* eq. nes_4, shift with 1/c_s^2 so the node carries m_c */
                    real s = 0, j[3] = {0, 0, 0};
                    for (int i = 0; i < q; ++i) {
                        s += gn[i];
                        j[0] += (real)CX[i] * gn[i];
                        j[1] += (real)CY[i] * gn[i];
                        j[2] += (real)CZ[i] * gn[i];
                    }
                    real rc = rho0 + mc[0];
                    real dr = s - mc[0];
                    real dj[3] = {j[0] - rc * mc[1], j[1] - rc * mc[2], j[2] - rc * mc[3]};
                    for (int i = 0; i < q; ++i)
                        gn[i] -= weight(q, i) * (dr + ((real)CX[i] * dj[0] + (real)CY[i] * dj[1] + (real)CZ[i] * dj[2]) / CS2);
                    for (int i = 0; i < q; ++i) g[(size_t)i * n + kb] = gn[i];
                }
    }
    free(mom);
    free(post);
    return 0;
}
