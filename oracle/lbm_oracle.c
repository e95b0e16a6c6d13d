/*
 * lbm_oracle.c -- plain, slow CPU oracle for the D2Q9 BGK lattice Boltzmann
 * method with the Non-equilibrium Symmetry Boundary Condition (NSBC) of
 * Euser & Vuik, "A non-reflective boundary condition for LBM based on the
 * assumption of non-equilibrium symmetry" (arXiv 2005.08674).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * Arithmetic type: `real`, double by default.  Built a second time with
 * -DORC_LONG_DOUBLE it runs in x87 extended precision, which the tests use as
 * a round-off check of the double build.
 *
 * State convention.  The stored state is the PRE-collision deviation
 *     g_i(x, t) = f_i(x, t) - w_i * rho0,
 * laid out as g[i][y][x] (x fastest), i numbered as in the paper's Fig. 1.
 * One time step, written in the order the paper describes it (Sec. 3,
 * eqs. lbe_0/lbe_1/feq_1; Sec. 5, eqs. nes_0..nes_4):
 *   1. moments m(x,t) = (rho, u) of every node          (eqs. cf_0, cf_1)
 *   2. collision of every node: BGK (eqs. lbe_1, feq_1), or the
 *      multiple-relaxation-time model of Sec. 4 (eqs. mrt_lbe, mrt_vm, mrt_rm)
 *   3. streaming, pull form: g_i(x,t+1) = g*_i(x - c_i); a population whose
 *      source lies outside the domain across a non-periodic edge is unknown
 *   4. NSBC on every node of an NSBC edge:
 *        predict m_p = m - gamma d_n m   (eq. nes_2, one-sided difference
 *                                         along the inward normal, time t)
 *        far field m_c = (1-beta) m_p + beta m0               (eq. nes_3)
 *        unknown i: g_i = g_i^eq(m_c) + g_opp - g_opp^eq(m_c)  (eqs. nes_0/1)
 *        correct all nine populations so that the node carries m_c (eq. nes_4)
 *   5. the corrected boundary node collides like any other node at the next
 *      step (the paragraph after eq. nes_4).
 * A left or right edge may instead be a Dirichlet velocity edge (the inlet of
 * the paper's test case 2, whose scheme the paper only cites): its node takes
 * the prescribed velocity u_w and the density that the known populations fix,
 * rho_w = (sum_{c.n = 0} f + 2 sum_{c.n > 0} f) / (1 + u_w.n) with n the
 * outward normal (mass and normal momentum of the node), and then the same
 * assignment and correction as NSBC at m = (rho_w, u_w).
 *
 * Readings taken where the paper is silent or ambiguous are listed in the
 * design notes; the flags below select the alternatives.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_LONG_DOUBLE
typedef long double real;
#else
typedef double real;
#endif

#define Q 9

/* Paper Fig. 1: c_0 = (0,0); c_1,c_2 = (+-1,0); c_3,c_4 = (0,+-1);
 * c_5 = (1,1), c_6 = (-1,-1), c_7 = (-1,1), c_8 = (1,-1) (the tikz arrows). */
static const int CX[Q] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 0, 1, -1, 1, -1, 1, -1};

/* Weight of direction i from the table in Fig. 1 (4/9, 1/9, 1/36). */
static real weight(int i) {
    if (i == 0) return (real)4 / (real)9;
    if (i <= 4) return (real)1 / (real)9;
    return (real)1 / (real)36;
}

/* The index of the direction opposite to i, found by search (c_opp = -c_i). */
static int opposite(int i) {
    for (int j = 0; j < Q; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i]) return j;
    return -1;
}

typedef struct {
    int nx, ny;
    double tau;           /* BGK relaxation time, dt = 1 (eq. lbe_1) */
    double rho0;          /* deviation base density */
    int bc[4];            /* 0 = periodic, 1 = NSBC, 2 = Dirichlet velocity (left/right only, with
                             periodic bottom and top); [left x=0, right, bottom y=0, top] */
    double gamma;         /* eq. nes_2 */
    double beta;          /* eq. nes_3, far-field factor */
    double m0_rho, m0_ux, m0_uy;  /* eq. nes_3 reference fluid vector */
    int corr_mode;        /* 0: shift by w_i (drho + c_i.dj / c_s^2); 1: literal w_i (drho + c_i.dj) */
    int grad_order;       /* 1: two-point one-sided difference; 2: three-point */
    int corner_mode;      /* 0: diagonal normal, gamma/sqrt(2); 1: gamma/2 */
    int coll;             /* 0: BGK, eq. lbe_1; 1: MRT, eq. mrt_lbe (omega_nu = 1/tau) */
    double omega_e, omega_eps, omega_q;  /* MRT rates of e, epsilon and q (eq. mrt_rm) */
    double uw_x, uw_y;    /* velocity of the Dirichlet velocity edges */
} orc_params;

enum { BC_PERIODIC = 0, BC_NSBC = 1, BC_VELOCITY = 2 };
enum { E_LEFT = 0, E_RIGHT = 1, E_BOTTOM = 2, E_TOP = 3 };

static const real CS2 = (real)1 / (real)3; /* c_s = 1/sqrt(3) */

/* Eqs. cf_0/cf_1 in discrete form: rho = sum f_i, rho u = sum c_i f_i.
 * With f_i = w_i rho0 + g_i and sum w_i = 1, sum w_i c_i = 0:
 *   rho - rho0 = sum g_i,  rho u = sum c_i g_i. */
static void node_moments(const real g[Q], real rho0, real *drho, real *ux, real *uy) {
    real s = 0, jx = 0, jy = 0;
    for (int i = 0; i < Q; ++i) {
        s += g[i];
        jx += (real)CX[i] * g[i];
        jy += (real)CY[i] * g[i];
    }
    real rho = rho0 + s;
    *drho = s;
    *ux = jx / rho;
    *uy = jy / rho;
}

/* Eq. feq_1, minus w_i rho0:
 *   g_i^eq = w_i [ (rho - rho0) + rho ( c.u/c_s^2 + (c.u)^2/(2 c_s^4) - u.u/(2 c_s^2) ) ] */
static void equilibrium(real rho0, real drho, real ux, real uy, real geq[Q]) {
    real rho = rho0 + drho;
    real uu = ux * ux + uy * uy;
    for (int i = 0; i < Q; ++i) {
        real cu = (real)CX[i] * ux + (real)CY[i] * uy;
        geq[i] = weight(i) * (drho + rho * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2)));
    }
}

/* Eq. lbe_1 with dt = 1: g* = g - (g - g^eq)/tau. */
static void collide(real tau, real rho0, const real g[Q], real out[Q]) {
    real drho, ux, uy, geq[Q];
    node_moments(g, rho0, &drho, &ux, &uy);
    equilibrium(rho0, drho, ux, uy, geq);
    for (int i = 0; i < Q; ++i) out[i] = g[i] - (g[i] - geq[i]) / tau;
}

/* ------------------------------------------------------------------ MRT (Sec. 4)
 * Eq. mrt_lbe: f* = f - M^-1 S (m - m^eq), m = M f, m^eq = M f^eq (eq. mrt_vm).
 * The rows of M are the Gram-Schmidt orthogonalisation, under the plain sum
 * over the nine directions, of the moments named by the relaxation matrix of
 * eq. mrt_rm, in its order: density, energy e, energy square epsilon, momentum
 * j_x, energy flux q_x, j_y, q_y and the two stress components p_xx, p_xy.
 * The raw moments taken for them are
 *   1, |c|^2, |c|^4, c_x, c_x |c|^2, c_y, c_y |c|^2, c_x^2 - c_y^2, c_x c_y.
 * S = diag(C_rho, w_e, w_eps, C_jx, w_q, C_jy, w_q, w_nu, w_nu) with
 * w_nu = 1/tau; the conserved moments' constants C are free (the paper lets
 * them take any value) and are set to 0 here: those moments are not relaxed. */
static real raw_moment(int k, int i) {
    const real cx = (real)CX[i], cy = (real)CY[i], c2 = cx * cx + cy * cy;
    switch (k) {
        case 0: return 1;
        case 1: return c2;
        case 2: return c2 * c2;
        case 3: return cx;
        case 4: return cx * c2;
        case 5: return cy;
        case 6: return cy * c2;
        case 7: return cx * cx - cy * cy;
        default: return cx * cy;
    }
}

/* Gram-Schmidt: row k = raw moment k minus its projections on rows 0..k-1. */
static void mrt_matrix(real M[Q][Q]) {
    for (int k = 0; k < Q; ++k) {
        for (int i = 0; i < Q; ++i) M[k][i] = raw_moment(k, i);
        for (int j = 0; j < k; ++j) {
            real num = 0, den = 0;
            for (int i = 0; i < Q; ++i) {
                num += M[k][i] * M[j][i];
                den += M[j][i] * M[j][i];
            }
            for (int i = 0; i < Q; ++i) M[k][i] -= num / den * M[j][i];
        }
    }
}

/* Inverse of a 9 x 9 matrix by Gauss-Jordan elimination with partial pivoting. */
static int invert9(real A[Q][Q], real X[Q][Q]) {
    real a[Q][2 * Q];
    for (int r = 0; r < Q; ++r)
        for (int c = 0; c < 2 * Q; ++c) a[r][c] = c < Q ? A[r][c] : (real)(c - Q == r);
    for (int c = 0; c < Q; ++c) {
        int piv = c;
        for (int r = c + 1; r < Q; ++r)
            if (fabsl((long double)a[r][c]) > fabsl((long double)a[piv][c])) piv = r;
        if (a[piv][c] == 0) return -1;
        if (piv != c)
            for (int k = 0; k < 2 * Q; ++k) {
                real t = a[c][k];
                a[c][k] = a[piv][k];
                a[piv][k] = t;
            }
        const real d = a[c][c];
        for (int k = 0; k < 2 * Q; ++k) a[c][k] /= d;
        for (int r = 0; r < Q; ++r) {
            if (r == c || a[r][c] == 0) continue;
            const real f = a[r][c];
            for (int k = 0; k < 2 * Q; ++k) a[r][k] -= f * a[c][k];
        }
    }
    for (int r = 0; r < Q; ++r)
        for (int c = 0; c < Q; ++c) X[r][c] = a[r][Q + c];
    return 0;
}

typedef struct {
    int on;              /* 0: BGK */
    real tau;
    real M[Q][Q], Minv[Q][Q], S[Q];
} orc_coll;

static int coll_setup(const orc_params *p, orc_coll *c) {
    c->on = p->coll;
    c->tau = (real)p->tau;
    if (!c->on) return 0;
    mrt_matrix(c->M);
    if (invert9(c->M, c->Minv)) return -1;
    const real wnu = (real)1 / (real)p->tau;
    const real S[Q] = {0, (real)p->omega_e, (real)p->omega_eps, 0, (real)p->omega_q,
                       0, (real)p->omega_q, wnu, wnu};
    for (int k = 0; k < Q; ++k) c->S[k] = S[k];
    return 0;
}

/* Eq. mrt_lbe on one node (deviation form: the constant w_i rho0 cancels in
 * m - m^eq). */
static void collide_mrt(const orc_coll *c, real rho0, const real g[Q], real out[Q]) {
    real drho, ux, uy, geq[Q], m[Q], meq[Q], d[Q];
    node_moments(g, rho0, &drho, &ux, &uy);
    equilibrium(rho0, drho, ux, uy, geq);
    for (int k = 0; k < Q; ++k) {
        m[k] = 0;
        meq[k] = 0;
        for (int i = 0; i < Q; ++i) {
            m[k] += c->M[k][i] * g[i];
            meq[k] += c->M[k][i] * geq[i];
        }
        d[k] = c->S[k] * (m[k] - meq[k]);
    }
    for (int i = 0; i < Q; ++i) {
        real s = 0;
        for (int k = 0; k < Q; ++k) s += c->Minv[i][k] * d[k];
        out[i] = g[i] - s;
    }
}

static void collide_node_any(const orc_coll *c, real rho0, const real g[Q], real out[Q]) {
    if (c->on) collide_mrt(c, rho0, g, out);
    else collide(c->tau, rho0, g, out);
}

static int check_params(const orc_params *p) {
    if (!p || p->nx < 3 || p->ny < 3) return -1;
    if (p->coll != 0 && p->coll != 1) return -1;
    if (p->coll == 0 && !(p->tau > 0.5)) return -1;
    if (p->coll == 1) {
        /* every rate in (0, 2]: tau = 1/2 (zero viscosity) is allowed */
        if (!(p->tau >= 0.5)) return -1;
        const double r[3] = {p->omega_e, p->omega_eps, p->omega_q};
        for (int k = 0; k < 3; ++k)
            if (!(r[k] > 0 && r[k] <= 2)) return -1;
    }
    for (int e = 0; e < 4; ++e)
        if (p->bc[e] != BC_PERIODIC && p->bc[e] != BC_NSBC && p->bc[e] != BC_VELOCITY) return -1;
    if (p->bc[E_BOTTOM] == BC_VELOCITY || p->bc[E_TOP] == BC_VELOCITY) return -1;
    if ((p->bc[E_LEFT] == BC_VELOCITY || p->bc[E_RIGHT] == BC_VELOCITY) && p->bc[E_BOTTOM] != BC_PERIODIC) return -1;
    if ((p->bc[E_LEFT] == BC_PERIODIC) != (p->bc[E_RIGHT] == BC_PERIODIC)) return -1;
    if ((p->bc[E_BOTTOM] == BC_PERIODIC) != (p->bc[E_TOP] == BC_PERIODIC)) return -1;
    if (p->grad_order != 1 && p->grad_order != 2) return -1;
    if (p->corr_mode != 0 && p->corr_mode != 1) return -1;
    if (p->corner_mode != 0 && p->corner_mode != 1) return -1;
    return 0;
}

/* ---------------------------------------------------------------- node API */

/* g_i^eq for one node (deviation form). */
int orc_feq(double rho0, double drho, double ux, double uy, real *out9) {
    equilibrium((real)rho0, (real)drho, (real)ux, (real)uy, out9);
    return 0;
}

/* One BGK collision of one node. */
int orc_collide_node(double tau, double rho0, const real *g9, real *out9) {
    collide((real)tau, (real)rho0, g9, out9);
    return 0;
}

/* One MRT collision of one node (eq. mrt_lbe), omega_nu = 1/tau. */
int orc_collide_node_mrt(double tau, double we, double weps, double wq, double rho0, const real *g9, real *out9) {
    orc_params p;
    memset(&p, 0, sizeof p);
    p.nx = p.ny = 3;
    p.grad_order = 1;
    p.tau = tau;
    p.coll = 1;
    p.omega_e = we;
    p.omega_eps = weps;
    p.omega_q = wq;
    if (check_params(&p)) return -1;
    orc_coll c;
    if (coll_setup(&p, &c)) return -1;
    collide_mrt(&c, (real)rho0, g9, out9);
    return 0;
}

/* The transformation matrix M of eq. mrt_vm, row-major (row k = moment k). */
int orc_mrt_matrix(real *out81) {
    real M[Q][Q];
    mrt_matrix(M);
    for (int k = 0; k < Q; ++k)
        for (int i = 0; i < Q; ++i) out81[k * Q + i] = M[k][i];
    return 0;
}

/* Moments of one node: (rho - rho0, ux, uy). */
int orc_moments_node(double rho0, const real *g9, real *out3) {
    node_moments(g9, (real)rho0, &out3[0], &out3[1], &out3[2]);
    return 0;
}

int orc_lattice_c(int *cx9, int *cy9, real *w9, int *opp9) {
    for (int i = 0; i < Q; ++i) {
        cx9[i] = CX[i];
        cy9[i] = CY[i];
        w9[i] = weight(i);
        opp9[i] = opposite(i);
    }
    return 0;
}

/* ------------------------------------------------------------- lattice API */

/* g(x, 0) = g^eq(rho, u): no initial non-equilibrium part.
 * drho = rho - rho0, ux, uy are row-major [ny][nx] fields. */
int orc_init(const orc_params *p, const double *drho, const double *ux, const double *uy, real *g) {
    if (check_params(p)) return -1;
    const size_t n = (size_t)p->nx * p->ny;
    for (size_t k = 0; k < n; ++k) {
        real geq[Q];
        equilibrium((real)p->rho0, (real)drho[k], (real)ux[k], (real)uy[k], geq);
        for (int i = 0; i < Q; ++i) g[(size_t)i * n + k] = geq[i];
    }
    return 0;
}

/* Moments of every node: rho - rho0, ux, uy as [ny][nx] doubles. */
int orc_moments(const orc_params *p, const real *g, double *drho, double *ux, double *uy) {
    if (check_params(p)) return -1;
    const size_t n = (size_t)p->nx * p->ny;
    for (size_t k = 0; k < n; ++k) {
        real gn[Q], d, a, b;
        for (int i = 0; i < Q; ++i) gn[i] = g[(size_t)i * n + k];
        node_moments(gn, (real)p->rho0, &d, &a, &b);
        drho[k] = (double)d;
        ux[k] = (double)a;
        uy[k] = (double)b;
    }
    return 0;
}

/* The post-collision populations g* of every node (step 2 of the step
 * alone): the quantity the GPU library keeps in its buffers. */
int orc_post_collision(const orc_params *p, const real *g, real *out) {
    if (check_params(p)) return -1;
    orc_coll c;
    if (coll_setup(p, &c)) return -1;
    const size_t n = (size_t)p->nx * p->ny;
    for (size_t k = 0; k < n; ++k) {
        real gn[Q], gs[Q];
        for (int i = 0; i < Q; ++i) gn[i] = g[(size_t)i * n + k];
        collide_node_any(&c, (real)p->rho0, gn, gs);
        for (int i = 0; i < Q; ++i) out[(size_t)i * n + k] = gs[i];
    }
    return 0;
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Population i of node (x, y) is unknown after streaming when its source
 * x - c_i lies outside the domain across a non-periodic (NSBC) edge. */
static int is_unknown(const orc_params *p, int x, int y, int i) {
    int sx = x - CX[i], sy = y - CY[i];
    if ((sx < 0 || sx >= p->nx) && p->bc[E_LEFT] != BC_PERIODIC) return 1;
    if ((sy < 0 || sy >= p->ny) && p->bc[E_BOTTOM] != BC_PERIODIC) return 1;
    return 0;
}

/* Normal-derivative estimate of one moment component along an inward
 * direction (ix, iy) from node (x, y): m_b - m_{b-n} (first order) or
 * (3 m_b - 4 m_{b-n} + m_{b-2n}) / 2 (second order), where b - n is the
 * node one step inward. The result is n . grad m for the OUTWARD normal n. */
static real normal_diff(const real *m, int nx, int x, int y, int ix, int iy, int order) {
    real mb = m[(size_t)y * nx + x];
    real m1 = m[(size_t)(y + iy) * nx + (x + ix)];
    if (order == 1) return mb - m1;
    real m2 = m[(size_t)(y + 2 * iy) * nx + (x + 2 * ix)];
    return (3 * mb - 4 * m1 + m2) / 2;
}

/* Advance the pre-collision state g by nsteps time steps. */
int orc_step(const orc_params *p, real *g, int nsteps) {
    if (check_params(p) || nsteps < 0) return -1;
    orc_coll coll;
    if (coll_setup(p, &coll)) return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    const real rho0 = (real)p->rho0;
    const real gamma = (real)p->gamma, beta = (real)p->beta;
    const real m0[3] = {(real)p->m0_rho - rho0, (real)p->m0_ux, (real)p->m0_uy};

    real *mr = malloc(n * sizeof(real));
    real *mu = malloc(n * sizeof(real));
    real *mv = malloc(n * sizeof(real));
    real *post = malloc(Q * n * sizeof(real));
    if (!mr || !mu || !mv || !post) {
        free(mr); free(mu); free(mv); free(post);
        return -2;
    }
    int opp[Q];
    for (int i = 0; i < Q; ++i) opp[i] = opposite(i);

    for (int step = 0; step < nsteps; ++step) {
        /* 1 + 2: moments at time t and collision of every node (BGK or MRT). */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                size_t k = (size_t)y * nx + x;
                real gn[Q], gs[Q];
                for (int i = 0; i < Q; ++i) gn[i] = g[(size_t)i * n + k];
                node_moments(gn, rho0, &mr[k], &mu[k], &mv[k]);
                collide_node_any(&coll, rho0, gn, gs);
                for (int i = 0; i < Q; ++i) post[(size_t)i * n + k] = gs[i];
            }
        }
        /* 3: pull streaming, eq. lbe_0.  Unknown populations are set to NaN
         * here and must all be overwritten by the boundary step. */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                for (int i = 0; i < Q; ++i) {
                    int known = !is_unknown(p, x, y, i);
                    int sx = wrap(x - CX[i], nx), sy = wrap(y - CY[i], ny);
                    g[(size_t)i * n + (size_t)y * nx + x] =
                        known ? post[(size_t)i * n + (size_t)sy * nx + sx] : (real)NAN;
                }
            }
        }
        /* 4: NSBC on every node that lies on an NSBC edge; the Dirichlet
         * velocity rule on every node of a velocity edge. */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                int on[4] = {x == 0 && p->bc[E_LEFT] == BC_NSBC,
                             x == nx - 1 && p->bc[E_RIGHT] == BC_NSBC,
                             y == 0 && p->bc[E_BOTTOM] == BC_NSBC,
                             y == ny - 1 && p->bc[E_TOP] == BC_NSBC};
                int count = on[0] + on[1] + on[2] + on[3];
                int vel_nx = 0;   /* outward normal x of a velocity edge this node is on */
                if (x == 0 && p->bc[E_LEFT] == BC_VELOCITY) vel_nx = -1;
                if (x == nx - 1 && p->bc[E_RIGHT] == BC_VELOCITY) vel_nx = 1;
                if (!count && !vel_nx) continue;
                size_t k = (size_t)y * nx + x;
                if (vel_nx) {
                    /* rho_w from the known populations (mass and normal momentum), then
                     * assignment and correction at m = (rho_w, u_w) */
                    real f[Q], known = 0;
                    for (int i = 0; i < Q; ++i) f[i] = g[(size_t)i * n + k] + weight(i) * rho0;
                    for (int i = 0; i < Q; ++i) {
                        int cn = CX[i] * vel_nx;
                        if (cn == 0) known += f[i];
                        else if (cn > 0) known += 2 * f[i];
                    }
                    const real uwx = (real)p->uw_x, uwy = (real)p->uw_y;
                    const real rhow = known / (1 + uwx * (real)vel_nx);
                    real mcv[3] = {rhow - rho0, uwx, uwy}, gn[Q], geq[Q];
                    int unknown[Q];
                    for (int i = 0; i < Q; ++i) {
                        gn[i] = g[(size_t)i * n + k];
                        unknown[i] = is_unknown(p, x, y, i);
                    }
                    equilibrium(rho0, mcv[0], mcv[1], mcv[2], geq);
                    for (int i = 0; i < Q; ++i) {
                        if (!unknown[i]) continue;
                        int o = opp[i];
                        gn[i] = unknown[o] ? geq[i] : geq[i] + (gn[o] - geq[o]);
                    }
                    real sm = 0, jx = 0, jy = 0;
                    for (int i = 0; i < Q; ++i) {
                        sm += gn[i];
                        jx += (real)CX[i] * gn[i];
                        jy += (real)CY[i] * gn[i];
                    }
                    const real rc = rho0 + mcv[0];
                    const real ddr = sm - mcv[0], djx = jx - rc * mcv[1], djy = jy - rc * mcv[2];
                    const real kf = p->corr_mode == 0 ? (real)1 / CS2 : (real)1;
                    for (int i = 0; i < Q; ++i)
                        gn[i] -= weight(i) * (ddr + kf * ((real)CX[i] * djx + (real)CY[i] * djy));
                    for (int i = 0; i < Q; ++i) g[(size_t)i * n + k] = gn[i];
                    continue;
                }
                /* inward unit steps of the (at most two) NSBC edges this node is on */
                int inx[2], iny[2], ne = 0;
                if (on[E_LEFT])   { inx[ne] = 1;  iny[ne] = 0;  ++ne; }
                if (on[E_RIGHT])  { inx[ne] = -1; iny[ne] = 0;  ++ne; }
                if (on[E_BOTTOM]) { inx[ne] = 0;  iny[ne] = 1;  ++ne; }
                if (on[E_TOP])    { inx[ne] = 0;  iny[ne] = -1; ++ne; }

                /* eq. nes_2: m_p = m - gamma d_n m, time-t moments. */
                const real *mf[3] = {mr, mu, mv};
                real mp[3], mc[3];
                for (int c = 0; c < 3; ++c) {
                    real mb = mf[c][k];
                    if (ne == 1) {
                        mp[c] = mb - gamma * normal_diff(mf[c], nx, x, y, inx[0], iny[0], p->grad_order);
                    } else {
                        /* corner: outward normal along the diagonal */
                        real fac = p->corner_mode == 0 ? (real)1 / sqrtl(2.0L) : (real)1 / (real)2;
                        real d = normal_diff(mf[c], nx, x, y, inx[0], iny[0], p->grad_order) +
                                 normal_diff(mf[c], nx, x, y, inx[1], iny[1], p->grad_order);
                        mp[c] = mb - gamma * fac * d;
                    }
                    /* eq. nes_3 */
                    mc[c] = (1 - beta) * mp[c] + beta * m0[c];
                }

                /* eqs. nes_0/nes_1: f_in = f_in^eq + f_out^neq, equilibria at m_c */
                real gn[Q], geq[Q];
                int unknown[Q];
                for (int i = 0; i < Q; ++i) {
                    gn[i] = g[(size_t)i * n + k];
                    unknown[i] = is_unknown(p, x, y, i);
                }
                equilibrium(rho0, mc[0], mc[1], mc[2], geq);
                for (int i = 0; i < Q; ++i) {
                    if (!unknown[i]) continue;
                    int o = opp[i];
                    if (unknown[o]) gn[i] = geq[i];          /* buried pair: no known partner */
                    else gn[i] = geq[i] + (gn[o] - geq[o]);
                }

                /* eq. nes_4: rescale with respect to rho_c, shift with respect to u_c */
                real s = 0, jx = 0, jy = 0;
                for (int i = 0; i < Q; ++i) {
                    s += gn[i];
                    jx += (real)CX[i] * gn[i];
                    jy += (real)CY[i] * gn[i];
                }
                real rhoc = rho0 + mc[0];
                real ddr = s - mc[0];                /* sum f_i - rho_c */
                real djx = jx - rhoc * mc[1];        /* sum c_i f_i - rho_c u_c */
                real djy = jy - rhoc * mc[2];
                real kfac = p->corr_mode == 0 ? (real)1 / CS2 : (real)1;
                for (int i = 0; i < Q; ++i)
                    gn[i] -= weight(i) * (ddr + kfac * ((real)CX[i] * djx + (real)CY[i] * djy));
                for (int i = 0; i < Q; ++i) g[(size_t)i * n + k] = gn[i];
            }
        }
    }
    free(mr); free(mu); free(mv); free(post);
    return 0;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int orc_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_real_bytes(void) { return (int)sizeof(real); }
