// lbm_device.h -- device-side building blocks of the D2Q9 BGK/MRT + NSBC
// sweep for gfx950: lattice constants, storage codecs, the per-node BGK and
// MRT updates, the NSBC boundary-node update, and the lattice descriptor every
// kernel takes.
//
// Method: Euser & Vuik (arXiv 2005.08674), Sec. 3 (eqs. lbe_0, lbe_1, feq_1,
// moments eqs. cf_0/cf_1), Sec. 4 (eqs. mrt_lbe, mrt_vm, mrt_rm) and Sec. 5
// (eqs. nes_0..nes_4).
//
// State convention: a population buffer holds the POST-collision deviations
// g*_i = f*_i - f^eq_i(rho0, u_b) of time t, the distance from the discrete
// equilibrium of a base state (rho0, u_b); with u_b = 0 this is
// f_i - w_i rho0.  All node arithmetic runs on (drho, du) = (rho - rho0,
// u - u_b), which keeps every operand proportional to the deviation from the
// base state and so keeps rounding errors proportional to it too.  One step pulls g*_i(x - c_i) into node x
// (streaming, eq. lbe_0), rebuilds the populations that no neighbour supplies
// on NSBC edges (eqs. nes_0..nes_4), collides (eq. lbe_1) and writes the
// post-collision set of time t+1 to the other buffer.  Collision conserves
// mass and momentum, so the moments of the stored set are the moments of the
// pre-collision state at the same time.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ------------------------------------------------------------------ lattice
// Directions as numbered in the paper's Fig. 1 (y up).
constexpr int kCx[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
constexpr int kOpp[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};

template <class R>
__host__ __device__ constexpr R wgt(int i) {
  return i == 0 ? R(4) / R(9) : (i <= 4 ? R(1) / R(9) : R(1) / R(36));
}

enum Store : int { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };
enum Edge : int { E_LEFT = 0, E_RIGHT = 1, E_BOTTOM = 2, E_TOP = 3 };
enum Bc : int { BC_PERIODIC = 0, BC_NSBC = 1, BC_VELOCITY = 2 };
enum Coll : int { COLL_BGK = 0, COLL_MRT = 1 };

// ------------------------------------------------------------------ codecs
// Stored type T, arithmetic type R.  The 16-bit codecs keep s = g / w_i * 2^k;
// dec multiplies by ds_i = w_i 2^-k, enc by es_i = 2^k / w_i, then rounds to
// nearest even.
template <int S> struct Codec;

// dec(v, s) = raw(v) * s and enc(v, s) = raw_enc(v * s): raw and raw_enc
// convert without the per-population scale (the stored value itself in the
// arithmetic type); `scaled` marks the formats whose scale is not 1.
template <> struct Codec<ST_F64> {
  using T = double;
  using R = double;
  static constexpr bool scaled = false;
  __device__ static inline R raw(T v) { return v; }
  __device__ static inline T raw_enc(R v) { return v; }
  __device__ static inline R dec(T v, float) { return v; }
  __device__ static inline T enc(R v, float) { return v; }
};

template <> struct Codec<ST_F32> {
  using T = float;
  using R = float;
  static constexpr bool scaled = false;
  __device__ static inline R raw(T v) { return v; }
  __device__ static inline T raw_enc(R v) { return v; }
  __device__ static inline R dec(T v, float) { return v; }
  __device__ static inline T enc(R v, float) { return v; }
};

template <> struct Codec<ST_F16> {
  using T = _Float16;
  using R = float;
  static constexpr bool scaled = true;
  __device__ static inline R raw(T v) { return static_cast<float>(v); }
  // The value is rounded to f32 first and then to f16 in every kernel: the
  // empty asm keeps the compiler from folding the operation that produced v
  // into one mixed-precision FMA that rounds to f16 once (it does so at some
  // sites and not at others, and the two roundings differ in rare ties).
  __device__ static inline T raw_enc(R v) {
    __asm__("" : "+v"(v));
    return static_cast<_Float16>(v);
  }
  __device__ static inline R dec(T v, float s) { return raw(v) * s; }
  __device__ static inline T enc(R v, float s) { return raw_enc(v * s); }
};

template <> struct Codec<ST_BF16> {
  using T = uint16_t;
  using R = float;
  static constexpr bool scaled = true;
  __device__ static inline R raw(T v) { return __uint_as_float(static_cast<uint32_t>(v) << 16); }
  // round to nearest, ties to even (one v_cvt_pk_bf16_f32 on gfx950)
  __device__ static inline T raw_enc(R v) { return __builtin_bit_cast(T, static_cast<__bf16>(v)); }
  __device__ static inline R dec(T v, float s) { return raw(v) * s; }
  __device__ static inline T enc(R v, float s) { return raw_enc(v * s); }
};

// ------------------------------------------------------------------ lattice descriptor
// Everything a kernel needs to update one lattice.  Buffers buf[0], buf[1]
// hold 9 planes each: population i of node (x, y) is at
// buf[b] + i * plane + y * pitch + x (elements of the stored type).
struct LatDesc {
  void* buf[2];
  int32_t nx, ny, pitch, store;
  int64_t plane;
  int32_t bc[4];
  int32_t corr_mode, grad_order, corner_mode, _pad1;
  double omega;     // 1 / tau
  double rho0;
  double gamma;
  double beta;
  double m0[3];     // far-field vector (rho - rho0, ux - ubx, uy - uby)
  double ub[2];     // base velocity u_b of the deviation form
  double pb[9];     // P_i(u_b) = 1 + 3 c_i.u_b + 9/2 (c_i.u_b)^2 - 3/2 |u_b|^2
  float ds[9];      // decode scale per population
  float es[9];      // encode scale per population
  float sc;         // 2^k: ds[i] = w_i / sc, es[i] = sc / w_i for the 16-bit formats; 1 otherwise
  const void* net;  // closure network (lbm::mlp::Net) or null
  int32_t closure;  // 1: the edge kernel replaces NSBC's m_c by the network's, NSBC as fallback
  int32_t ub_zero;  // 1 when u_b = (0, 0): the arithmetic drops the u_b terms
  float ubf[2];     // u_b and P_i(u_b) rounded to fp32 once, for the fp32 arithmetic
  float pbf[9];
  int32_t coll;     // COLL_BGK or COLL_MRT
  double mk[4];     // MRT: omega_e/36, omega_eps/36, omega_q/12, omega_nu/4 (see mrt())
  float mkf[4];     // the same rounded to fp32
  double uw[2];     // velocity of Dirichlet velocity edges
  double duw[2];    // uw - u_b
  float uwf[2];     // the same two rounded to fp32
  float duwf[2];
};

// Buffer `parity` (0 or 1) of a lattice.  A select rather than an indexed
// access, so a descriptor copied into registers stays in registers.
__host__ __device__ inline void* buf_of(const LatDesc& L, int parity) { return parity ? L.buf[1] : L.buf[0]; }

// Base state of the deviation form in the arithmetic type.  `zero` marks
// u_b = 0, for which the u_b terms below vanish exactly and are skipped (the
// remaining operations and their order are unchanged, so both forms round
// alike).
template <class R> struct Base;
template <> struct Base<double> {
  double ubx, uby;
  double pb[9];
  bool zero;
  __device__ inline explicit Base(const LatDesc& L) : ubx(L.ub[0]), uby(L.ub[1]), zero(L.ub_zero != 0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) pb[i] = L.pb[i];
  }
};
template <> struct Base<float> {
  float ubx, uby;
  float pb[9];
  bool zero;
  __device__ inline explicit Base(const LatDesc& L) : ubx(L.ubf[0]), uby(L.ubf[1]), zero(L.ub_zero != 0) {
#pragma unroll
    for (int i = 0; i < 9; ++i) pb[i] = L.pbf[i];
  }
};

// ------------------------------------------------------------------ per-node arithmetic
// 1 / x: fp64 divides (correctly rounded); fp32 takes the hardware
// reciprocal (v_rcp_f32, within 1 ulp), which every kernel shares, so all
// launch paths of one storage format still round alike.
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Moments of one node (eqs. cf_0/cf_1) from the deviations: with
// sum_i f^eq_i(rho0, u_b) = rho0 and sum_i c_i f^eq_i(rho0, u_b) = rho0 u_b,
//   drho = sum g_i,  rho u = rho0 u_b + sum c_i g_i,
//   du = u - u_b = (sum c_i g_i - drho u_b) / (rho0 + drho).
template <class R>
__device__ inline void moments(const R g[9], R rho0, const Base<R>& b, R& drho, R& dux, R& duy) {
  drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  const R jx = (g[1] - g[2]) + (g[5] - g[6]) + (g[8] - g[7]);
  const R jy = (g[3] - g[4]) + (g[5] - g[6]) + (g[7] - g[8]);
  const R ir = recip(rho0 + drho);
  if (b.zero) {
    dux = jx * ir;
    duy = jy * ir;
  } else {
    dux = (jx - drho * b.ubx) * ir;
    duy = (jy - drho * b.uby) * ir;
  }
}

// Discrete equilibrium (eq. feq_1, c_s^2 = 1/3) minus the base equilibrium:
//   f^eq_i(rho, u) - f^eq_i(rho0, u_b) = w_i [ drho P_i(u_b) + rho (P_i(u) - P_i(u_b)) ],
//   P_i(u) - P_i(u_b) = a (3 + 9/2 (a + 2 b_i)) - 3/2 du.(du + 2 u_b),
// with a = c_i.du and b_i = c_i.u_b.  For u_b = 0 this is
//   w_i [ drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u) ].
template <class R>
__device__ inline void equilibrium(R rho0, const Base<R>& b, R drho, R dux, R duy, R geq[9]) {
  const R rho = rho0 + drho;
  if (b.zero) {
    // u_b = 0: b_i = 0 and P_i(u_b) = 1, so w_i [drho + rho (a (3 + 9/2 a) - 3/2 du.du)]
    const R q = R(1.5) * (dux * dux + duy * duy);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const R a = R(kCx[i]) * dux + R(kCy[i]) * duy;
      geq[i] = wgt<R>(i) * (drho + rho * fma(a, fma(R(4.5), a, R(3)), -q));
    }
    return;
  }
  const R q = R(1.5) * (dux * (dux + R(2) * b.ubx) + duy * (duy + R(2) * b.uby));
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const R a = R(kCx[i]) * dux + R(kCy[i]) * duy;
    const R bi2 = R(2) * (R(kCx[i]) * b.ubx + R(kCy[i]) * b.uby);
    geq[i] = wgt<R>(i) * fma(drho, b.pb[i], rho * fma(a, fma(R(4.5), a + bi2, R(3)), -q));
  }
}

// BGK collision in place (eq. lbe_1, dt = 1): g <- g + omega (g^eq - g).
// For u_b = 0 the update is written per pair of opposite directions (i, i'),
// whose a = c_i.du differ in sign only:
//   g^eq_i = w_i (E + rho (9/2 a^2 +- 3 a)),  E = drho - 3/2 rho |du|^2,
//   g_i <- (1 - omega) g_i + (omega w_i) (E + 9/2 rho a^2 +- 3 rho a),
// which shares the even part between the two directions and folds w_i into
// omega (about a fifth fewer operations than the per-direction form below).
template <class R>
__device__ inline void bgk(R g[9], R rho0, const Base<R>& b, R omega) {
  R drho, dux, duy;
  moments(g, rho0, b, drho, dux, duy);
  if (b.zero) {
    const R rho = rho0 + drho;
    const R e = fma(-rho, R(1.5) * fma(dux, dux, duy * duy), drho);
    const R r45 = R(4.5) * rho, r3 = R(3) * rho;
    const R om1 = R(1) - omega;
    const R ow0 = omega * wgt<R>(0), ow1 = omega * wgt<R>(1), ow5 = omega * wgt<R>(5);
    g[0] = fma(ow0, e, om1 * g[0]);
    // one pair: directions i (a) and j (-a)
    auto pair = [&](int i, int j, R a, R ow) {
      const R even = fma(r45 * a, a, e), odd = r3 * a;
      g[i] = fma(ow, even + odd, om1 * g[i]);
      g[j] = fma(ow, even - odd, om1 * g[j]);
    };
    pair(1, 2, dux, ow1);
    pair(3, 4, duy, ow1);
    pair(5, 6, dux + duy, ow5);
    pair(7, 8, duy - dux, ow5);
    return;
  }
  R geq[9];
  equilibrium(rho0, b, drho, dux, duy, geq);
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i] = fma(omega, geq[i] - g[i], g[i]);
}

// MRT collision in place (eq. mrt_lbe): g <- g - M^-1 S M (g - g^eq).
// The rows of M are orthogonal, so M^-1 = M^T diag(1 / |row_k|^2) and the
// update is a sum over the six non-conserved moments k of
//   row_k[i] * s_k / |row_k|^2 * (row_k . n),   n = g - g^eq.
// For the Fig. 1 numbering the rows (Gram-Schmidt of 1, |c|^2, |c|^4, c_x,
// c_x |c|^2, c_y, c_y |c|^2, c_x^2 - c_y^2, c_x c_y, up to a scale each) are
//   e   = (-4, -1, -1, -1, -1,  2,  2,  2,  2)     |e|^2   = 36
//   eps = ( 4, -2, -2, -2, -2,  1,  1,  1,  1)     |eps|^2 = 36
//   q_x = ( 0, -2,  2,  0,  0,  1, -1, -1,  1)     |q|^2   = 12
//   q_y = ( 0,  0,  0, -2,  2,  1, -1,  1, -1)
//   p_xx = (0,  1,  1, -1, -1,  0,  0,  0,  0)     |p|^2   = 4
//   p_xy = (0,  0,  0,  0,  0,  1,  1, -1, -1)
// k = (omega_e/36, omega_eps/36, omega_q/12, omega_nu/4).  The conserved
// moments (density, momentum) are not relaxed: their non-equilibrium parts
// are zero up to rounding.
template <class R>
__device__ inline void mrt(R g[9], R rho0, const Base<R>& b, const R k[4]) {
  R drho, dux, duy, n[9];
  moments(g, rho0, b, drho, dux, duy);
  equilibrium(rho0, b, drho, dux, duy, n);
#pragma unroll
  for (int i = 0; i < 9; ++i) n[i] = g[i] - n[i];
  const R ax = (n[1] + n[2]) + (n[3] + n[4]);
  const R dg = (n[5] + n[6]) + (n[7] + n[8]);
  const R E = k[0] * ((dg + dg) - (ax + R(4) * n[0]));
  const R P = k[1] * ((R(4) * n[0] + dg) - (ax + ax));
  const R d56 = n[5] - n[6], d78 = n[7] - n[8];
  const R QX = k[2] * ((d56 - d78) - R(2) * (n[1] - n[2]));
  const R QY = k[2] * ((d56 + d78) - R(2) * (n[3] - n[4]));
  const R XX = k[3] * ((n[1] + n[2]) - (n[3] + n[4]));
  const R XY = k[3] * ((n[5] + n[6]) - (n[7] + n[8]));
  const R axial = E + R(2) * P;                 // common part of directions 1..4: -(-E - 2P)
  const R diag = R(2) * E + P;                  // common part of directions 5..8
  g[0] -= R(4) * (P - E);
  g[1] += axial + R(2) * QX - XX;
  g[2] += axial - R(2) * QX - XX;
  g[3] += axial + R(2) * QY + XX;
  g[4] += axial - R(2) * QY + XX;
  g[5] -= diag + (QX + QY) + XY;
  g[6] -= diag - (QX + QY) + XY;
  g[7] -= diag - (QX - QY) - XY;
  g[8] -= diag + (QX - QY) - XY;
}

// A descriptor value in the arithmetic type: the fp64 field, or its fp32 copy.
template <class R> __device__ inline R in_type(double d, float f);
template <> __device__ inline double in_type<double>(double d, float) { return d; }
template <> __device__ inline float in_type<float>(double, float f) { return f; }

template <class R> __device__ inline const R* mrt_k(const LatDesc& L);
template <> __device__ inline const double* mrt_k<double>(const LatDesc& L) { return L.mk; }
template <> __device__ inline const float* mrt_k<float>(const LatDesc& L) { return L.mkf; }

// The lattice's collision (BGK, eq. lbe_1, or MRT, eq. mrt_lbe), in place.
// CM fixes the model at compile time (COLL_BGK or COLL_MRT); the default -1
// reads it from the descriptor.
template <class R, int CM = -1>
__device__ inline void collide(const LatDesc& L, R g[9], R rho0, const Base<R>& b, R omega);

// BGK on the stored values s_i = g_i / d_i of the 16-bit formats (d_i =
// w_i / 2^k, three values: rest, axis, diagonal).  The moments are summed
// from s by weight class, and with g^eq_i = w_i X_i (eq. feq_1) the update
// g_i <- g_i + omega (g^eq_i - g_i) becomes s_i <- s_i + omega (2^k X_i - s_i):
// the weights cancel, so no population is scaled on the way in or out.  For
// u_b = 0 it is written per pair of opposite directions as in bgk, with
// omega 2^k taken into the pair's terms once per node (one factor for all
// nine directions): s_i <- (1 - omega) s_i + (q_E + q_45 a^2 +- q_3 a).
template <class R>
__device__ inline void bgk_stored(R s[9], R rho0, const Base<R>& b, R omega, R d0, R d1, R d5, R sc) {
  const R drho = fma(d0, s[0], fma(d1, (s[1] + s[2]) + (s[3] + s[4]), d5 * ((s[5] + s[6]) + (s[7] + s[8]))));
  const R jx = fma(d1, s[1] - s[2], d5 * ((s[5] - s[6]) + (s[8] - s[7])));
  const R jy = fma(d1, s[3] - s[4], d5 * ((s[5] - s[6]) + (s[7] - s[8])));
  const R ir = recip(rho0 + drho);
  const R rho = rho0 + drho;
  if (b.zero) {
    const R dux = jx * ir, duy = jy * ir;
    const R e = fma(-rho, R(1.5) * fma(dux, dux, duy * duy), drho);
    const R om1 = R(1) - omega, osc = omega * sc;
    const R qe = osc * e, q45 = (R(4.5) * osc) * rho, q3 = (R(3) * osc) * rho;
    s[0] = fma(om1, s[0], qe);
    auto pair = [&](int i, int j, R a) {
      const R even = fma(q45 * a, a, qe), odd = q3 * a;
      s[i] = fma(om1, s[i], even + odd);
      s[j] = fma(om1, s[j], even - odd);
    };
    pair(1, 2, dux);
    pair(3, 4, duy);
    pair(5, 6, dux + duy);
    pair(7, 8, duy - dux);
    return;
  }
  // u_b != 0, per pair (i, j) of opposite directions, where a = c_i.du and
  // b = c_i.u_b both change sign: with P_i(u_b) = pe + 3 b,
  //   X_i = drho (pe +- 3 b) + rho (9/2 a (a + 2 b) +- 3 a - q),
  // so the pair shares the even part; omega 2^k is taken into drho and rho
  // once per node
  const R dux = (jx - drho * b.ubx) * ir, duy = (jy - drho * b.uby) * ir;
  const R q = R(1.5) * (dux * (dux + R(2) * b.ubx) + duy * (duy + R(2) * b.uby));
  const R om1 = R(1) - omega, osc = omega * sc;
  const R dro = osc * drho, rro = osc * rho, dro3 = R(3) * dro, rro3 = R(3) * rro;
  s[0] = fma(om1, s[0], fma(dro, b.pb[0], -(rro * q)));
  auto pair = [&](int i, int j, R a) {
    const R bi = R(kCx[i]) * b.ubx + R(kCy[i]) * b.uby;
    const R pe = R(0.5) * (b.pb[i] + b.pb[j]);
    const R even = fma(dro, pe, rro * fma(a, R(4.5) * (a + R(2) * bi), -q));
    const R odd = fma(rro3, a, dro3 * bi);
    s[i] = fma(om1, s[i], even + odd);
    s[j] = fma(om1, s[j], even - odd);
  };
  pair(1, 2, dux);
  pair(3, 4, duy);
  pair(5, 6, dux + duy);
  pair(7, 8, duy - dux);
}

// Collision of an interior node on its values as stored (Codec::raw, back
// with Codec::raw_enc), the form every sweep uses for interior nodes; NSBC
// and velocity-edge nodes decode, take collide and encode.  The 32/64-bit
// formats store g itself; the 16-bit ones take bgk_stored for BGK and the
// scaled round trip for MRT (the same operations as decode, collide,
// encode).
template <int S, int CM>
__device__ inline void collide_stored(const LatDesc& L, typename Codec<S>::R s[9], typename Codec<S>::R rho0,
                                      const Base<typename Codec<S>::R>& b, typename Codec<S>::R omega) {
  using R = typename Codec<S>::R;
  if constexpr (!Codec<S>::scaled) {
    collide<R, CM>(L, s, rho0, b, omega);
  } else {
    if (CM == COLL_MRT || (CM < 0 && L.coll == COLL_MRT)) {
#pragma unroll
      for (int i = 0; i < 9; ++i) s[i] *= L.ds[i];
      collide<R, COLL_MRT>(L, s, rho0, b, omega);
#pragma unroll
      for (int i = 0; i < 9; ++i) s[i] *= L.es[i];
    } else {
      bgk_stored<R>(s, rho0, b, omega, R(L.ds[0]), R(L.ds[1]), R(L.ds[5]), R(L.sc));
    }
  }
}

template <class R, int CM>
__device__ inline void collide(const LatDesc& L, R g[9], R rho0, const Base<R>& b, R omega) {
  if (CM == COLL_MRT || (CM < 0 && L.coll == COLL_MRT)) {
    const R* kp = mrt_k<R>(L);
    const R k[4] = {kp[0], kp[1], kp[2], kp[3]};
    mrt<R>(g, rho0, b, k);
  } else {
    bgk<R>(g, rho0, b, omega);
  }
}

template <int S>
__device__ inline typename Codec<S>::R load_pop(const LatDesc& L, const typename Codec<S>::T* base, int i,
                                                int64_t idx) {
  return Codec<S>::dec(base[i * L.plane + idx], L.ds[i]);
}

// ------------------------------------------------------------------ NSBC
// Moment triple (drho, ux - ubx, uy - uby).
template <class R> struct M3 {
  R v[3];
};

// Dirichlet velocity edge (left or right, with periodic bottom and top): the
// node takes the prescribed velocity u_w and the density its known
// populations fix -- mass and normal momentum give
//   rho_w (1 + u_w.n) = sum_{c.n = 0} f + 2 sum_{c.n > 0} f,
// n the outward normal; with f = g + f^eq(rho0, u_b), whose own sums give
// rho0 (1 + u_b.n), that is
//   rho_w - rho0 = (sum_{c.n = 0} g + 2 sum_{c.n > 0} g - rho0 (u_w - u_b).n) / (1 + u_w.n).
// The caller then applies NSBC's assignment and correction at that vector.
template <class R>
__device__ inline M3<R> velocity_edge_moments(const R g[9], int nout_x, R rho0, R uwx, R duwx, R duwy) {
  R s = R(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cn = kCx[i] * nout_x;
    if (cn == 0) s += g[i];
    else if (cn > 0) s += R(2) * g[i];
  }
  const R un = R(nout_x) * uwx, dn = R(nout_x) * duwx;
  M3<R> m;
  m.v[0] = (s - rho0 * dn) * recip(R(1) + un);
  m.v[1] = duwx;
  m.v[2] = duwy;
  return m;
}


// Rebuild the unknown populations of one boundary node and correct it
// (eqs. nes_0..nes_4).  `unknown` has bit i set for every population whose
// pull source lies outside the domain; g holds the streamed (known) values.
// mc is the corrected macroscopic vector (drho, du_x, du_y).
template <class R>
__device__ inline void nsbc_assign_correct(R g[9], uint32_t unknown, const M3<R>& mc, R rho0, const Base<R>& b,
                                           int corr_mode) {
  R geq[9];
  equilibrium(rho0, b, mc.v[0], mc.v[1], mc.v[2], geq);
  // eqs. nes_0/nes_1: f_in = f_in^eq + (f_out - f_out^eq); a population whose
  // opposite is unknown too (corner "buried" pair) takes its equilibrium.
  // The base equilibrium cancels, so the same formula holds for deviations.
  R gn[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int o = kOpp[i];
    if (unknown & (1u << i)) {
      gn[i] = (unknown & (1u << o)) ? geq[i] : geq[i] + (g[o] - geq[o]);
    } else {
      gn[i] = g[i];
    }
  }
  // eq. nes_4: rescale (mass) and shift (momentum) so the node carries m_c:
  //   drho_err = sum f - rho_c = sum g - drho_c,
  //   dj = sum c f - rho_c u_c = sum c g - rho_c du_c - drho_c u_b.
  const R s = ((gn[0] + gn[1]) + (gn[2] + gn[3])) + ((gn[4] + gn[5]) + (gn[6] + gn[7])) + gn[8];
  const R jx = (gn[1] - gn[2]) + (gn[5] - gn[6]) + (gn[8] - gn[7]);
  const R jy = (gn[3] - gn[4]) + (gn[5] - gn[6]) + (gn[7] - gn[8]);
  const R rhoc = rho0 + mc.v[0];
  const R ddr = s - mc.v[0];
  const R k = corr_mode == 0 ? R(3) : R(1);
  const R djx = k * (jx - rhoc * mc.v[1] - mc.v[0] * b.ubx);
  const R djy = k * (jy - rhoc * mc.v[2] - mc.v[0] * b.uby);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    g[i] = gn[i] - wgt<R>(i) * (ddr + (R(kCx[i]) * djx + R(kCy[i]) * djy));
  }
}

}  // namespace lbm
