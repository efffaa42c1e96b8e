// Device numerics of the HGKS hot path (arXiv 2207.01173, Sec. 2):
// fifth-order WENO-Z pieces, Maxwellian moments, micro-slope solves and the
// time-integrated BGK flux at one Gauss point.  Everything is a template on
// the arithmetic type R (double for the FP64 path, float for the mixed path).
#pragma once
#include <hip/hip_runtime.h>

namespace hgks {

// ---------------------------------------------------------------------------
// WENO-Z (Borges et al.) on five cell averages v[0..4] centred at -2..2.
// ---------------------------------------------------------------------------

template <class R> struct WenoEps;
template <> struct WenoEps<double> { static constexpr double v = 1e-20; };
template <> struct WenoEps<float> { static constexpr float v = 1e-20f; };

// Reciprocal of a positive, normal number: the hardware estimate refined by
// two Newton steps (a few ulp at most in FP64; the FP32 path uses 1/x).
template <class R> __device__ __forceinline__ R pos_rcp(R x);
template <> __device__ __forceinline__ double pos_rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}
// FP32 (mixed path): the hardware reciprocal, within 1 ulp.
template <> __device__ __forceinline__ float pos_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// Reciprocal of a WENO-Z weight sum.  It scales every weight of a set by the
// same factor, so its relative error e moves a reconstructed value v2 + s sum
// w_k b_k only by e times the correction s sum w_k b_k, not by e times the
// value: FP64 takes one Newton step on the hardware estimate (the estimate is
// within 2^-24 of 1/x, the step within 2^-48), FP32 the hardware reciprocal.
template <class R> __device__ __forceinline__ R wz_rcp(R x);
template <> __device__ __forceinline__ double wz_rcp<double>(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(fma(-x, r, 1.0), r, r);
}
template <> __device__ __forceinline__ float wz_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// The three quadratic candidates through averages (v0,v1,v2), (v1,v2,v3),
// (v2,v3,v4), written about the centre cell (x in [-1/2, 1/2]) as
// p_k(x) = v2 - c_k/24 + b_k x + c_k x^2 / 2: c_k is the candidate's second
// difference, b_k its slope at the centre, both formed from the first
// differences d_j = v_{j+1} - v_j (c_0 = d_1 - d_0, c_1 = d_2 - d_1,
// c_2 = d_3 - d_2, b_0 = d_1 + c_0/2, b_1 = (d_1 + d_2)/2, b_2 = d_2 - c_2/2).
// be_k is the Jiang-Shu smoothness indicator 13/12 c_k^2 + b_k^2 with the
// WENO-Z epsilon already added.
template <class R> struct Candidates { R c[3], b[3], be[3]; };

template <class R>
__device__ __forceinline__ Candidates<R> candidates(const R v[5]) {
  Candidates<R> k;
  const R d0 = v[1] - v[0], d1 = v[2] - v[1], d2 = v[3] - v[2], d3 = v[4] - v[3];
  k.c[0] = d1 - d0;
  k.c[1] = d2 - d1;
  k.c[2] = d3 - d2;
  k.b[0] = d1 + R(0.5) * k.c[0];
  k.b[1] = R(0.5) * (d1 + d2);
  k.b[2] = d2 - R(0.5) * k.c[2];
  const R c13 = R(13.0 / 12.0), eps = WenoEps<R>::v;
#pragma unroll
  for (int i = 0; i < 3; ++i) k.be[i] = (c13 * k.c[i]) * k.c[i] + (k.b[i] * k.b[i] + eps);
  return k;
}

// Nonlinear weights alpha_k = d_k (1 + tau5 / b_k), b_k = beta_k + eps,
// tau5 = |beta_0 - beta_2|, normalised.  wz_factors gives e_k with alpha_k
// proportional to d_k e_k; they depend on the stencil only, so every set of
// linear weights (both Gauss points, value and slope weights) shares them.
// Multiplying every alpha by b0 b1 b2 leaves the normalised weights unchanged
// and needs a single reciprocal per set (FP64: the products stay far from
// underflow for b >= eps).  The FP32 path keeps one reciprocal per b_k,
// whose products could underflow.
template <class R>
__device__ __forceinline__ void wz_factors(const R be[3], R e[3]) {
  const R t5 = fabs(be[0] - be[2]);
  if (sizeof(R) == 8) {
    e[0] = (be[0] + t5) * (be[1] * be[2]);
    e[1] = (be[1] + t5) * (be[0] * be[2]);
    e[2] = (be[2] + t5) * (be[0] * be[1]);
  } else {
    e[0] = R(1) + t5 * pos_rcp(be[0]);
    e[1] = R(1) + t5 * pos_rcp(be[1]);
    e[2] = R(1) + t5 * pos_rcp(be[2]);
  }
}

// Unnormalised weights a_k = d_k e_k for the linear weights (d0, d1, d2);
// returns 1 / sum a.  A weighted candidate sum sum_k w_k x_k is formed as
// (sum_k a_k x_k) / sum a: one multiply by the reciprocal instead of three.
template <class R>
__device__ __forceinline__ R wz_alpha(const R e[3], R d0, R d1, R d2, R a[3]) {
  a[0] = d0 * e[0];
  a[1] = d1 * e[1];
  a[2] = d2 * e[2];
  return wz_rcp(a[0] + a[1] + a[2]);
}

// sum_k a_k x_k
template <class R> __device__ __forceinline__ R wz_dot(const R a[3], R x0, R x1, R x2) {
  return a[0] * x0 + a[1] * x1 + a[2] * x2;
}

// Gauss points of the unit cell: s = -sqrt(3)/6 (g = 0) and +sqrt(3)/6 (g = 1).
struct GaussConst {
  static constexpr double r3 = 1.7320508075688772935274463;
  static constexpr double s = r3 / 6.0;
  // value linear weights at s = +sqrt3/6; reversed at -sqrt3/6
  static constexpr double dv0 = 7.0 / 36.0 - r3 / 1080.0, dv1 = 11.0 / 18.0, dv2 = 7.0 / 36.0 + r3 / 1080.0;
  // derivative linear weights at s = +sqrt3/6 (reproduce the quartic's slope)
  static constexpr double dd0 = 11.0 / 36.0 - 5.0 * r3 / 36.0, dd1 = 7.0 / 18.0, dd2 = 11.0 / 36.0 + 5.0 * r3 / 36.0;
};

// Position and linear weights of one Gauss point, chosen per lane at run time
// (g = 0: s = -sqrt3/6, g = 1: s = +sqrt3/6; the weights mirror with s).
template <class R> struct GaussPoint {
  R s, dv0, dv1, dv2;
  __device__ __forceinline__ explicit GaussPoint(int g) {
    const bool p = g != 0;
    s = p ? R(GaussConst::s) : R(-GaussConst::s);
    dv0 = p ? R(GaussConst::dv0) : R(GaussConst::dv2);
    dv1 = R(GaussConst::dv1);
    dv2 = p ? R(GaussConst::dv2) : R(GaussConst::dv0);
  }
};

// Both Gauss points of one stencil (index 0: s = -sqrt3/6, 1: s = +sqrt3/6)
// from one set of candidates and WENO-Z factors.  At +s the value is
// v2 + s sum w_k b_k with the value weights (dv0, dv1, dv2) and the slope
// sum w_k (b_k + s c_k) with the slope weights (dd0, dd1, dd2); at -s the
// weights are reversed and s changes sign.  With y_k = e_k b_k and
// z_k = e_k c_k every such sum is (sum_k d_k y_k [+- s sum_k d_k z_k]) /
// sum_k d_k e_k, the factors s d_k being constants.
template <class R>
__device__ __forceinline__ void gauss_value2(const R v[5], R val[2]) {
  using G = GaussConst;
  const Candidates<R> k = candidates(v);
  R e[3];
  wz_factors(k.be, e);
  const R y0 = e[0] * k.b[0], y1 = e[1] * k.b[1], y2 = e[2] * k.b[2];
  const R nm = R(G::s * G::dv2) * y0 + R(G::s * G::dv1) * y1 + R(G::s * G::dv0) * y2;
  const R dm = R(G::dv2) * e[0] + R(G::dv1) * e[1] + R(G::dv0) * e[2];
  const R np = R(G::s * G::dv0) * y0 + R(G::s * G::dv1) * y1 + R(G::s * G::dv2) * y2;
  const R dp = R(G::dv0) * e[0] + R(G::dv1) * e[1] + R(G::dv2) * e[2];
  val[0] = v[2] - nm * wz_rcp(dm);
  val[1] = v[2] + np * wz_rcp(dp);
}

template <class R>
__device__ __forceinline__ void gauss_value_slope2(const R v[5], R val[2], R der[2]) {
  using G = GaussConst;
  const Candidates<R> k = candidates(v);
  R e[3];
  wz_factors(k.be, e);
  const R y0 = e[0] * k.b[0], y1 = e[1] * k.b[1], y2 = e[2] * k.b[2];
  const R z0 = e[0] * k.c[0], z1 = e[1] * k.c[1], z2 = e[2] * k.c[2];
  const R nm = R(G::s * G::dv2) * y0 + R(G::s * G::dv1) * y1 + R(G::s * G::dv0) * y2;
  const R dm = R(G::dv2) * e[0] + R(G::dv1) * e[1] + R(G::dv0) * e[2];
  const R np = R(G::s * G::dv0) * y0 + R(G::s * G::dv1) * y1 + R(G::s * G::dv2) * y2;
  const R dp = R(G::dv0) * e[0] + R(G::dv1) * e[1] + R(G::dv2) * e[2];
  val[0] = v[2] - nm * wz_rcp(dm);
  val[1] = v[2] + np * wz_rcp(dp);
  const R sm = R(G::dd2) * y0 + R(G::dd1) * y1 + R(G::dd0) * y2 + R(-G::s * G::dd2) * z0 +
               R(-G::s * G::dd1) * z1 + R(-G::s * G::dd0) * z2;
  const R em = R(G::dd2) * e[0] + R(G::dd1) * e[1] + R(G::dd0) * e[2];
  const R sp = R(G::dd0) * y0 + R(G::dd1) * y1 + R(G::dd2) * y2 + R(G::s * G::dd0) * z0 +
               R(G::s * G::dd1) * z1 + R(G::s * G::dd2) * z2;
  const R ep = R(G::dd0) * e[0] + R(G::dd1) * e[1] + R(G::dd2) * e[2];
  der[0] = sm * wz_rcp(em);
  der[1] = sp * wz_rcp(ep);
}

template <class R>
__device__ __forceinline__ void gauss_linear2(const R v[5], R val[2]) {
  const R b0 = R(1.5) * v[2] - R(2) * v[1] + R(0.5) * v[0];
  const R b1 = R(0.5) * (v[3] - v[1]);
  const R b2 = R(2) * v[3] - R(1.5) * v[2] - R(0.5) * v[4];
  const R s = R(GaussConst::s);
  const R d0 = R(GaussConst::dv0), d1 = R(GaussConst::dv1), d2 = R(GaussConst::dv2);
  val[0] = v[2] - s * (d2 * b0 + d1 * b1 + d0 * b2);
  val[1] = v[2] + s * (d0 * b0 + d1 * b1 + d2 * b2);
}

// Linear (fifth-order) value at a Gauss point: the quartic through the averages.
template <class R>
__device__ __forceinline__ R gauss_linear(const R v[5], const GaussPoint<R>& gp) {
  const R b0 = R(1.5) * v[2] - R(2) * v[1] + R(0.5) * v[0];
  const R b1 = R(0.5) * (v[3] - v[1]);
  const R b2 = R(2) * v[3] - R(1.5) * v[2] - R(0.5) * v[4];
  return v[2] + gp.s * (gp.dv0 * b0 + gp.dv1 * b1 + gp.dv2 * b2);
}

// Value and slope at the right face (s = 1/2) of the centre cell: candidate
// value v2 + b_k/2 + c_k/12, slope b_k + c_k/2.
template <class R>
__device__ __forceinline__ void face_value_slope(const R v[5], R& val, R& der) {
  const Candidates<R> k = candidates(v);
  R e[3], a[3];
  wz_factors(k.be, e);
  const R inv = wz_alpha(e, R(0.1), R(0.6), R(0.3), a);
  const R twelfth = R(1.0 / 12.0);
  val = v[2] + inv * wz_dot(a, R(0.5) * k.b[0] + twelfth * k.c[0], R(0.5) * k.b[1] + twelfth * k.c[1],
                            R(0.5) * k.b[2] + twelfth * k.c[2]);
  der = inv * wz_dot(a, k.b[0] + R(0.5) * k.c[0], k.b[1] + R(0.5) * k.c[1], k.b[2] + R(0.5) * k.c[2]);
}

// Normal sweep at face i+1/2 from c[0..5] = Q_{i-2..i+3}: left/right values and
// slopes, and the equilibrium slope (Q_{i-1} - 15 Q_i + 15 Q_{i+1} - Q_{i+2})/12.
template <class R>
__device__ __forceinline__ void normal_sweep(const R c[6], R& ql, R& qr, R& dl, R& dr, R& d0) {
  R vl[5] = {c[0], c[1], c[2], c[3], c[4]};
  face_value_slope(vl, ql, dl);
  R vr[5] = {c[5], c[4], c[3], c[2], c[1]};
  R m;
  face_value_slope(vr, qr, m);
  dr = -m;
  d0 = (c[1] - c[4] + R(15) * (c[3] - c[2])) * R(1.0 / 12.0);
}

// ---------------------------------------------------------------------------
// Maxwellian moments (normalised by density)
// ---------------------------------------------------------------------------

template <class R> struct State { R rho, U, V, W, lam; };

template <class R>
__device__ __forceinline__ State<R> primitive(const R q[5], R gm1, R& ir, R& ihl) {
  State<R> s;
  s.rho = q[0];
  ir = pos_rcp(q[0]);
  s.U = q[1] * ir;
  s.V = q[2] * ir;
  s.W = q[3] * ir;
  const R p = gm1 * (q[4] - R(0.5) * (q[1] * s.U + q[2] * s.V + q[3] * s.W));
  s.lam = R(0.5) * q[0] * pos_rcp(p);
  ihl = p * ir;  // 1/(2 lambda) = p/rho
  return s;
}

// <c^n>, n = 0..N-1, of a Gaussian with the given mean and 1/(2 lambda) = ihl,
// from the first two: <c^(n+2)> = mean <c^(n+1)> + (n+1) ihl <c^n>.
template <class R, int N>
__device__ __forceinline__ void chain(R mean, R ihl, R m0, R m1, R o[N]) {
  o[0] = m0;
  o[1] = m1;
#pragma unroll
  for (int n = 0; n + 2 < N; ++n) o[n + 2] = mean * o[n + 1] + R(n + 1) * ihl * o[n];
}

// Zeroth and first half-space u-moments, u > 0 (SIDE = +1) or u < 0 (SIDE = -1).
template <class R, int SIDE>
__device__ __forceinline__ void half_moments01(const State<R>& s, R& m0, R& m1) {
  R sl = sqrt(s.lam);
  R e = exp(-s.lam * s.U * s.U) * R(0.28209479177387814347) * pos_rcp(sl);  // e^{-l U^2} / (2 sqrt(pi l))
  m0 = R(0.5) * erfc(-R(SIDE) * sl * s.U);
  m1 = s.U * m0 + R(SIDE) * e;
}

// Moments over (v, w, xi) of one Maxwellian, r = v^2 + w^2 + xi^2:
// E[v^b w^c r^e] for the monomials the flux needs.  The u-direction is kept
// apart (full or half space), so every moment of a product factorises into a
// u-moment times one of these.
template <class R> struct VW {
  R v, w, r, vv, vw, ww, vr, wr, rr, vvv, vvw, vww, www, vvr, vwr, wwr, vrr, wrr;
};

template <class R>
__device__ __forceinline__ void vw_moments(const State<R>& s, R ihl, R K, VW<R>& e) {
  R V[6], W[6];
  chain<R, 6>(s.V, ihl, R(1), s.V, V);
  chain<R, 6>(s.W, ihl, R(1), s.W, W);
  const R x1 = K * ihl;                          // <xi^2>
  const R x2 = K * (K + R(2)) * ihl * ihl;       // <xi^4>
  e.v = V[1];
  e.w = W[1];
  e.r = V[2] + W[2] + x1;
  e.vv = V[2];
  e.vw = V[1] * W[1];
  e.ww = W[2];
  e.vr = V[3] + V[1] * (W[2] + x1);
  e.wr = W[3] + W[1] * (V[2] + x1);
  e.rr = V[4] + W[4] + x2 + R(2) * (V[2] * W[2] + (V[2] + W[2]) * x1);
  e.vvv = V[3];
  e.vvw = V[2] * W[1];
  e.vww = V[1] * W[2];
  e.www = W[3];
  e.vvr = V[4] + V[2] * (W[2] + x1);
  e.vwr = V[3] * W[1] + V[1] * W[3] + V[1] * W[1] * x1;
  e.wwr = W[4] + W[2] * (V[2] + x1);
  e.vrr = V[5] + V[1] * (W[4] + x2) + R(2) * (V[3] * W[2] + (V[3] + V[1] * W[2]) * x1);
  e.wrr = W[5] + W[1] * (V[4] + x2) + R(2) * (V[2] * W[3] + (W[3] + V[2] * W[1]) * x1);
}

// (v, w, xi)-moments of a polynomial g(v, w, xi^2): E[g], E[v g], E[w g], E[r g].
template <class R> struct Quad { R e0, ev, ew, er; };

// For a moment coefficient vector a, a . psi = p + a1 u + h u^2 with
// p = a0 + a2 v + a3 w + h r and h = a4 / 2.  Quad of p times 1, v or w:
template <class R>
__device__ __forceinline__ Quad<R> quad_p(const R a[5], const VW<R>& e) {
  const R h = R(0.5) * a[4];
  return {a[0] + a[2] * e.v + a[3] * e.w + h * e.r, a[0] * e.v + a[2] * e.vv + a[3] * e.vw + h * e.vr,
          a[0] * e.w + a[2] * e.vw + a[3] * e.ww + h * e.wr, a[0] * e.r + a[2] * e.vr + a[3] * e.wr + h * e.rr};
}
template <class R>
__device__ __forceinline__ Quad<R> quad_vp(const R a[5], const VW<R>& e) {
  const R h = R(0.5) * a[4];
  return {a[0] * e.v + a[2] * e.vv + a[3] * e.vw + h * e.vr, a[0] * e.vv + a[2] * e.vvv + a[3] * e.vvw + h * e.vvr,
          a[0] * e.vw + a[2] * e.vvw + a[3] * e.vww + h * e.vwr, a[0] * e.vr + a[2] * e.vvr + a[3] * e.vwr + h * e.vrr};
}
template <class R>
__device__ __forceinline__ Quad<R> quad_wp(const R a[5], const VW<R>& e) {
  const R h = R(0.5) * a[4];
  return {a[0] * e.w + a[2] * e.vw + a[3] * e.ww + h * e.wr, a[0] * e.vw + a[2] * e.vvw + a[3] * e.vww + h * e.vwr,
          a[0] * e.ww + a[2] * e.vww + a[3] * e.www + h * e.wwr, a[0] * e.wr + a[2] * e.vwr + a[3] * e.wwr + h * e.wrr};
}
// Quad of c (1, v, w, r-weighted): c times the unit polynomial.
template <class R>
__device__ __forceinline__ Quad<R> quad_c(R c, const VW<R>& e) {
  return {c, c * e.v, c * e.w, c * e.r};
}
// Quad of c0 + c1 v + c2 w (tangential-linear polynomial).
template <class R>
__device__ __forceinline__ Quad<R> quad_lin(R c0, R c1, R c2, const VW<R>& e) {
  return {c0 + c1 * e.v + c2 * e.w, c0 * e.v + c1 * e.vv + c2 * e.vw, c0 * e.w + c1 * e.vw + c2 * e.ww,
          c0 * e.r + c1 * e.vr + c2 * e.wr};
}
template <class R>
__device__ __forceinline__ Quad<R> qadd(const Quad<R>& a, const Quad<R>& b) {
  return {a.e0 + b.e0, a.ev + b.ev, a.ew + b.ew, a.er + b.er};
}

// <u^X G psi> for G = sum_{i < NS} u^i g_i, given the quads of the g_i and a
// u-moment table Mu (full or half space), psi = (1, u, v, w, (u^2 + r)/2).
template <class R, int X, int NS>
__device__ __forceinline__ void assemble(const Quad<R> q[NS], const R Mu[7], R o[5]) {
  R a0 = R(0), a1 = R(0), a2 = R(0), a3 = R(0), a4 = R(0);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    a0 += Mu[X + i] * q[i].e0;
    a1 += Mu[X + i + 1] * q[i].e0;
    a2 += Mu[X + i] * q[i].ev;
    a3 += Mu[X + i] * q[i].ew;
    a4 += Mu[X + i + 2] * q[i].e0 + Mu[X + i] * q[i].er;
  }
  o[0] = a0;
  o[1] = a1;
  o[2] = a2;
  o[3] = a3;
  o[4] = R(0.5) * a4;
}

// u-series of a . psi: (p, a1, h).
template <class R>
__device__ __forceinline__ void series_apsi(const R a[5], const VW<R>& e, Quad<R> q[3]) {
  q[0] = quad_p(a, e);
  q[1] = quad_c(a[1], e);
  q[2] = quad_c(R(0.5) * a[4], e);
}

// u-series of Pi = u (an . psi) + v (at1 . psi) + w (at2 . psi):
// Pi_0 = v p_t1 + w p_t2, Pi_1 = p_n + at1_1 v + at2_1 w, Pi_2 = an_1 + h_t1 v + h_t2 w, Pi_3 = h_n.
template <class R>
__device__ __forceinline__ void series_pi(const R a[3][5], const VW<R>& e, Quad<R> q[4]) {
  q[0] = qadd(quad_vp(a[1], e), quad_wp(a[2], e));
  q[1] = qadd(quad_p(a[0], e), quad_lin(R(0), a[1][1], a[2][1], e));
  q[2] = quad_lin(a[0][1], R(0.5) * a[1][4], R(0.5) * a[2][4], e);
  q[3] = quad_c(R(0.5) * a[0][4], e);
}

// Closed-form solution of <(a . psi) psi> = b for a Maxwellian state.
template <class R>
__device__ __forceinline__ void slope_solve(const State<R>& s, R ihl, R K3, R iK3, const R b[5], R a[5]) {
  R q2 = s.U * s.U + s.V * s.V + s.W * s.W + K3 * ihl;
  R r2 = b[1] - s.U * b[0];
  R r3 = b[2] - s.V * b[0];
  R r4 = b[3] - s.W * b[0];
  R r5 = R(2) * b[4] - q2 * b[0];
  R tl = R(2) * s.lam;
  a[4] = tl * tl * iK3 * (r5 - R(2) * (s.U * r2 + s.V * r3 + s.W * r4));
  a[3] = tl * r4 - s.W * a[4];
  a[2] = tl * r3 - s.V * a[4];
  a[1] = tl * r2 - s.U * a[4];
  a[0] = b[0] - s.U * a[1] - s.V * a[2] - s.W * a[3] - R(0.5) * a[4] * q2;
}

// ---------------------------------------------------------------------------
// Gauss-point flux
// ---------------------------------------------------------------------------

template <class R> struct GasParams {
  R gm1;       // gamma - 1
  R K;         // internal degrees of freedom
  R K3, iK3;   // K + 3 and its reciprocal
  R mu_ref, iT_ref, mu_exp;
  R pr_fix;    // 1/Pr - 1
};

// Time coefficients of the two face quantities the update uses, the flux
// F^n = (4 F(dt/2) - F(dt)) / dt and its derivative 4 (F(dt) - 2 F(dt/2)) / dt^2,
// where F(delta) = sum_i C_i(delta) X_i with the six integrals over [0, delta]
// of the BGK solution's time factors,
//   C1 = delta - tau o, C2 = 2 tau^2 o - tau delta (1 + eta),
//   C3 = delta^2/2 - tau delta + tau^2 o, C4 = tau o,
//   C5 = tau delta eta - 2 tau^2 o, C6 = -tau^2 o  (eta = e^{-delta/tau}, o = 1 - eta).
// Both windows share h = e^{-dt/(2 tau)} (e^{-dt/tau} = h^2), and the window
// combinations N_i = 4 C_i(dt/2) - C_i(dt) and D_i = C_i(dt) - 2 C_i(dt/2)
// reduce in closed form to products of o = 1 - h and g = 3 - h with no
// difference of O(dt) terms left (combining the two windows' fluxes instead
// would lose the rounding of dt |F| in a difference of order dt^2 |dF/dt|).
// Cn = N / dt, Cd = 4 D / dt^2.  tau = 0 (h = 0) gives the Euler limits
// Cn = (1, 0, 0, 0, 0, 0) and Cd = (0, 0, 1, 0, 0, 0) with no special case.
template <class R>
__device__ __forceinline__ void time_integrals(R tau, R itau, R dt, R Cn[6], R Cd[6]) {
  const R h = tau > R(0) ? exp(-(R(0.5) * dt) * itau) : R(0);
  const R o = R(1) - h, t2 = tau * tau, og = o * (R(3) - h), o2 = o * o;
  const R idt = pos_rcp(dt), i4dt2 = R(4) * idt * idt;
  Cn[0] = (dt - tau * og) * idt;
  Cn[1] = (R(2) * t2 * og - tau * dt * (R(1) + R(2) * h - h * h)) * idt;
  Cn[2] = (t2 * og - tau * dt) * idt;
  Cn[3] = tau * og * idt;
  Cn[4] = (tau * dt * h * (R(2) - h) - R(2) * t2 * og) * idt;
  Cn[5] = -t2 * og * idt;
  Cd[0] = tau * o2 * i4dt2;
  Cd[1] = tau * o * (dt * h - R(2) * tau * o) * i4dt2;
  Cd[2] = (R(0.25) * dt * dt - t2 * o2) * i4dt2;
  Cd[3] = -tau * o2 * i4dt2;
  Cd[4] = tau * o * (R(2) * tau * o - dt * h) * i4dt2;
  Cd[5] = t2 * o2 * i4dt2;
}

// Energy in the frame of U0 carried by a moment vector of psi:
// v_E - U0 . v_m + |U0|^2/2 v_rho.
template <class R>
__device__ __forceinline__ R thermal(const R v[5], R U, R V, R W, R hu2) {
  return v[4] - (U * v[1] + V * v[2] + W * v[3]) + hu2 * v[0];
}

// thermal() of a u^0 moment <G psi> of a u-series G = sum_i u^i g_i (quads of
// the g_i, u-table Mu), without forming the moment vector:
//   sum_i [ e0_i Tw_i + Mu[i] (er_i / 2 - V ev_i - W ew_i) ],
// Tw_i = Mu[i+2]/2 - U Mu[i+1] + hu2 Mu[i] the weights (thermal_weights) that
// the energy, momentum and density rows of the moment give u^i in the frame
// of (U, V, W).
template <class R>
__device__ __forceinline__ void thermal_weights(const R Mu[7], R U, R hu2, R Tw[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) Tw[i] = R(0.5) * Mu[i + 2] - U * Mu[i + 1] + hu2 * Mu[i];
}
template <class R, int NS>
__device__ __forceinline__ R thermal_series(const Quad<R> q[NS], const R Mu[7], const R Tw[4], R V, R W) {
  R t = R(0);
#pragma unroll
  for (int i = 0; i < NS; ++i) t += q[i].e0 * Tw[i] + Mu[i] * (R(0.5) * q[i].er - V * q[i].ev - W * q[i].ew);
  return t;
}

// Running state of one Gauss-point flux evaluation, filled in phases so that
// the caller can reconstruct the left inputs, consume them, then the right
// ones, keeping few values live at a time.
template <class R> struct FluxAcc {
  State<R> s0;          // interface equilibrium
  R ihl0, hu2;          // 1/(2 lambda0), |U0|^2 / 2
  R Cn[6], Cd[6];       // time coefficients of F^n and of its time derivative
  R lm0, lm1, rm0, rm1; // half-space zeroth/first u-moments of the left/right states
  R Fn[5], Fd[5];       // F^n and dF^n/dt at the Gauss point (partial sums)
  R wn, wd;             // thermal part of the conserved-variable integrals (Prandtl correction)
  R dq0t[2][5];         // tangential slopes of Q0 (exact derivative of the compatibility map)
};

// Phase 1: equilibrium at the interface from the compatibility condition,
// Q0 = rho_l <psi>_{u>0, l} + rho_r <psi>_{u<0, r}, collision time and the
// time integrals.
template <class R>
__device__ __forceinline__ void flux_begin(const R ql[5], const R qr[5], const GasParams<R>& g, R dt, FluxAcc<R>& A) {
  R q0[5];
  {
    R irl, irr, il, ir;
    const State<R> sl = primitive(ql, g.gm1, irl, il), sr = primitive(qr, g.gm1, irr, ir);
    half_moments01<R, 1>(sl, A.lm0, A.lm1);
    half_moments01<R, -1>(sr, A.rm0, A.rm1);
    // <psi> with half-space u: (m0, m1, V m0, W m0, (m2 + m0 (V^2 + W^2 + (K + 2) ihl)) / 2)
    const R l2 = sl.U * A.lm1 + il * A.lm0, r2 = sr.U * A.rm1 + ir * A.rm0;
    const R lt = sl.V * sl.V + sl.W * sl.W + (g.K + R(2)) * il;
    const R rt = sr.V * sr.V + sr.W * sr.W + (g.K + R(2)) * ir;
    q0[0] = sl.rho * A.lm0 + sr.rho * A.rm0;
    q0[1] = sl.rho * A.lm1 + sr.rho * A.rm1;
    q0[2] = sl.rho * sl.V * A.lm0 + sr.rho * sr.V * A.rm0;
    q0[3] = sl.rho * sl.W * A.lm0 + sr.rho * sr.W * A.rm0;
    q0[4] = R(0.5) * (sl.rho * (l2 + A.lm0 * lt) + sr.rho * (r2 + A.rm0 * rt));
  }
  R ir0;
  A.s0 = primitive(q0, g.gm1, ir0, A.ihl0);
  // collision time tau = mu(T0) / p0, T0 = p0/rho0 = 1/(2 lambda0)
  const R p0 = A.s0.rho * A.ihl0;
  R mu = g.mu_ref;
  if (g.mu_exp != R(0)) mu = g.mu_ref * pow(A.ihl0 * g.iT_ref, g.mu_exp);
  const R tau = mu * pos_rcp(p0);
  const R itau = tau > R(0) ? pos_rcp(tau) : R(0);
  time_integrals(tau, itau, dt, A.Cn, A.Cd);
  A.hu2 = R(0.5) * (A.s0.U * A.s0.U + A.s0.V * A.s0.V + A.s0.W * A.s0.W);
#pragma unroll
  for (int k = 0; k < 5; ++k) { A.Fn[k] = R(0); A.Fd[k] = R(0); A.dq0t[0][k] = R(0); A.dq0t[1][k] = R(0); }
  A.wn = R(0);
  A.wd = R(0);
}

// Phase 2/3: contributions of one non-equilibrium side (g_l with u > 0 when
// LEFT, g_r with u < 0 otherwise): flux moments weighted by C4, C5, C6, the
// thermal part of the same terms' conserved-variable moments, and the side's
// part of the tangential slopes of Q0.
template <class R, bool LEFT>
__device__ __forceinline__ void flux_side(const R q[5], const R dq[3][5], const GasParams<R>& g, FluxAcc<R>& Acc) {
  R ir, ihl;
  State<R> s = primitive(q, g.gm1, ir, ihl);
  VW<R> e;
  vw_moments(s, ihl, g.K, e);
  R a[3][5];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    R b[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = dq[d][k] * ir;
    slope_solve(s, ihl, g.K3, g.iK3, b, a[d]);
  }
  Quad<R> pi[4];
  series_pi(a, e, pi);
  R A[5];
  {
    R Mf[7], T[5];
    chain<R, 7>(s.U, ihl, R(1), s.U, Mf);
    assemble<R, 0, 4>(pi, Mf, T);
#pragma unroll
    for (int k = 0; k < 5; ++k) T[k] = -T[k];
    slope_solve(s, ihl, g.K3, g.iK3, T, A);
  }
  R Mh[7];
  if (LEFT) chain<R, 7>(s.U, ihl, Acc.lm0, Acc.lm1, Mh);
  else chain<R, 7>(s.U, ihl, Acc.rm0, Acc.rm1, Mh);
  const Quad<R> unit[1] = {quad_c(R(1), e)};
  Quad<R> qa[3];
  series_apsi(A, e, qa);
  const R rho = s.rho;
  const R U0 = Acc.s0.U, V0 = Acc.s0.V, W0 = Acc.s0.W;
  {
    R X1[5], X2[5], X3[5];
    assemble<R, 1, 1>(unit, Mh, X1);
    assemble<R, 1, 4>(pi, Mh, X2);
    assemble<R, 1, 3>(qa, Mh, X3);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      Acc.Fn[k] += rho * (Acc.Cn[3] * X1[k] + Acc.Cn[4] * X2[k] + Acc.Cn[5] * X3[k]);
      Acc.Fd[k] += rho * (Acc.Cd[3] * X1[k] + Acc.Cd[4] * X2[k] + Acc.Cd[5] * X3[k]);
    }
  }
  {
    R Tw[4];
    thermal_weights(Mh, U0, Acc.hu2, Tw);
    const R y1 = thermal_series<R, 1>(unit, Mh, Tw, V0, W0);
    const R y2 = thermal_series<R, 4>(pi, Mh, Tw, V0, W0);
    const R y3 = thermal_series<R, 3>(qa, Mh, Tw, V0, W0);
    Acc.wn += rho * (Acc.Cn[3] * y1 + Acc.Cn[4] * y2 + Acc.Cn[5] * y3);
    Acc.wd += rho * (Acc.Cd[3] * y1 + Acc.Cd[4] * y2 + Acc.Cd[5] * y3);
  }
#pragma unroll
  for (int d = 1; d < 3; ++d) {
    Quad<R> qt[3];
    series_apsi(a[d], e, qt);
    R t[5];
    assemble<R, 0, 3>(qt, Mh, t);
#pragma unroll
    for (int k = 0; k < 5; ++k) Acc.dq0t[d - 1][k] += rho * t[k];
  }
}

// Phase 4: equilibrium part with the normal slope of Q0 (dq0n) and the
// accumulated tangential ones, then the Prandtl correction of the energy
// flux, q = thermal(F) - U0_n thermal(W).
template <class R>
__device__ __forceinline__ void flux_finish(const R dq0n[5], const GasParams<R>& g, FluxAcc<R>& Acc, R Fn[5],
                                            R Fd[5]) {
  const State<R>& s0 = Acc.s0;
  const R ihl0 = Acc.ihl0;
  VW<R> e;
  vw_moments(s0, ihl0, g.K, e);
  R Mf[7];
  chain<R, 7>(s0.U, ihl0, R(1), s0.U, Mf);
  R a[3][5];
  const R ir = pos_rcp(s0.rho);
  {
    R b[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = dq0n[k] * ir;
    slope_solve(s0, ihl0, g.K3, g.iK3, b, a[0]);
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = Acc.dq0t[0][k] * ir;
    slope_solve(s0, ihl0, g.K3, g.iK3, b, a[1]);
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = Acc.dq0t[1][k] * ir;
    slope_solve(s0, ihl0, g.K3, g.iK3, b, a[2]);
  }
  Quad<R> pi[4];
  series_pi(a, e, pi);
  R T[5];  // sum_d <s_d (a_d . psi) psi>_0
  assemble<R, 0, 4>(pi, Mf, T);
  R A[5];
  {
    R b[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = -T[k];
    slope_solve(s0, ihl0, g.K3, g.iK3, b, A);
  }
  const Quad<R> unit[1] = {quad_c(R(1), e)};
  Quad<R> qa[3];
  series_apsi(A, e, qa);
  const R rho = s0.rho;
  R X1[5], X2[5], X3[5];
  assemble<R, 1, 1>(unit, Mf, X1);
  assemble<R, 1, 4>(pi, Mf, X2);
  assemble<R, 1, 3>(qa, Mf, X3);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    Fn[k] = Acc.Fn[k] + rho * (Acc.Cn[0] * X1[k] + Acc.Cn[1] * X2[k] + Acc.Cn[2] * X3[k]);
    Fd[k] = Acc.Fd[k] + rho * (Acc.Cd[0] * X1[k] + Acc.Cd[1] * X2[k] + Acc.Cd[2] * X3[k]);
  }
  R Tw[4];
  thermal_weights(Mf, s0.U, Acc.hu2, Tw);
  const R y1 = thermal_series<R, 1>(unit, Mf, Tw, s0.V, s0.W);
  const R y2 = thermal(T, s0.U, s0.V, s0.W, Acc.hu2);
  const R y3 = thermal_series<R, 3>(qa, Mf, Tw, s0.V, s0.W);
  const R wn = Acc.wn + rho * (Acc.Cn[0] * y1 + Acc.Cn[1] * y2 + Acc.Cn[2] * y3);
  const R wd = Acc.wd + rho * (Acc.Cd[0] * y1 + Acc.Cd[1] * y2 + Acc.Cd[2] * y3);
  // the heat flux is linear in the window, so the correction applies to F^n
  // and to its derivative alike
  const R qhn = thermal(Fn, s0.U, s0.V, s0.W, Acc.hu2) - s0.U * wn;
  const R qhd = thermal(Fd, s0.U, s0.V, s0.W, Acc.hu2) - s0.U * wd;
  Fn[4] += g.pr_fix * qhn;
  Fd[4] += g.pr_fix * qhd;
}

// F^n and dF^n/dt at one Gauss point, local frame (n, t1, t2).  Slopes in
// physical units.
template <class R>
__device__ __forceinline__ void gp_flux(const R ql[5], const R qr[5], const R dql[3][5], const R dqr[3][5],
                                        const R dq0n[5], const GasParams<R>& g, R dt, R Fn[5], R Fd[5]) {
  FluxAcc<R> A;
  flux_begin(ql, qr, g, dt, A);
  flux_side<R, true>(ql, dql, g, A);
  flux_side<R, false>(qr, dqr, g, A);
  flux_finish(dq0n, g, A, Fn, Fd);
}

}  // namespace hgks
