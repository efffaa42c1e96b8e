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

// Jiang-Shu smoothness indicators of the three quadratic candidates.
template <class R>
__device__ __forceinline__ void js_smoothness(const R v[5], R b[3]) {
  const R c13 = R(13.0 / 12.0);
  R d0 = v[0] - R(2) * v[1] + v[2], e0 = v[0] - R(4) * v[1] + R(3) * v[2];
  R d1 = v[1] - R(2) * v[2] + v[3], e1 = v[1] - v[3];
  R d2 = v[2] - R(2) * v[3] + v[4], e2 = R(3) * v[2] - R(4) * v[3] + v[4];
  b[0] = c13 * d0 * d0 + R(0.25) * e0 * e0;
  b[1] = c13 * d1 * d1 + R(0.25) * e1 * e1;
  b[2] = c13 * d2 * d2 + R(0.25) * e2 * e2;
}

// Nonlinear weights alpha_k = d_k (1 + tau5 / (beta_k + eps)), normalised.
template <class R>
__device__ __forceinline__ void wz_weights(const R b[3], R d0, R d1, R d2, R w[3]) {
  const R eps = WenoEps<R>::v;
  R t5 = fabs(b[0] - b[2]);
  R a0 = d0 * (R(1) + t5 / (b[0] + eps));
  R a1 = d1 * (R(1) + t5 / (b[1] + eps));
  R a2 = d2 * (R(1) + t5 / (b[2] + eps));
  R inv = R(1) / (a0 + a1 + a2);
  w[0] = a0 * inv;
  w[1] = a1 * inv;
  w[2] = a2 * inv;
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
  R s, dv0, dv1, dv2, dd0, dd1, dd2;
  __device__ __forceinline__ explicit GaussPoint(int g) {
    const bool p = g != 0;
    s = p ? R(GaussConst::s) : R(-GaussConst::s);
    dv0 = p ? R(GaussConst::dv0) : R(GaussConst::dv2);
    dv1 = R(GaussConst::dv1);
    dv2 = p ? R(GaussConst::dv2) : R(GaussConst::dv0);
    dd0 = p ? R(GaussConst::dd0) : R(GaussConst::dd2);
    dd1 = R(GaussConst::dd1);
    dd2 = p ? R(GaussConst::dd2) : R(GaussConst::dd0);
  }
};

// Candidate values and slopes (per unit index) at a Gauss point.
template <class R>
__device__ __forceinline__ void gauss_candidates(const R v[5], R s, R p[3], R dp[3]) {
  // quadratic through three averages: value a + b s at the Gauss point (the
  // s^2 = 1/12 term cancels the 1/12 offset of the averages), slope b + 2 c s
  R c0 = v[0] - R(2) * v[1] + v[2];
  R b0 = R(1.5) * v[2] - R(2) * v[1] + R(0.5) * v[0];
  R c1 = v[1] - R(2) * v[2] + v[3];
  R b1 = R(0.5) * (v[3] - v[1]);
  R c2 = v[2] - R(2) * v[3] + v[4];
  R b2 = R(2) * v[3] - R(1.5) * v[2] - R(0.5) * v[4];
  p[0] = v[2] + b0 * s;
  p[1] = v[2] + b1 * s;
  p[2] = v[2] + b2 * s;
  dp[0] = b0 + c0 * s;
  dp[1] = b1 + c1 * s;
  dp[2] = b2 + c2 * s;
}

// WENO-Z value at a Gauss point.
template <class R>
__device__ __forceinline__ R gauss_value(const R v[5], const GaussPoint<R>& gp) {
  R b[3], w[3], p[3], dp[3];
  js_smoothness(v, b);
  wz_weights(b, gp.dv0, gp.dv1, gp.dv2, w);
  gauss_candidates(v, gp.s, p, dp);
  return w[0] * p[0] + w[1] * p[1] + w[2] * p[2];
}

// WENO-Z value and slope at a Gauss point (slope with the slope weights).
template <class R>
__device__ __forceinline__ void gauss_value_slope(const R v[5], const GaussPoint<R>& gp, R& val, R& der) {
  R b[3], w[3], p[3], dp[3];
  js_smoothness(v, b);
  gauss_candidates(v, gp.s, p, dp);
  wz_weights(b, gp.dv0, gp.dv1, gp.dv2, w);
  val = w[0] * p[0] + w[1] * p[1] + w[2] * p[2];
  wz_weights(b, gp.dd0, gp.dd1, gp.dd2, w);
  der = w[0] * dp[0] + w[1] * dp[1] + w[2] * dp[2];
}

// Linear (fifth-order) value at a Gauss point: the quartic through the averages.
template <class R>
__device__ __forceinline__ R gauss_linear(const R v[5], const GaussPoint<R>& gp) {
  R p[3], dp[3];
  gauss_candidates(v, gp.s, p, dp);
  return gp.dv0 * p[0] + gp.dv1 * p[1] + gp.dv2 * p[2];
}

// Value and slope at the right face (s = 1/2) of the centre cell.
template <class R>
__device__ __forceinline__ void face_value_slope(const R v[5], R& val, R& der) {
  R b[3], w[3];
  js_smoothness(v, b);
  wz_weights(b, R(0.1), R(0.6), R(0.3), w);
  const R sixth = R(1.0 / 6.0);
  R p0 = (R(2) * v[0] - R(7) * v[1] + R(11) * v[2]) * sixth;
  R p1 = (R(5) * v[2] - v[1] + R(2) * v[3]) * sixth;
  R p2 = (R(2) * v[2] + R(5) * v[3] - v[4]) * sixth;
  R s0 = v[0] - R(3) * v[1] + R(2) * v[2];
  R s12 = v[3] - v[2];
  val = w[0] * p0 + w[1] * p1 + w[2] * p2;
  der = w[0] * s0 + (w[1] + w[2]) * s12;
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
__device__ __forceinline__ State<R> primitive(const R q[5], R gm1) {
  State<R> s;
  s.rho = q[0];
  R ir = R(1) / q[0];
  s.U = q[1] * ir;
  s.V = q[2] * ir;
  s.W = q[3] * ir;
  R p = gm1 * (q[4] - R(0.5) * (q[1] * s.U + q[2] * s.V + q[3] * s.W));
  s.lam = R(0.5) * q[0] / p;
  return s;
}

template <class R> struct Mom { R u[7], v[7], w[7], x[3]; };

template <class R>
__device__ __forceinline__ void chain(R mean, R ihl, R m0, R m1, R o[7]) {
  // ihl = 1/(2 lambda): <c^(n+2)> = mean <c^(n+1)> + (n+1) ihl <c^n>
  o[0] = m0;
  o[1] = m1;
#pragma unroll
  for (int n = 0; n < 5; ++n) o[n + 2] = mean * o[n + 1] + R(n + 1) * ihl * o[n];
}

// Half-space u-chain for u > 0 (SIDE = +1) or u < 0 (SIDE = -1).
template <class R, int SIDE>
__device__ __forceinline__ void half_chain(const State<R>& s, R ihl, R o[7]) {
  R sl = sqrt(s.lam);
  R e = exp(-s.lam * s.U * s.U) * R(0.28209479177387814347) / sl;  // e^{-l U^2} / (2 sqrt(pi l))
  R m0 = R(0.5) * erfc(-R(SIDE) * sl * s.U);
  R m1 = s.U * m0 + R(SIDE) * e;
  chain(s.U, ihl, m0, m1, o);
}

template <class R>
__device__ __forceinline__ void full_tangential(const State<R>& s, R ihl, R K, Mom<R>& m) {
  chain(s.V, ihl, R(1), s.V, m.v);
  chain(s.W, ihl, R(1), s.W, m.w);
  m.x[0] = R(1);
  m.x[1] = K * ihl;
  m.x[2] = K * (K + R(2)) * ihl * ihl;
}

template <class R, int A, int B, int C, int E>
__device__ __forceinline__ R mono(const Mom<R>& m) {
  return m.u[A] * m.v[B] * m.w[C] * m.x[E];
}

// <u^A v^B w^C (xi^2)^E psi>
template <class R, int A, int B, int C, int E>
__device__ __forceinline__ void mpsi(const Mom<R>& m, R o[5]) {
  o[0] = mono<R, A, B, C, E>(m);
  o[1] = mono<R, A + 1, B, C, E>(m);
  o[2] = mono<R, A, B + 1, C, E>(m);
  o[3] = mono<R, A, B, C + 1, E>(m);
  o[4] = R(0.5) * (mono<R, A + 2, B, C, E>(m) + mono<R, A, B + 2, C, E>(m) + mono<R, A, B, C + 2, E>(m) +
                   mono<R, A, B, C, E + 1>(m));
}

// o (+)= <(a . psi) u^A v^B w^C psi>
template <class R, int A, int B, int C, bool ACC>
__device__ __forceinline__ void mapsi(const Mom<R>& m, const R a[5], R o[5]) {
  R t0[5], t1[5], t2[5], t3[5], s0[5], s1[5], s2[5], s3[5];
  mpsi<R, A, B, C, 0>(m, t0);
  mpsi<R, A + 1, B, C, 0>(m, t1);
  mpsi<R, A, B + 1, C, 0>(m, t2);
  mpsi<R, A, B, C + 1, 0>(m, t3);
  mpsi<R, A + 2, B, C, 0>(m, s0);
  mpsi<R, A, B + 2, C, 0>(m, s1);
  mpsi<R, A, B, C + 2, 0>(m, s2);
  mpsi<R, A, B, C, 1>(m, s3);
  const R h = R(0.5) * a[4];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    R r = a[0] * t0[k] + a[1] * t1[k] + a[2] * t2[k] + a[3] * t3[k] + h * (s0[k] + s1[k] + s2[k] + s3[k]);
    o[k] = ACC ? o[k] + r : r;
  }
}

// Closed-form solution of <(a . psi) psi> = b for a Maxwellian state.
template <class R>
__device__ __forceinline__ void slope_solve(const State<R>& s, R ihl, R K, const R b[5], R a[5]) {
  R q2 = s.U * s.U + s.V * s.V + s.W * s.W + (K + R(3)) * ihl;
  R r2 = b[1] - s.U * b[0];
  R r3 = b[2] - s.V * b[0];
  R r4 = b[3] - s.W * b[0];
  R r5 = R(2) * b[4] - q2 * b[0];
  R tl = R(2) * s.lam;
  a[4] = tl * tl / (K + R(3)) * (r5 - R(2) * (s.U * r2 + s.V * r3 + s.W * r4));
  a[3] = tl * r4 - s.W * a[4];
  a[2] = tl * r3 - s.V * a[4];
  a[1] = tl * r2 - s.U * a[4];
  a[0] = b[0] - s.U * a[1] - s.V * a[2] - s.W * a[3] - R(0.5) * a[4] * q2;
}

// ---------------------------------------------------------------------------
// Gauss-point flux
// ---------------------------------------------------------------------------

template <class R> struct GasParams {
  R gm1;      // gamma - 1
  R K;        // internal degrees of freedom
  R mu_ref, T_ref, mu_exp;
  R pr_fix;   // 1/Pr - 1
};

// Integrals over [0, delta] of the six time factors of the BGK solution.
template <class R>
__device__ __forceinline__ void time_integrals(R tau, R delta, R C[6]) {
  if (tau > R(0)) {
    R eta = exp(-delta / tau);
    R om = R(1) - eta;
    R t2 = tau * tau;
    C[0] = delta - tau * om;
    C[1] = R(2) * t2 * om - tau * delta * (R(1) + eta);
    C[2] = R(0.5) * delta * delta - tau * delta + t2 * om;
    C[3] = tau * om;
    C[4] = tau * delta * eta - R(2) * t2 * om;
    C[5] = -t2 * om;
  } else {
    C[0] = delta; C[1] = R(0); C[2] = R(0.5) * delta * delta; C[3] = R(0); C[4] = R(0); C[5] = R(0);
  }
}

// Scalar part of the heat-flux correction: for a moment vector v of psi,
// v_E - U0 . v_m + |U0|^2/2 v_rho (energy in the frame of U0).
template <class R>
__device__ __forceinline__ R thermal(const R v[5], R U, R V, R W, R hu2) {
  return v[4] - (U * v[1] + V * v[2] + W * v[3]) + hu2 * v[0];
}

// Contributions of one non-equilibrium side (g_l with u > 0 or g_r with u < 0):
// flux moments weighted by C4, C5, C6 and the moments W of the same terms used
// by the Prandtl correction; also the side's part of the tangential slopes of
// Q0 (exact derivative of the compatibility map).
template <class R, int SIDE>
__device__ __forceinline__ void side_terms(const R q[5], const R dq[3][5], const GasParams<R>& g,
                                           const R C1[6], const R C2[6], R U0, R V0, R W0, R hu2,
                                           R F1[5], R F2[5], R& w1, R& w2, R dq0t[2][5]) {
  State<R> s = primitive(q, g.gm1);
  R ihl = R(0.5) / s.lam;
  Mom<R> m;
  full_tangential(s, ihl, g.K, m);
  // full u-chain first, for the time slope
  chain(s.U, ihl, R(1), s.U, m.u);
  R a[3][5], A[5];
  R ir = R(1) / s.rho;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    R b[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = dq[d][k] * ir;
    slope_solve(s, ihl, g.K, b, a[d]);
  }
  {
    R b[5];
    mapsi<R, 1, 0, 0, false>(m, a[0], b);
    mapsi<R, 0, 1, 0, true>(m, a[1], b);
    mapsi<R, 0, 0, 1, true>(m, a[2], b);
#pragma unroll
    for (int k = 0; k < 5; ++k) b[k] = -b[k];
    slope_solve(s, ihl, g.K, b, A);
  }
  // switch to the half-space u-chain
  half_chain<R, SIDE>(s, ihl, m.u);
  R X1[5], X2[5], X3[5];
  mpsi<R, 1, 0, 0, 0>(m, X1);
  mapsi<R, 2, 0, 0, false>(m, a[0], X2);
  mapsi<R, 1, 1, 0, true>(m, a[1], X2);
  mapsi<R, 1, 0, 1, true>(m, a[2], X2);
  mapsi<R, 1, 0, 0, false>(m, A, X3);
  const R rho = s.rho;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    F1[k] += rho * (C1[3] * X1[k] + C1[4] * X2[k] + C1[5] * X3[k]);
    F2[k] += rho * (C2[3] * X1[k] + C2[4] * X2[k] + C2[5] * X3[k]);
  }
  R Y1[5], Y2[5], Y3[5];
  mpsi<R, 0, 0, 0, 0>(m, Y1);
  mapsi<R, 1, 0, 0, false>(m, a[0], Y2);
  mapsi<R, 0, 1, 0, true>(m, a[1], Y2);
  mapsi<R, 0, 0, 1, true>(m, a[2], Y2);
  mapsi<R, 0, 0, 0, false>(m, A, Y3);
  R y1 = thermal(Y1, U0, V0, W0, hu2), y2 = thermal(Y2, U0, V0, W0, hu2), y3 = thermal(Y3, U0, V0, W0, hu2);
  w1 += rho * (C1[3] * y1 + C1[4] * y2 + C1[5] * y3);
  w2 += rho * (C2[3] * y1 + C2[4] * y2 + C2[5] * y3);
  R t[5];
  mapsi<R, 0, 0, 0, false>(m, a[1], t);
#pragma unroll
  for (int k = 0; k < 5; ++k) dq0t[0][k] += rho * t[k];
  mapsi<R, 0, 0, 0, false>(m, a[2], t);
#pragma unroll
  for (int k = 0; k < 5; ++k) dq0t[1][k] += rho * t[k];
}

// Time-integrated flux at one Gauss point, local frame (n, t1, t2), for the
// windows [0, dt] (F1) and [0, dt/2] (F2).  Slopes in physical units.
template <class R>
__device__ __forceinline__ void gp_flux(const R ql[5], const R qr[5], const R dql[3][5], const R dqr[3][5],
                                        const R dq0n[5], const GasParams<R>& g, R dt, R F1[5], R F2[5]) {
  // interface equilibrium from the compatibility condition
  R q0[5];
  {
    State<R> sl = primitive(ql, g.gm1), sr = primitive(qr, g.gm1);
    Mom<R> m;
    R ihl = R(0.5) / sl.lam;
    full_tangential(sl, ihl, g.K, m);
    half_chain<R, 1>(sl, ihl, m.u);
    R h[5];
    mpsi<R, 0, 0, 0, 0>(m, h);
#pragma unroll
    for (int k = 0; k < 5; ++k) q0[k] = sl.rho * h[k];
    ihl = R(0.5) / sr.lam;
    full_tangential(sr, ihl, g.K, m);
    half_chain<R, -1>(sr, ihl, m.u);
    mpsi<R, 0, 0, 0, 0>(m, h);
#pragma unroll
    for (int k = 0; k < 5; ++k) q0[k] += sr.rho * h[k];
  }
  State<R> s0 = primitive(q0, g.gm1);
  R ihl0 = R(0.5) / s0.lam;
  // collision time tau = mu(T0) / p0, T0 = p0/rho0 = 1/(2 lambda0)
  R p0 = s0.rho * ihl0;
  R mu = g.mu_ref;
  if (g.mu_exp != R(0)) mu = g.mu_ref * pow(ihl0 / g.T_ref, g.mu_exp);
  R tau = mu / p0;
  R C1[6], C2[6];
  time_integrals(tau, dt, C1);
  time_integrals(tau, R(0.5) * dt, C2);
  R hu2 = R(0.5) * (s0.U * s0.U + s0.V * s0.V + s0.W * s0.W);
#pragma unroll
  for (int k = 0; k < 5; ++k) { F1[k] = R(0); F2[k] = R(0); }
  R w1 = R(0), w2 = R(0);
  R dq0t[2][5];
#pragma unroll
  for (int k = 0; k < 5; ++k) { dq0t[0][k] = R(0); dq0t[1][k] = R(0); }
  side_terms<R, 1>(ql, dql, g, C1, C2, s0.U, s0.V, s0.W, hu2, F1, F2, w1, w2, dq0t);
  side_terms<R, -1>(qr, dqr, g, C1, C2, s0.U, s0.V, s0.W, hu2, F1, F2, w1, w2, dq0t);
  // equilibrium part
  {
    Mom<R> m;
    full_tangential(s0, ihl0, g.K, m);
    chain(s0.U, ihl0, R(1), s0.U, m.u);
    R a[3][5], A[5];
    R ir = R(1) / s0.rho;
    {
      R b[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) b[k] = dq0n[k] * ir;
      slope_solve(s0, ihl0, g.K, b, a[0]);
#pragma unroll
      for (int k = 0; k < 5; ++k) b[k] = dq0t[0][k] * ir;
      slope_solve(s0, ihl0, g.K, b, a[1]);
#pragma unroll
      for (int k = 0; k < 5; ++k) b[k] = dq0t[1][k] * ir;
      slope_solve(s0, ihl0, g.K, b, a[2]);
    }
    R Y2[5];  // sum_d <s_d (a_d . psi) psi>_0
    mapsi<R, 1, 0, 0, false>(m, a[0], Y2);
    mapsi<R, 0, 1, 0, true>(m, a[1], Y2);
    mapsi<R, 0, 0, 1, true>(m, a[2], Y2);
    {
      R b[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) b[k] = -Y2[k];
      slope_solve(s0, ihl0, g.K, b, A);
    }
    R X1[5], X2[5], X3[5];
    mpsi<R, 1, 0, 0, 0>(m, X1);
    mapsi<R, 2, 0, 0, false>(m, a[0], X2);
    mapsi<R, 1, 1, 0, true>(m, a[1], X2);
    mapsi<R, 1, 0, 1, true>(m, a[2], X2);
    mapsi<R, 1, 0, 0, false>(m, A, X3);
    const R rho = s0.rho;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      F1[k] += rho * (C1[0] * X1[k] + C1[1] * X2[k] + C1[2] * X3[k]);
      F2[k] += rho * (C2[0] * X1[k] + C2[1] * X2[k] + C2[2] * X3[k]);
    }
    // W-moments of the equilibrium terms: <psi>_0, Y2 and <A psi>_0 = -Y2
    R Y1[5];
    mpsi<R, 0, 0, 0, 0>(m, Y1);
    R Y3[5];
    mapsi<R, 0, 0, 0, false>(m, A, Y3);
    R y1 = thermal(Y1, s0.U, s0.V, s0.W, hu2);
    R y2 = thermal(Y2, s0.U, s0.V, s0.W, hu2);
    R y3 = thermal(Y3, s0.U, s0.V, s0.W, hu2);
    w1 += rho * (C1[0] * y1 + C1[1] * y2 + C1[2] * y3);
    w2 += rho * (C2[0] * y1 + C2[1] * y2 + C2[2] * y3);
  }
  // Prandtl correction of the energy flux: q = thermal(F) - U0_n thermal(W)
  R qh1 = thermal(F1, s0.U, s0.V, s0.W, hu2) - s0.U * w1;
  R qh2 = thermal(F2, s0.U, s0.V, s0.W, hu2) - s0.U * w2;
  F1[4] += g.pr_fix * qh1;
  F2[4] += g.pr_fix * qh2;
}

}  // namespace hgks
