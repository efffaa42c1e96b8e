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

// Reciprocals of the two weight sums of a Gauss-point pair.  FP64: both from
// one reciprocal of their product (the hardware reciprocal issues at a
// quarter of the FMA rate; the sums lie between about 1e-60 and the sixth
// power of the data's squared variation, so the product stays in range);
// FP32, whose sums can reach 1e20, one each.
template <class R> __device__ __forceinline__ void wz_rcp2(R x, R y, R& ix, R& iy);
template <> __device__ __forceinline__ void wz_rcp2<double>(double x, double y, double& ix, double& iy) {
  const double r = wz_rcp(x * y);
  ix = y * r;
  iy = x * r;
}
template <> __device__ __forceinline__ void wz_rcp2<float>(float x, float y, float& ix, float& iy) {
  ix = wz_rcp(x);
  iy = wz_rcp(y);
}

// The three quadratic candidates through averages (v0,v1,v2), (v1,v2,v3),
// (v2,v3,v4), written about the centre cell (x in [-1/2, 1/2]) as
// p_k(x) = v2 - c_k/24 + b_k x + c_k x^2 / 2: c_k is the candidate's second
// difference, b_k its slope at the centre, both formed from the first
// differences d_j = v_{j+1} - v_j: c_0 = d_1 - d_0, c_1 = d_2 - d_1,
// c_2 = d_3 - d_2, and tb_k = 2 b_k: tb_0 = 2 d_1 + c_0, tb_1 = d_1 + d_2,
// tb_2 = 2 d_2 - c_2.  be_k = 13/3 c_k^2 + tb_k^2 + 4 eps is four times the
// Jiang-Shu smoothness indicator 13/12 c_k^2 + b_k^2 plus the WENO-Z
// epsilon: the normalised weights do not change when every indicator and
// tau5 are scaled alike.
template <class R> struct Candidates { R c[3], tb[3], be[3]; };

template <class R>
__device__ __forceinline__ Candidates<R> candidates(const R v[5]) {
  Candidates<R> k;
  const R d0 = v[1] - v[0], d1 = v[2] - v[1], d2 = v[3] - v[2], d3 = v[4] - v[3];
  k.c[0] = d1 - d0;
  k.c[1] = d2 - d1;
  k.c[2] = d3 - d2;
  k.tb[0] = R(2) * d1 + k.c[0];
  k.tb[1] = d1 + d2;
  k.tb[2] = R(2) * d2 - k.c[2];
  const R c13 = R(13.0 / 3.0), eps4 = R(4) * WenoEps<R>::v;
#pragma unroll
  for (int i = 0; i < 3; ++i) k.be[i] = (c13 * k.c[i]) * k.c[i] + (k.tb[i] * k.tb[i] + eps4);
  return k;
}

// Nonlinear weights alpha_k = d_k (1 + tau5 / b_k), b_k = beta_k + eps,
// tau5 = |beta_0 - beta_2|, normalised (from be_k = 4 b_k and 4 tau5, the
// same weights).  wz_factors gives e_k with alpha_k
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
    // e_k = (b_k + tau5) prod_{j != k} b_j = P + tau5 prod_{j != k} b_j
    const R q12 = be[1] * be[2], q02 = be[0] * be[2], q01 = be[0] * be[1];
    const R P = be[0] * q12;
    e[0] = P + t5 * q12;
    e[1] = P + t5 * q02;
    e[2] = P + t5 * q01;
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

// Both Gauss points of one stencil (index 0: s = -sqrt3/6, 1: s = +sqrt3/6)
// from one set of candidates and WENO-Z factors.  At +s the value is
// v2 + s sum w_k b_k with the value weights (dv0, dv1, dv2) and the slope
// sum w_k (b_k + s c_k) with the slope weights (dd0, dd1, dd2); at -s the
// weights are reversed and s changes sign.  With y_k = e_k tb_k = 2 e_k b_k
// and z_k = e_k c_k every such sum is
// (sum_k (d_k/2) y_k [+- s sum_k d_k z_k]) / sum_k d_k e_k, the factors
// being constants.
template <class R>
__device__ __forceinline__ void gauss_value2(const R v[5], R val[2]) {
  using G = GaussConst;
  const Candidates<R> k = candidates(v);
  R e[3];
  wz_factors(k.be, e);
  const R y0 = e[0] * k.tb[0], y1 = e[1] * k.tb[1], y2 = e[2] * k.tb[2];
  const R nm = R(0.5 * G::s * G::dv2) * y0 + R(0.5 * G::s * G::dv1) * y1 + R(0.5 * G::s * G::dv0) * y2;
  const R dm = R(G::dv2) * e[0] + R(G::dv1) * e[1] + R(G::dv0) * e[2];
  const R np = R(0.5 * G::s * G::dv0) * y0 + R(0.5 * G::s * G::dv1) * y1 + R(0.5 * G::s * G::dv2) * y2;
  const R dp = R(G::dv0) * e[0] + R(G::dv1) * e[1] + R(G::dv2) * e[2];
  R im, ip;
  wz_rcp2(dm, dp, im, ip);
  val[0] = v[2] - nm * im;
  val[1] = v[2] + np * ip;
}

template <class R>
__device__ __forceinline__ void gauss_value_slope2(const R v[5], R val[2], R der[2]) {
  using G = GaussConst;
  const Candidates<R> k = candidates(v);
  R e[3];
  wz_factors(k.be, e);
  const R y0 = e[0] * k.tb[0], y1 = e[1] * k.tb[1], y2 = e[2] * k.tb[2];
  const R z0 = e[0] * k.c[0], z1 = e[1] * k.c[1], z2 = e[2] * k.c[2];
  const R nm = R(0.5 * G::s * G::dv2) * y0 + R(0.5 * G::s * G::dv1) * y1 + R(0.5 * G::s * G::dv0) * y2;
  const R dm = R(G::dv2) * e[0] + R(G::dv1) * e[1] + R(G::dv0) * e[2];
  const R np = R(0.5 * G::s * G::dv0) * y0 + R(0.5 * G::s * G::dv1) * y1 + R(0.5 * G::s * G::dv2) * y2;
  const R dp = R(G::dv0) * e[0] + R(G::dv1) * e[1] + R(G::dv2) * e[2];
  R im, ip;
  wz_rcp2(dm, dp, im, ip);
  val[0] = v[2] - nm * im;
  val[1] = v[2] + np * ip;
  const R sm = R(0.5 * G::dd2) * y0 + R(0.5 * G::dd1) * y1 + R(0.5 * G::dd0) * y2 + R(-G::s * G::dd2) * z0 +
               R(-G::s * G::dd1) * z1 + R(-G::s * G::dd0) * z2;
  const R em = R(G::dd2) * e[0] + R(G::dd1) * e[1] + R(G::dd0) * e[2];
  const R sp = R(0.5 * G::dd0) * y0 + R(0.5 * G::dd1) * y1 + R(0.5 * G::dd2) * y2 + R(G::s * G::dd0) * z0 +
               R(G::s * G::dd1) * z1 + R(G::s * G::dd2) * z2;
  const R ep = R(G::dd0) * e[0] + R(G::dd1) * e[1] + R(G::dd2) * e[2];
  wz_rcp2(em, ep, im, ip);
  der[0] = sm * im;
  der[1] = sp * ip;
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

// Linear (fifth-order) value at a Gauss point: the quartic through the
// averages, v2 + s (dv0 b0 + dv1 b1 + dv2 b2) with the candidates' slopes b_k
// written out, a fixed weighted sum of the five averages.  Weights at
// s = +sqrt3/6; at -sqrt3/6 they apply to the reversed stencil.
struct LinearGauss {
  static constexpr double s = GaussConst::s, d0 = GaussConst::dv0, d1 = GaussConst::dv1, d2 = GaussConst::dv2;
  static constexpr double w0 = s * d0 * 0.5;
  static constexpr double w1 = s * (-2.0 * d0 - 0.5 * d1);
  static constexpr double w2 = 1.0 + s * (1.5 * d0 - 1.5 * d2);
  static constexpr double w3 = s * (0.5 * d1 + 2.0 * d2);
  static constexpr double w4 = -s * d2 * 0.5;
};
// The weights of a lane's Gauss point (g = 1: +sqrt3/6, g = 0: -sqrt3/6).
template <class R> struct LinearWeights {
  R w[5];
  __device__ __forceinline__ explicit LinearWeights(int g) {
    using L = LinearGauss;
    const bool p = g != 0;
    w[0] = p ? R(L::w0) : R(L::w4);
    w[1] = p ? R(L::w1) : R(L::w3);
    w[2] = R(L::w2);
    w[3] = p ? R(L::w3) : R(L::w1);
    w[4] = p ? R(L::w4) : R(L::w0);
  }
};
template <class R>
__device__ __forceinline__ R gauss_linear(const R v[5], const LinearWeights<R>& lw) {
  return lw.w[0] * v[0] + lw.w[1] * v[1] + lw.w[2] * v[2] + lw.w[3] * v[3] + lw.w[4] * v[4];
}

// Value and slope at the right face (s = 1/2) of the centre cell: candidate
// value v2 + b_k/2 + c_k/12 = v2 + tb_k/4 + c_k/12, slope b_k + c_k/2 =
// (tb_k + c_k)/2.
template <class R>
__device__ __forceinline__ void face_value_slope(const Candidates<R>& k, R v2, R& val, R& der) {
  R e[3], a[3];
  wz_factors(k.be, e);
  const R inv = wz_alpha(e, R(0.1), R(0.6), R(0.3), a);
  const R twelfth = R(1.0 / 12.0);
  val = v2 + inv * wz_dot(a, R(0.25) * k.tb[0] + twelfth * k.c[0], R(0.25) * k.tb[1] + twelfth * k.c[1],
                          R(0.25) * k.tb[2] + twelfth * k.c[2]);
  der = (R(0.5) * inv) * wz_dot(a, k.tb[0] + k.c[0], k.tb[1] + k.c[1], k.tb[2] + k.c[2]);
}

// Normal sweep at face i+1/2 from c[0..5] = Q_{i-2..i+3}: left/right values and
// slopes, and the equilibrium slope (Q_{i-1} - 15 Q_i + 15 Q_{i+1} - Q_{i+2})/12.
// The left state's stencil is (c0, ..., c4), the right state's the mirrored
// (c5, ..., c1): with the first differences e_j = c_{j+1} - c_j the right
// stencil's differences are (-e4, -e3, -e2, -e1), so the two candidate sets
// share four differences and two second differences (c_1 and c_2 swapped),
// each formed once (the same values, bit for bit, as from each stencil alone).
template <class R>
__device__ __forceinline__ void normal_sweep(const R c[6], R& ql, R& qr, R& dl, R& dr, R& d0) {
  const R e0 = c[1] - c[0], e1 = c[2] - c[1], e2 = c[3] - c[2], e3 = c[4] - c[3], e4 = c[5] - c[4];
  Candidates<R> kl, kr;
  kl.c[0] = e1 - e0;
  kl.c[1] = e2 - e1;
  kl.c[2] = e3 - e2;
  kl.tb[0] = R(2) * e1 + kl.c[0];
  kl.tb[1] = e1 + e2;
  kl.tb[2] = R(2) * e2 - kl.c[2];
  kr.c[0] = e4 - e3;
  kr.c[1] = kl.c[2];
  kr.c[2] = kl.c[1];
  kr.tb[0] = R(-2) * e3 + kr.c[0];
  kr.tb[1] = -(e3 + e2);
  kr.tb[2] = R(-2) * e2 - kr.c[2];
  const R c13 = R(13.0 / 3.0), eps4 = R(4) * WenoEps<R>::v;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    kl.be[i] = (c13 * kl.c[i]) * kl.c[i] + (kl.tb[i] * kl.tb[i] + eps4);
    kr.be[i] = (c13 * kr.c[i]) * kr.c[i] + (kr.tb[i] * kr.tb[i] + eps4);
  }
  face_value_slope(kl, c[2], ql, dl);
  R m;
  face_value_slope(kr, c[3], qr, m);
  dr = -m;
  d0 = (c[1] - c[4] + R(15) * e2) * R(1.0 / 12.0);
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

// sqrt(x) and 1/sqrt(x) of a positive, normal number.  FP64: the hardware
// reciprocal-square-root estimate refined by two Newton steps
// y <- y + y (1 - x y^2) / 2 (the estimate's relative error squares at each
// step, leaving a few ulp), sqrt(x) = x y.  FP32: sqrt and its hardware
// reciprocal.
__device__ __forceinline__ void sqrt_rsqrt(double x, double& sq, double& rs) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  rs = y;
  sq = x * y;
}
__device__ __forceinline__ void sqrt_rsqrt(float x, float& sq, float& rs) {
  sq = sqrtf(x);
  rs = __builtin_amdgcn_rcpf(sq);
}

// n! as a compile-time constant.
template <int N> struct Factorial { static constexpr double value = N * Factorial<N - 1>::value; };
template <> struct Factorial<0> { static constexpr double value = 1.0; };

// Taylor coefficients in t = x^2: e^{-t} = sum_n (-t)^n / n!, and
// erf(x) / x = 2/sqrt(pi) sum_n (-t)^n / (n! (2n + 1)).
struct ExpNegSeries {
  template <int n> static constexpr double coef() { return ((n & 1) ? -1.0 : 1.0) / Factorial<n>::value; }
};
struct ErfSeries {
  template <int n> static constexpr double coef() {
    return 1.1283791670955125739 * ((n & 1) ? -1.0 : 1.0) / (Factorial<n>::value * (2 * n + 1));
  }
};
// A compile-time constant held in scalar registers for the one FMA that
// reads it.  As an FMA's addend the compiler would otherwise copy it into
// vector registers first (two VALU moves per FP64 constant, for the
// two-operand FMA form); from scalar registers it is an operand of the
// three-operand form, and the scalar moves issue beside another wave's VALU
// work.
template <class R> __device__ __forceinline__ R in_sgpr(R c) {
  asm volatile("" : "+s"(c));
  return c;
}

// sum_{n <= N} S::coef<n>() t^n in Horner form (p enters as the t^N coefficient).
template <class R, class S, int N>
__device__ __forceinline__ R horner(R t, R p) {
  if constexpr (N == 0) {
    return p;
  } else {
    return horner<R, S, N - 1>(t, p * t + in_sgpr(R(S::template coef<N - 1>())));
  }
}
template <class R, class S, int N> __device__ __forceinline__ R series(R t) {
  return horner<R, S, N>(t, R(S::template coef<N>()));
}
// e^r = sum_n r^n / n!.
struct ExpSeries {
  template <int n> static constexpr double coef() { return 1.0 / Factorial<n>::value; }
};

// e^x for x <= 0.  FP64: x = k ln2 + r with k = rint(x / ln2) and
// |r| <= ln2 / 2 (Cody-Waite reduction: ln 2 split into a head of 42
// significant bits, so that k ln2_hi is exact for the |k| < 2^11 of the
// exponent range, and the rounded remainder), e^r from its Taylor series of
// degree 13 (first omitted term below 4e-18 of the sum), times 2^k.
// Arguments below -1000 (and -inf) give 0.  FP32: the device library's exp.
constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;   // ln 2 rounded to 42 bits
constexpr double kLn2Lo = 0x1.ef35793c76730p-45;  // ln 2 - kLn2Hi, rounded
__device__ __forceinline__ double exp_nonpos(double x) {
  x = fmax(x, -1000.0);
  const double k = __builtin_rint(x * 1.4426950408889634);  // x / ln 2
  double r = fma(-k, kLn2Hi, x);
  r = fma(-k, kLn2Lo, r);
  return __builtin_amdgcn_ldexp(series<double, ExpSeries, 13>(r), (int)k);
}
__device__ __forceinline__ float exp_nonpos(float x) { return expf(x); }

// Degrees for |x| <= 1/2 (t <= 1/4): the first omitted term is below 3e-18
// (FP64) or 4e-10 (FP32) of the sum.
template <class R> struct HalfSeries;
template <> struct HalfSeries<double> { static constexpr int kExp = 12, kErf = 11; };
template <> struct HalfSeries<float> { static constexpr int kExp = 7, kErf = 6; };

// Zeroth and first half-space u-moments, u > 0 (SIDE = +1) or u < 0 (SIDE = -1):
// with x = sqrt(lambda) U, m0 = erfc(-SIDE x) / 2 and
// m1 = U m0 + SIDE e^{-x^2} / (2 sqrt(pi lambda)).  For |x| <= 1/2 (the
// low-Mach states) e^{-x^2} and erf(x) come from their Taylor series, and
// erfc(-SIDE x) = 1 + SIDE erf(x); elsewhere from the device library.
template <class R, int SIDE>
__device__ __forceinline__ void half_moments01(const State<R>& s, R& m0, R& m1) {
  R sl, isl;
  sqrt_rsqrt(s.lam, sl, isl);
  const R x = sl * s.U;
  R ex, ec;
  if (fabs(x) <= R(0.5)) {
    const R t = x * x;
    ex = series<R, ExpNegSeries, HalfSeries<R>::kExp>(t);
    ec = R(1) + R(SIDE) * (x * series<R, ErfSeries, HalfSeries<R>::kErf>(t));
  } else {
    ex = exp(-s.lam * s.U * s.U);
    ec = erfc(-R(SIDE) * x);
  }
  const R e = ex * R(0.28209479177387814347) * isl;  // e^{-l U^2} / (2 sqrt(pi l))
  m0 = R(0.5) * ec;
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

// u-series of Pi = u (an . psi) + v (at1 . psi) + w (at2 . psi):
// Pi_0 = v p_t1 + w p_t2, Pi_1 = p_n + at1_1 v + at2_1 w, Pi_2 = an_1 + h_t1 v + h_t2 w, Pi_3 = h_n.
// Each term's coefficients are gathered per monomial before its moments are
// taken: Pi_0 = at1_0 v + at2_0 w + at1_2 v^2 + (at1_3 + at2_2) v w + at2_3 w^2
// + h_t1 v r + h_t2 w r, and Pi_1 is p of (an_0, ., an_2 + at1_1, an_3 + at2_1, an_4).
template <class R>
__device__ __forceinline__ void series_pi(const R a[3][5], const VW<R>& e, Quad<R> q[4]) {
  const R h1 = R(0.5) * a[1][4], h2 = R(0.5) * a[2][4];
  const R cvw = a[1][3] + a[2][2];
  q[0].e0 = a[1][0] * e.v + a[2][0] * e.w + a[1][2] * e.vv + cvw * e.vw + a[2][3] * e.ww + h1 * e.vr + h2 * e.wr;
  q[0].ev = a[1][0] * e.vv + a[2][0] * e.vw + a[1][2] * e.vvv + cvw * e.vvw + a[2][3] * e.vww + h1 * e.vvr +
            h2 * e.vwr;
  q[0].ew = a[1][0] * e.vw + a[2][0] * e.ww + a[1][2] * e.vvw + cvw * e.vww + a[2][3] * e.www + h1 * e.vwr +
            h2 * e.wwr;
  q[0].er = a[1][0] * e.vr + a[2][0] * e.wr + a[1][2] * e.vvr + cvw * e.vwr + a[2][3] * e.wwr + h1 * e.vrr +
            h2 * e.wrr;
  const R p1[5] = {a[0][0], R(0), a[0][2] + a[1][1], a[0][3] + a[2][1], a[0][4]};
  q[1] = quad_p(p1, e);
  q[2] = quad_lin(a[0][1], h1, h2, e);
  q[3] = quad_c(R(0.5) * a[0][4], e);
}

// Closed-form solution of <(a . psi) psi> = c b for a Maxwellian state
// (normalised by density).  The common scale c of the right-hand side is
// folded into the solve's constants, t1 = 2 lambda c and
// t2 = (2 lambda)^2 c / (K + 3): the flux solves with c = 1 for the
// micro-slopes times the density (b the slopes of the conserved variables)
// and with c = -1 for the time-derivative condition.
template <class R> struct SlopeSolve { R U, V, W, q2, c, t1, t2; };

template <class R>
__device__ __forceinline__ SlopeSolve<R> slope_solver(const State<R>& s, R ihl, R K3, R iK3, R c) {
  SlopeSolve<R> S;
  S.U = s.U;
  S.V = s.V;
  S.W = s.W;
  S.q2 = s.U * s.U + s.V * s.V + s.W * s.W + K3 * ihl;
  const R tl = R(2) * s.lam;
  S.c = c;
  S.t1 = tl * c;
  S.t2 = tl * tl * iK3 * c;
  return S;
}

template <class R>
__device__ __forceinline__ void slope_solve(const SlopeSolve<R>& S, const R b[5], R a[5]) {
  const R r2 = b[1] - S.U * b[0];
  const R r3 = b[2] - S.V * b[0];
  const R r4 = b[3] - S.W * b[0];
  const R r5 = R(2) * b[4] - S.q2 * b[0];
  a[4] = S.t2 * (r5 - R(2) * (S.U * r2 + S.V * r3 + S.W * r4));
  a[3] = S.t1 * r4 - S.W * a[4];
  a[2] = S.t1 * r3 - S.V * a[4];
  a[1] = S.t1 * r2 - S.U * a[4];
  a[0] = S.c * b[0] - S.U * a[1] - S.V * a[2] - S.W * a[3] - R(0.5) * a[4] * S.q2;
}

// <u^X (a . psi) psi> for a u-moment table Mu, in closed form.  With
// p = a0 + a2 v + a3 w + h r (h = a4/2), (a . psi) = p + a1 u + h u^2; qp
// holds the (v, w, xi)-moments of p (quad_p) and c = Mu[X+1] a1 + Mu[X+2] h:
//   o0 = Mu[X] E[p] + c,  o1 = Mu[X+1] E[p] + Mu[X+2] a1 + Mu[X+3] h,
//   o2 = Mu[X] E[v p] + E[v] c,  o3 = Mu[X] E[w p] + E[w] c,
//   o4 = (Mu[X+2] E[p] + Mu[X+3] a1 + Mu[X+4] h + Mu[X] E[r p] + E[r] c) / 2
// (the assembly of the u-series (p, a1, h) with its two constant terms
// gathered).
template <class R, int X>
__device__ __forceinline__ void assemble_apsi(const R a[5], const Quad<R>& qp, const VW<R>& e, const R Mu[7],
                                              R o[5]) {
  const R h = R(0.5) * a[4];
  const R c = Mu[X + 1] * a[1] + Mu[X + 2] * h;
  o[0] = Mu[X] * qp.e0 + c;
  o[1] = Mu[X + 1] * qp.e0 + Mu[X + 2] * a[1] + Mu[X + 3] * h;
  o[2] = Mu[X] * qp.ev + e.v * c;
  o[3] = Mu[X] * qp.ew + e.w * c;
  o[4] = R(0.5) * (Mu[X + 2] * qp.e0 + Mu[X + 3] * a[1] + Mu[X + 4] * h + Mu[X] * qp.er + e.r * c);
}

// ---------------------------------------------------------------------------
// Gauss-point flux
// ---------------------------------------------------------------------------

template <class R> struct GasParams {
  R gm1;       // gamma - 1
  R K;         // internal degrees of freedom
  R K3, iK3;   // K + 3 and its reciprocal
  R mu_ref, iT_ref, mu_exp;
  R imu_ref;   // 1/mu_ref (0 for mu_ref = 0)
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
  const R h = tau > R(0) ? exp_nonpos(-(R(0.5) * dt) * itau) : R(0);
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

// thermal() of the u^0 moment <(a . psi) psi> (the u-series (p, a1, h) of
// assemble_apsi): the p term as in thermal_series, the constant terms
// gathered, theta = E[r]/2 - V E[v] - W E[w] the frame's weight of the
// unit polynomial.
template <class R>
__device__ __forceinline__ R thermal_apsi(const R a[5], const Quad<R>& qp, const R Mu[7], const R Tw[4], R theta,
                                          R V, R W) {
  const R h = R(0.5) * a[4];
  return qp.e0 * Tw[0] + Mu[0] * (R(0.5) * qp.er - V * qp.ev - W * qp.ew) + a[1] * Tw[1] + h * Tw[2] +
         (Mu[1] * a[1] + Mu[2] * h) * theta;
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
  // collision time tau = mu(T0) / p0, T0 = p0/rho0 = 1/(2 lambda0); the
  // reciprocals come from those already formed: 1/p0 = 2 lambda0 / rho0 and
  // 1/tau = p0 / mu
  const R p0 = A.s0.rho * A.ihl0;
  const R ip0 = R(2) * A.s0.lam * ir0;
  R mu = g.mu_ref, imu = g.imu_ref;
  if (g.mu_exp != R(0)) {
    mu = g.mu_ref * pow(A.ihl0 * g.iT_ref, g.mu_exp);
    imu = pos_rcp(mu);
  }
  const R tau = mu * ip0;
  const R itau = tau > R(0) ? p0 * imu : R(0);
  time_integrals(tau, itau, dt, A.Cn, A.Cd);
  A.hu2 = R(0.5) * (A.s0.U * A.s0.U + A.s0.V * A.s0.V + A.s0.W * A.s0.W);
  // The accumulators start at -0: -0 + x = x exactly for every x, so the
  // compiler drops the first addition into each (from +0 it could not, as
  // +0 + -0 = +0).
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    A.Fn[k] = R(-0.0);
    A.Fd[k] = R(-0.0);
    A.dq0t[0][k] = R(-0.0);
    A.dq0t[1][k] = R(-0.0);
  }
  A.wn = R(-0.0);
  A.wd = R(-0.0);
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
  // micro-slopes of the three directions times the side's density,
  // <(a_d . psi) psi> = dq_d: every term below that is linear in them (the
  // C5 and C6 moments, the time slope, the tangential slopes of Q0) then
  // carries its factor rho already
  const SlopeSolve<R> Sq = slope_solver(s, ihl, g.K3, g.iK3, R(1));
  R a[3][5];
#pragma unroll
  for (int d = 0; d < 3; ++d) slope_solve(Sq, dq[d], a[d]);
  Quad<R> pi[4];
  series_pi(a, e, pi);
  R A[5];
  {
    // time slope from <(A . psi) psi> = -<Pi psi>
    R Mf[7], T[5];
    chain<R, 7>(s.U, ihl, R(1), s.U, Mf);
    assemble<R, 0, 4>(pi, Mf, T);
    slope_solve(slope_solver(s, ihl, g.K3, g.iK3, R(-1)), T, A);
  }
  R Mh[7];
  if (LEFT) chain<R, 7>(s.U, ihl, Acc.lm0, Acc.lm1, Mh);
  else chain<R, 7>(s.U, ihl, Acc.rm0, Acc.rm1, Mh);
  const Quad<R> unit[1] = {quad_c(R(1), e)};
  const Quad<R> qA = quad_p(A, e);
  const R U0 = Acc.s0.U, V0 = Acc.s0.V, W0 = Acc.s0.W;
  // the time coefficients of the side's three terms, times its density for
  // the first (the other two carry it through the slopes)
  const R rn[3] = {s.rho * Acc.Cn[3], Acc.Cn[4], Acc.Cn[5]};
  const R rd[3] = {s.rho * Acc.Cd[3], Acc.Cd[4], Acc.Cd[5]};
  {
    R X1[5], X2[5], X3[5];
    assemble<R, 1, 1>(unit, Mh, X1);
    assemble<R, 1, 4>(pi, Mh, X2);
    assemble_apsi<R, 1>(A, qA, e, Mh, X3);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      Acc.Fn[k] = ((Acc.Fn[k] + rn[0] * X1[k]) + rn[1] * X2[k]) + rn[2] * X3[k];
      Acc.Fd[k] = ((Acc.Fd[k] + rd[0] * X1[k]) + rd[1] * X2[k]) + rd[2] * X3[k];
    }
  }
  {
    R Tw[4];
    thermal_weights(Mh, U0, Acc.hu2, Tw);
    const R theta = R(0.5) * e.r - V0 * e.v - W0 * e.w;
    const R y1 = Tw[0] + Mh[0] * theta;
    const R y2 = thermal_series<R, 4>(pi, Mh, Tw, V0, W0);
    const R y3 = thermal_apsi(A, qA, Mh, Tw, theta, V0, W0);
    Acc.wn = ((Acc.wn + rn[0] * y1) + rn[1] * y2) + rn[2] * y3;
    Acc.wd = ((Acc.wd + rd[0] * y1) + rd[1] * y2) + rd[2] * y3;
  }
#pragma unroll
  for (int d = 1; d < 3; ++d) {
    R t[5];
    assemble_apsi<R, 0>(a[d], quad_p(a[d], e), e, Mh, t);
#pragma unroll
    for (int k = 0; k < 5; ++k) Acc.dq0t[d - 1][k] += t[k];
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
  R a[3][5];  // the equilibrium's micro-slopes times rho0, as on the sides
  {
    const SlopeSolve<R> Sq = slope_solver(s0, ihl0, g.K3, g.iK3, R(1));
    slope_solve(Sq, dq0n, a[0]);
    slope_solve(Sq, Acc.dq0t[0], a[1]);
    slope_solve(Sq, Acc.dq0t[1], a[2]);
  }
  Quad<R> pi[4];
  series_pi(a, e, pi);
  R T[5];  // rho0 sum_d <s_d (a_d . psi) psi>_0
  assemble<R, 0, 4>(pi, Mf, T);
  R A[5];
  slope_solve(slope_solver(s0, ihl0, g.K3, g.iK3, R(-1)), T, A);
  const Quad<R> unit[1] = {quad_c(R(1), e)};
  const Quad<R> qA = quad_p(A, e);
  const R rn[3] = {s0.rho * Acc.Cn[0], Acc.Cn[1], Acc.Cn[2]};
  const R rd[3] = {s0.rho * Acc.Cd[0], Acc.Cd[1], Acc.Cd[2]};
  R X1[5], X2[5], X3[5];
  assemble<R, 1, 1>(unit, Mf, X1);
  assemble<R, 1, 4>(pi, Mf, X2);
  assemble_apsi<R, 1>(A, qA, e, Mf, X3);
  // the equilibrium flux term (X1, of the size of the pressure) is added
  // last: the smaller terms summed after it would each be rounded at its
  // magnitude, which in FP32 made the mixed path lose kinetic energy against
  // FP64 about 50 times faster on the low-Mach TGV
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    Fn[k] = ((Acc.Fn[k] + rn[1] * X2[k]) + rn[2] * X3[k]) + rn[0] * X1[k];
    Fd[k] = ((Acc.Fd[k] + rd[1] * X2[k]) + rd[2] * X3[k]) + rd[0] * X1[k];
  }
  R Tw[4];
  thermal_weights(Mf, s0.U, Acc.hu2, Tw);
  const R theta = R(0.5) * e.r - s0.V * e.v - s0.W * e.w;
  const R y1 = Tw[0] + Mf[0] * theta;
  const R y2 = thermal(T, s0.U, s0.V, s0.W, Acc.hu2);
  const R y3 = thermal_apsi(A, qA, Mf, Tw, theta, s0.V, s0.W);
  const R wn = ((Acc.wn + rn[0] * y1) + rn[1] * y2) + rn[2] * y3;
  const R wd = ((Acc.wd + rd[0] * y1) + rd[1] * y2) + rd[2] * y3;
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
