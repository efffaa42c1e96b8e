/*
 * HGKS oracle: a plain, slow FP64 CPU implementation of the high-order
 * gas-kinetic scheme's hot path (arXiv 2207.01173, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant table with the HIP
 * path.
 *
 * What it computes, in the paper's order:
 *   - ghost cells (periodic wrap; isothermal no-slip wall by mirroring),
 *   - the CFL time step,
 *   - per cell interface: fifth-order WENO-Z reconstruction of the conserved
 *     variables (normal sweep on cell averages, then two tangential sweeps to
 *     the 2x2 Gauss points of the face, dimension by dimension, Sec. 2 last
 *     paragraph), values and slopes,
 *   - per Gauss point: the equilibrium state g0 from the compatibility
 *     condition, micro-slopes a and A for the left, right and equilibrium
 *     states, the collision time tau = mu/p, and the time integral of the
 *     moments of the second-order distribution function, Eq. (flux),
 *   - the Gauss sum over the face, the linear-in-time flux F^n and dF^n/dt
 *     from the integrals over [0,dt] and [0,dt/2], Eq. (expansion-1),
 *   - L and dL/dt per cell, Eq. (semi2), and the two-stage fourth-order
 *     update, Eq. (two-stage),
 *   - statistics: volume-averaged kinetic energy and total viscous
 *     dissipation (Sec. 4.1).
 *
 * Readings of points the paper leaves open are listed where they are used and
 * in the design notes (R1..R21).  Parity unpinned: multi-step TGV and channel
 * runs (no numbers in the paper); they rest on the unit pins plus agreement.
 *
 * The per-face numerics are templates over the scalar type so that a counting
 * scalar can tally the floating-point operations of one face; the normal
 * build instantiates them with double only.
 *
 * Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace hgo {

/* ------------------------------------------------------------------------ */
/* Operation-counting scalar (only used by hgo_count_face_flops)            */
/* ------------------------------------------------------------------------ */
struct OpCount {
  long long add = 0, mul = 0, div = 0, sqrt = 0, exp = 0, erfc = 0, pow = 0;
};
static OpCount g_ops;

struct Counted {
  double v;
  Counted(double x = 0.0) : v(x) {}
};
inline Counted operator+(Counted a, Counted b) { g_ops.add++; return a.v + b.v; }
inline Counted operator-(Counted a, Counted b) { g_ops.add++; return a.v - b.v; }
inline Counted operator*(Counted a, Counted b) { g_ops.mul++; return a.v * b.v; }
inline Counted operator/(Counted a, Counted b) { g_ops.div++; return a.v / b.v; }
inline Counted operator-(Counted a) { return -a.v; }
inline Counted& operator+=(Counted& a, Counted b) { a = a + b; return a; }
inline Counted& operator-=(Counted& a, Counted b) { a = a - b; return a; }
inline Counted& operator*=(Counted& a, Counted b) { a = a * b; return a; }
inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
inline bool operator==(Counted a, Counted b) { return a.v == b.v; }
inline Counted sqrt(Counted a) { g_ops.sqrt++; return std::sqrt(a.v); }
inline Counted exp(Counted a) { g_ops.exp++; return std::exp(a.v); }
inline Counted erfc(Counted a) { g_ops.erfc++; return std::erfc(a.v); }
inline Counted pow(Counted a, Counted b) { g_ops.pow++; return std::pow(a.v, b.v); }
inline Counted fabs(Counted a) { return std::fabs(a.v); }

using std::erfc;
using std::exp;
using std::fabs;
using std::pow;
using std::sqrt;

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Gas parameters                                                          */
/* ------------------------------------------------------------------------ */
template <class R> struct Gas {
  R gamma;   // specific heat ratio
  R K;       // internal degrees of freedom, K = (5 - 3 gamma)/(gamma - 1)  (Sec. 2)
  R mu_ref;  // mu = mu_ref * (T/T_ref)^mu_exp, T = p/rho  (Sec. 4.2 power law)
  R T_ref;
  R mu_exp;
  R Pr;      // Prandtl number
};

/* Macroscopic state of a Maxwellian: density, velocity, lambda = rho/(2p). */
template <class R> struct State {
  R rho, U, V, W, lam;
};

template <class R> State<R> primitive(const R q[5], R gamma) {
  State<R> s;
  s.rho = q[0];
  s.U = q[1] / q[0];
  s.V = q[2] / q[0];
  s.W = q[3] / q[0];
  R p = (gamma - 1.0) * (q[4] - 0.5 * (q[1] * s.U + q[2] * s.V + q[3] * s.W));
  s.lam = 0.5 * q[0] / p;
  return s;
}

/* ------------------------------------------------------------------------ */
/* Moments of the Maxwellian, normalised by density (Sec. 2, <...>)         */
/* ------------------------------------------------------------------------ */
/* u[n] = <u^n>, v[n], w[n] for n = 0..6, xi[e] = <xi^(2e)> for e = 0..2.
 * For a half-space table only u[] is restricted (u > 0 or u < 0).          */
template <class R> struct Moments {
  R u[7], v[7], w[7], xi[3];
};

/* Gaussian recurrence <c^(n+2)> = mean <c^(n+1)> + (n+1)/(2 lam) <c^n>.
 * Holds on the full line and on either half line (the boundary term at
 * c = 0 vanishes for n + 1 >= 1).                                            */
template <class R> void gauss_chain(R mean, R lam, R m0, R m1, R out[7]) {
  out[0] = m0;
  out[1] = m1;
  for (int n = 0; n < 5; ++n) out[n + 2] = mean * out[n + 1] + (n + 1.0) / (2.0 * lam) * out[n];
}

/* side: 0 = full space, +1 = u > 0, -1 = u < 0 (half-space in u only). */
template <class R> void maxwell_moments(const State<R>& s, R K, int side, Moments<R>& m) {
  if (side == 0) {
    gauss_chain(s.U, s.lam, R(1.0), s.U, m.u);
  } else {
    R sl = sqrt(s.lam);
    R e = exp(-s.lam * s.U * s.U) / (2.0 * sqrt(PI * s.lam));
    R m0, m1;
    if (side > 0) {
      m0 = 0.5 * erfc(-sl * s.U);
      m1 = s.U * m0 + e;
    } else {
      m0 = 0.5 * erfc(sl * s.U);
      m1 = s.U * m0 - e;
    }
    gauss_chain(s.U, s.lam, m0, m1, m.u);
  }
  gauss_chain(s.V, s.lam, R(1.0), s.V, m.v);
  gauss_chain(s.W, s.lam, R(1.0), s.W, m.w);
  m.xi[0] = 1.0;
  m.xi[1] = K / (2.0 * s.lam);
  m.xi[2] = K * (K + 2.0) / (4.0 * s.lam * s.lam);
}

/* <u^a v^b w^c xi^(2e)> factorises into the four one-dimensional moments. */
template <class R> R mono(const Moments<R>& m, int a, int b, int c, int e) {
  return m.u[a] * m.v[b] * m.w[c] * m.xi[e];
}

/* <u^a v^b w^c (xi^2)^e psi>, psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2). */
template <class R> void mom_psi(const Moments<R>& m, int a, int b, int c, int e, R out[5]) {
  out[0] = mono(m, a, b, c, e);
  out[1] = mono(m, a + 1, b, c, e);
  out[2] = mono(m, a, b + 1, c, e);
  out[3] = mono(m, a, b, c + 1, e);
  out[4] = 0.5 * (mono(m, a + 2, b, c, e) + mono(m, a, b + 2, c, e) + mono(m, a, b, c + 2, e) +
                  mono(m, a, b, c, e + 1));
}

/* <(coef . psi) u^a v^b w^c psi>: expand coef . psi term by term. */
template <class R> void mom_apsi(const Moments<R>& m, const R coef[5], int a, int b, int c, R out[5]) {
  R t0[5], t1[5], t2[5], t3[5], s0[5], s1[5], s2[5], s3[5];
  mom_psi(m, a, b, c, 0, t0);
  mom_psi(m, a + 1, b, c, 0, t1);
  mom_psi(m, a, b + 1, c, 0, t2);
  mom_psi(m, a, b, c + 1, 0, t3);
  mom_psi(m, a + 2, b, c, 0, s0);
  mom_psi(m, a, b + 2, c, 0, s1);
  mom_psi(m, a, b, c + 2, 0, s2);
  mom_psi(m, a, b, c, 1, s3);
  for (int k = 0; k < 5; ++k)
    out[k] = coef[0] * t0[k] + coef[1] * t1[k] + coef[2] * t2[k] + coef[3] * t3[k] +
             coef[4] * 0.5 * (s0[k] + s1[k] + s2[k] + s3[k]);
}

/* ------------------------------------------------------------------------ */
/* Micro-slopes: solve <(a . psi) psi> = b for a, closed form of the 5x5     */
/* moment system (Sec. 2, <a^k_1> = dQ_k/dx etc., divided by density).       */
/* ------------------------------------------------------------------------ */
template <class R> void slope_solve(const State<R>& s, R K, const R b[5], R a[5]) {
  R q2 = s.U * s.U + s.V * s.V + s.W * s.W + (K + 3.0) / (2.0 * s.lam);
  R r2 = b[1] - s.U * b[0];
  R r3 = b[2] - s.V * b[0];
  R r4 = b[3] - s.W * b[0];
  R r5 = 2.0 * b[4] - q2 * b[0];
  a[4] = 4.0 * s.lam * s.lam / (K + 3.0) * (r5 - 2.0 * s.U * r2 - 2.0 * s.V * r3 - 2.0 * s.W * r4);
  a[3] = 2.0 * s.lam * r4 - s.W * a[4];
  a[2] = 2.0 * s.lam * r3 - s.V * a[4];
  a[1] = 2.0 * s.lam * r2 - s.U * a[4];
  a[0] = b[0] - s.U * a[1] - s.V * a[2] - s.W * a[3] - 0.5 * a[4] * q2;
}

/* Time slope A from <a_1 u + a_2 v + a_3 w + A> = 0 with full moments of the
 * same state: <A psi> = -sum_d <(a_d . psi) s_d psi>, s = (u, v, w).        */
template <class R> void time_slope(const State<R>& s, const Moments<R>& full, R K, const R a[3][5], R A[5]) {
  R t0[5], t1[5], t2[5], b[5];
  mom_apsi(full, a[0], 1, 0, 0, t0);
  mom_apsi(full, a[1], 0, 1, 0, t1);
  mom_apsi(full, a[2], 0, 0, 1, t2);
  for (int k = 0; k < 5; ++k) b[k] = -(t0[k] + t1[k] + t2[k]);
  slope_solve(s, K, b, A);
}

/* ------------------------------------------------------------------------ */
/* Collision time and time coefficients of Eq. (flux)                      */
/* ------------------------------------------------------------------------ */
/* tau = mu / p with p and T = p/rho from Q0 (Sec. 2, flow without discontinuities). */
template <class R> R collision_time(const State<R>& s0, const Gas<R>& g) {
  R p0 = 0.5 * s0.rho / s0.lam;
  R T0 = 0.5 / s0.lam;
  R mu = g.mu_ref;
  if (!(g.mu_exp == R(0.0))) mu = g.mu_ref * pow(T0 / g.T_ref, g.mu_exp);
  return mu / p0;
}

/* Integrals over [0, delta] of the time factors of Eq. (flux):
 * C1: 1 - e^{-t/tau}          C2: (t + tau) e^{-t/tau} - tau     C3: t - tau + tau e^{-t/tau}
 * C4: e^{-t/tau}              C5: -(t + tau) e^{-t/tau}          C6: -tau e^{-t/tau}
 * tau = 0 is the limit (Euler, g = g0 instantly).                           */
template <class R> void time_coefficients(R tau, R delta, R C[6]) {
  if (!(tau > R(0.0))) {
    C[0] = delta;
    C[1] = 0.0;
    C[2] = 0.5 * delta * delta;
    C[3] = 0.0;
    C[4] = 0.0;
    C[5] = 0.0;
    return;
  }
  R eta = exp(-delta / tau);
  C[0] = delta - tau * (1.0 - eta);
  C[1] = 2.0 * tau * tau * (1.0 - eta) - tau * delta * (1.0 + eta);
  C[2] = 0.5 * delta * delta - tau * delta + tau * tau * (1.0 - eta);
  C[3] = tau * (1.0 - eta);
  C[4] = tau * delta * eta - 2.0 * tau * tau * (1.0 - eta);
  C[5] = -tau * tau * (1.0 - eta);
}

/* ------------------------------------------------------------------------ */
/* Gauss-point flux (Sec. 2, Eq. (flux) and the moments of it)              */
/* ------------------------------------------------------------------------ */
/* Inputs, in the face's local frame (n, t1, t2); momentum components in the
 * same frame:
 *   ql, qr        reconstructed conserved variables left/right of the face
 *   dql[d], dqr[d] their derivatives along n, t1, t2 (physical units)
 *   dq0n          normal derivative of the equilibrium (R4)
 * Outputs: F(delta) = int_0^delta int u psi f dXi dt for delta = dt1, dt2,
 * with the Prandtl correction (R11) applied to the energy component.        */
template <class R>
void gp_flux(const R ql[5], const R qr[5], const R dql[3][5], const R dqr[3][5], const R dq0n[5],
             const Gas<R>& g, R dt1, R dt2, R F1[5], R F2[5]) {
  const R K = g.K;
  State<R> sl = primitive(ql, g.gamma);
  State<R> sr = primitive(qr, g.gamma);
  Moments<R> ml_full, ml_half, mr_full, mr_half;
  maxwell_moments(sl, K, 0, ml_full);
  maxwell_moments(sl, K, +1, ml_half);
  maxwell_moments(sr, K, 0, mr_full);
  maxwell_moments(sr, K, -1, mr_half);

  /* Equilibrium at the interface from the compatibility condition (R6):
   * Q0 = int_{u>0} psi g_l + int_{u<0} psi g_r.                              */
  R hl[5], hr[5], q0[5];
  mom_psi(ml_half, 0, 0, 0, 0, hl);
  mom_psi(mr_half, 0, 0, 0, 0, hr);
  for (int k = 0; k < 5; ++k) q0[k] = sl.rho * hl[k] + sr.rho * hr[k];
  State<R> s0 = primitive(q0, g.gamma);
  Moments<R> m0;
  maxwell_moments(s0, K, 0, m0);

  /* Spatial micro-slopes of the left and right states: <a psi> = dQ/rho. */
  R al[3][5], ar[3][5], b[5];
  for (int d = 0; d < 3; ++d) {
    for (int k = 0; k < 5; ++k) b[k] = dql[d][k] / sl.rho;
    slope_solve(sl, K, b, al[d]);
    for (int k = 0; k < 5; ++k) b[k] = dqr[d][k] / sr.rho;
    slope_solve(sr, K, b, ar[d]);
  }
  R Al[5], Ar[5];
  time_slope(sl, ml_full, K, al, Al);
  time_slope(sr, mr_full, K, ar, Ar);

  /* Equilibrium slopes: normal from the reconstruction (R4); tangential as
   * the exact derivative of the compatibility map (R7):
   * dQ0/dt = rho_l <(a^l_t . psi) psi>_{u>0} + rho_r <(a^r_t . psi) psi>_{u<0}. */
  R dq0[3][5];
  for (int k = 0; k < 5; ++k) dq0[0][k] = dq0n[k];
  for (int d = 1; d < 3; ++d) {
    R tl[5], tr[5];
    mom_apsi(ml_half, al[d], 0, 0, 0, tl);
    mom_apsi(mr_half, ar[d], 0, 0, 0, tr);
    for (int k = 0; k < 5; ++k) dq0[d][k] = sl.rho * tl[k] + sr.rho * tr[k];
  }
  R a0[3][5], A0[5];
  for (int d = 0; d < 3; ++d) {
    for (int k = 0; k < 5; ++k) b[k] = dq0[d][k] / s0.rho;
    slope_solve(s0, K, b, a0[d]);
  }
  time_slope(s0, m0, K, a0, A0);

  R tau = collision_time(s0, g);

  /* Moment vectors of the three groups of terms for each of g0, g_l, g_r:
   *   X1 = <u^x psi>, X2 = sum_d <u^x s_d (a_d . psi) psi>, X3 = <u^x (A . psi) psi>
   * with x = 1 for the flux F and x = 0 for the conserved-variable integral
   * W used by the Prandtl correction.                                         */
  R f0[3][5], fl[3][5], fr[3][5];  // x = 1
  R w0[3][5], wl[3][5], wr[3][5];  // x = 0
  const Moments<R>* tab[3] = {&m0, &ml_half, &mr_half};
  const R(*aa[3])[5] = {a0, al, ar};
  const R* AA[3] = {A0, Al, Ar};
  R(*fo[3])[5] = {f0, fl, fr};
  R(*wo[3])[5] = {w0, wl, wr};
  for (int side = 0; side < 3; ++side) {
    const Moments<R>& m = *tab[side];
    for (int x = 0; x <= 1; ++x) {
      R(*o)[5] = x ? fo[side] : wo[side];
      R t0[5], t1[5], t2[5];
      mom_psi(m, x, 0, 0, 0, o[0]);
      mom_apsi(m, aa[side][0], x + 1, 0, 0, t0);
      mom_apsi(m, aa[side][1], x, 1, 0, t1);
      mom_apsi(m, aa[side][2], x, 0, 1, t2);
      for (int k = 0; k < 5; ++k) o[1][k] = t0[k] + t1[k] + t2[k];
      mom_apsi(m, AA[side], x, 0, 0, o[2]);
    }
  }

  for (int which = 0; which < 2; ++which) {
    R delta = which == 0 ? dt1 : dt2;
    R* F = which == 0 ? F1 : F2;
    R C[6];
    time_coefficients(tau, delta, C);
    R Wt[5];
    for (int k = 0; k < 5; ++k) {
      F[k] = s0.rho * (C[0] * f0[0][k] + C[1] * f0[1][k] + C[2] * f0[2][k]) +
             sl.rho * (C[3] * fl[0][k] + C[4] * fl[1][k] + C[5] * fl[2][k]) +
             sr.rho * (C[3] * fr[0][k] + C[4] * fr[1][k] + C[5] * fr[2][k]);
      Wt[k] = s0.rho * (C[0] * w0[0][k] + C[1] * w0[1][k] + C[2] * w0[2][k]) +
              sl.rho * (C[3] * wl[0][k] + C[4] * wl[1][k] + C[5] * wl[2][k]) +
              sr.rho * (C[3] * wr[0][k] + C[4] * wr[1][k] + C[5] * wr[2][k]);
    }
    /* Prandtl correction (R11): heat flux of the time-integrated distribution
     * in the frame moving with the interface velocity U0,
     * q = int c_n (|c|^2 + xi^2)/2 f,  c = u - U0;  F_E += (1/Pr - 1) q.     */
    R U2 = s0.U * s0.U + s0.V * s0.V + s0.W * s0.W;
    R q = F[4] - (s0.U * F[1] + s0.V * F[2] + s0.W * F[3]) + 0.5 * U2 * F[0] -
          s0.U * (Wt[4] - (s0.U * Wt[1] + s0.V * Wt[2] + s0.W * Wt[3]) + 0.5 * U2 * Wt[0]);
    F[4] = F[4] + (1.0 / g.Pr - 1.0) * q;
  }
}

/* ------------------------------------------------------------------------ */
/* Fifth-order WENO-Z reconstruction (Sec. 2 last paragraph; R1-R5, R8)      */
/* ------------------------------------------------------------------------ */
/* Five consecutive cell averages v[0..4] centred at cells -2..2 (unit cell
 * width).  The three candidates are the quadratics through (v0,v1,v2),
 * (v1,v2,v3), (v2,v3,v4); each is evaluated at position s of the centre cell
 * (s in [-1/2, 1/2]).  Derivatives are per unit index.                      */
template <class R> void quad_candidates(const R v[5], R s, R val[3], R der[3]) {
  /* quadratic alpha + beta x + gamma x^2 with given averages over three unit cells */
  R gam[3], bet[3], alp[3];
  gam[0] = 0.5 * (v[0] - 2.0 * v[1] + v[2]);
  bet[0] = 0.5 * (v[0] - 4.0 * v[1] + 3.0 * v[2]);
  alp[0] = v[2] - gam[0] / 12.0;
  gam[1] = 0.5 * (v[1] - 2.0 * v[2] + v[3]);
  bet[1] = 0.5 * (v[3] - v[1]);
  alp[1] = v[2] - gam[1] / 12.0;
  gam[2] = 0.5 * (v[2] - 2.0 * v[3] + v[4]);
  bet[2] = 0.5 * (-3.0 * v[2] + 4.0 * v[3] - v[4]);
  alp[2] = v[2] - gam[2] / 12.0;
  for (int k = 0; k < 3; ++k) {
    val[k] = alp[k] + bet[k] * s + gam[k] * s * s;
    der[k] = bet[k] + 2.0 * gam[k] * s;
  }
}

/* Jiang-Shu smoothness indicators of the three candidates. */
template <class R> void smoothness(const R v[5], R beta[3]) {
  R d0 = v[0] - 2.0 * v[1] + v[2], e0 = v[0] - 4.0 * v[1] + 3.0 * v[2];
  R d1 = v[1] - 2.0 * v[2] + v[3], e1 = v[1] - v[3];
  R d2 = v[2] - 2.0 * v[3] + v[4], e2 = 3.0 * v[2] - 4.0 * v[3] + v[4];
  beta[0] = 13.0 / 12.0 * d0 * d0 + 0.25 * e0 * e0;
  beta[1] = 13.0 / 12.0 * d1 * d1 + 0.25 * e1 * e1;
  beta[2] = 13.0 / 12.0 * d2 * d2 + 0.25 * e2 * e2;
}

static const double WENO_EPS = 1e-20;  // R1

/* WENO-Z weights (Borges et al.), exponent 1: alpha_k = d_k (1 + tau5/(beta_k + eps)). */
template <class R> void wenoz_weights(const R beta[3], const R d[3], R w[3]) {
  R tau5 = fabs(beta[0] - beta[2]);
  R a0 = d[0] * (1.0 + tau5 / (beta[0] + WENO_EPS));
  R a1 = d[1] * (1.0 + tau5 / (beta[1] + WENO_EPS));
  R a2 = d[2] * (1.0 + tau5 / (beta[2] + WENO_EPS));
  R sum = a0 + a1 + a2;
  w[0] = a0 / sum;
  w[1] = a1 / sum;
  w[2] = a2 / sum;
}

/* Linear weights reproducing the quartic through the five averages:
 * at s = +1/2: (1/10, 3/5, 3/10); at s = +-sqrt(3)/6 (Gauss points):
 * (7/36 -+ sqrt3/1080, 11/18, 7/36 +- sqrt3/1080).                          */
template <class R> void linear_weights(int where, R d[3]) {
  /* where: 0 -> s = +1/2, 1 -> s = -sqrt3/6, 2 -> s = +sqrt3/6 */
  const double r3 = std::sqrt(3.0);
  if (where == 0) {
    d[0] = 0.1; d[1] = 0.6; d[2] = 0.3;
  } else if (where == 1) {
    d[0] = 7.0 / 36.0 + r3 / 1080.0; d[1] = 11.0 / 18.0; d[2] = 7.0 / 36.0 - r3 / 1080.0;
  } else {
    d[0] = 7.0 / 36.0 - r3 / 1080.0; d[1] = 11.0 / 18.0; d[2] = 7.0 / 36.0 + r3 / 1080.0;
  }
}

static double s_of(int where) {
  return where == 0 ? 0.5 : (where == 1 ? -std::sqrt(3.0) / 6.0 : std::sqrt(3.0) / 6.0);
}

/* Linear weights for the derivative at the Gauss points: the combination of
 * the three candidate derivatives that equals the derivative of the quartic
 * through the five averages, (11/36 -+ 5 sqrt3/36, 7/18, 11/36 +- 5 sqrt3/36)
 * at s = +-sqrt3/6.  At s = 1/2 no such combination exists (two candidates
 * share one derivative there), so the face uses the value weights (R3).      */
template <class R> void derivative_linear_weights(int where, R d[3]) {
  const double r3 = std::sqrt(3.0);
  if (where == 0) {
    linear_weights(0, d);
  } else if (where == 1) {
    d[0] = 11.0 / 36.0 + 5.0 * r3 / 36.0; d[1] = 7.0 / 18.0; d[2] = 11.0 / 36.0 - 5.0 * r3 / 36.0;
  } else {
    d[0] = 11.0 / 36.0 - 5.0 * r3 / 36.0; d[1] = 7.0 / 18.0; d[2] = 11.0 / 36.0 + 5.0 * r3 / 36.0;
  }
}

/* WENO-Z value at 'where'. */
template <class R> R wenoz_value(const R v[5], int where) {
  R beta[3], d[3], w[3], pv[3], pd[3];
  smoothness(v, beta);
  linear_weights(where, d);
  wenoz_weights(beta, d, w);
  quad_candidates(v, R(s_of(where)), pv, pd);
  return w[0] * pv[0] + w[1] * pv[1] + w[2] * pv[2];
}

/* WENO-Z value and derivative at 'where'.  Both use the same smoothness
 * indicators; the derivative uses the derivative linear weights (R3).        */
template <class R> void wenoz(const R v[5], int where, R& val, R& der) {
  R beta[3], d[3], w[3], pv[3], pd[3];
  smoothness(v, beta);
  linear_weights(where, d);
  wenoz_weights(beta, d, w);
  quad_candidates(v, R(s_of(where)), pv, pd);
  val = w[0] * pv[0] + w[1] * pv[1] + w[2] * pv[2];
  if (where != 0) {
    derivative_linear_weights(where, d);
    wenoz_weights(beta, d, w);
  }
  der = w[0] * pd[0] + w[1] * pd[1] + w[2] * pd[2];
}

/* Linear-weight (fifth-order, non-oscillatory-free) value at 'where'. */
template <class R> R linear_value(const R v[5], int where) {
  R d[3], pv[3], pd[3];
  linear_weights(where, d);
  quad_candidates(v, R(s_of(where)), pv, pd);
  return d[0] * pv[0] + d[1] * pv[1] + d[2] * pv[2];
}

/* Normal sweep at face i+1/2 from six cell averages c[0..5] = Q_{i-2..i+3}
 * of one component.  Outputs (per unit index): left and right values and
 * normal derivatives, and the equilibrium normal slope (R4): the derivative
 * at the face of the quartic through four cell averages and the face value,
 * (Q_{i-1} - 15 Q_i + 15 Q_{i+1} - Q_{i+2}) / 12.                           */
template <class R> void normal_sweep(const R c[6], R& ql, R& qr, R& dl, R& dr, R& d0) {
  R vl[5] = {c[0], c[1], c[2], c[3], c[4]};
  wenoz(vl, 0, ql, dl);
  R vr[5] = {c[5], c[4], c[3], c[2], c[1]};  // mirror image: right state
  R dmr;
  wenoz(vr, 0, qr, dmr);
  dr = -dmr;
  d0 = (c[1] - 15.0 * c[2] + 15.0 * c[3] - c[4]) / 12.0;
}

/* ------------------------------------------------------------------------ */
/* Per-face pipeline: normal sweep results -> two tangential sweeps -> four  */
/* Gauss points -> flux.                                                      */
/* ------------------------------------------------------------------------ */
/* Quantities carried per face after the normal sweep, 5 components each. */
enum { N_QL = 0, N_QR, N_DLN, N_DRN, N_D0, N_COUNT };  // 25 values
/* After the first tangential sweep (per Gauss point along t1). */
enum { T_QL = 0, T_QR, T_DLN, T_DRN, T_D0, T_DLT1, T_DRT1, T_COUNT };  // 35 values

/* First tangential sweep from the normal-sweep results of five faces along t1. */
template <class R> void tangential_sweep_1(const R in[5][N_COUNT][5], int where, R out[T_COUNT][5]) {
  for (int k = 0; k < 5; ++k) {
    R v[5];
    for (int j = 0; j < 5; ++j) v[j] = in[j][N_QL][k];
    wenoz(v, where, out[T_QL][k], out[T_DLT1][k]);
    for (int j = 0; j < 5; ++j) v[j] = in[j][N_QR][k];
    wenoz(v, where, out[T_QR][k], out[T_DRT1][k]);
    for (int j = 0; j < 5; ++j) v[j] = in[j][N_DLN][k];
    out[T_DLN][k] = wenoz_value(v, where);
    for (int j = 0; j < 5; ++j) v[j] = in[j][N_DRN][k];
    out[T_DRN][k] = wenoz_value(v, where);
    for (int j = 0; j < 5; ++j) v[j] = in[j][N_D0][k];
    out[T_D0][k] = linear_value(v, where);
  }
}

/* Gauss-point inputs after the second tangential sweep. */
template <class R> struct GPInput {
  R ql[5], qr[5], dql[3][5], dqr[3][5], dq0n[5];  // derivatives per unit index
};

template <class R> void tangential_sweep_2(const R in[5][T_COUNT][5], int where, GPInput<R>& o) {
  for (int k = 0; k < 5; ++k) {
    R v[5];
    for (int j = 0; j < 5; ++j) v[j] = in[j][T_QL][k];
    wenoz(v, where, o.ql[k], o.dql[2][k]);
    for (int j = 0; j < 5; ++j) v[j] = in[j][T_QR][k];
    wenoz(v, where, o.qr[k], o.dqr[2][k]);
    for (int j = 0; j < 5; ++j) v[j] = in[j][T_DLN][k];
    o.dql[0][k] = wenoz_value(v, where);
    for (int j = 0; j < 5; ++j) v[j] = in[j][T_DRN][k];
    o.dqr[0][k] = wenoz_value(v, where);
    for (int j = 0; j < 5; ++j) v[j] = in[j][T_DLT1][k];
    o.dql[1][k] = wenoz_value(v, where);
    for (int j = 0; j < 5; ++j) v[j] = in[j][T_DRT1][k];
    o.dqr[1][k] = wenoz_value(v, where);
    for (int j = 0; j < 5; ++j) v[j] = in[j][T_D0][k];
    o.dq0n[k] = linear_value(v, where);
  }
}

/* One Gauss point: scale index derivatives to physical ones, then flux. */
template <class R>
void gp_flux_scaled(const GPInput<R>& in, R sn, R st1, R st2, const Gas<R>& g, R dt, R F1[5], R F2[5]) {
  R dql[3][5], dqr[3][5], dq0n[5];
  const R sc[3] = {sn, st1, st2};
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < 5; ++k) {
      dql[d][k] = in.dql[d][k] * sc[d];
      dqr[d][k] = in.dqr[d][k] * sc[d];
    }
  for (int k = 0; k < 5; ++k) dq0n[k] = in.dq0n[k] * sn;
  gp_flux(in.ql, in.qr, dql, dqr, dq0n, g, dt, R(0.5) * dt, F1, F2);
}

/* ------------------------------------------------------------------------ */
/* Grid, ghost cells, metrics                                               */
/* ------------------------------------------------------------------------ */
struct Config {
  int32_t n[3];
  double lo[3], hi[3];
  int32_t bc[3];       // 0 periodic, 1 isothermal no-slip wall (axis 1 only)
  double y_stretch;    // tanh parameter b of axis 1; 0 => uniform
  double gamma, prandtl;
  double mu_ref, T_ref, mu_exp;
  double T_wall;
  double body_force[3];
  double cfl;
  int32_t flags;       // bit 0: constant streamwise mass flux (force from a controller, R24)
};

static const int G = 3;  // ghost layers

struct Grid {
  Config c;
  int n[3], p[3];                  // interior and padded sizes
  std::vector<double> h[3];        // cell widths
  std::vector<double> xc[3];       // cell-centre coordinates
  std::vector<double> dface[3];    // d(index)/dx at faces 0..n
  std::vector<double> dgp[3];      // d(index)/dx at Gauss points (2 per cell: s = -sqrt3/6, +sqrt3/6)
};

/* Coordinate map of axis d: x(xi), xi in [0, n] the continuous index.
 * Uniform: x = lo + xi (hi - lo)/n.  Stretched (axis 1, Sec. 4.2):
 * x = lo + (hi - lo) (1 + tanh(b (2 xi/n - 1)) / tanh b) / 2.                */
static double coord(const Config& c, int d, double xi) {
  double L = c.hi[d] - c.lo[d];
  if (d == 1 && c.y_stretch > 0.0) {
    double b = c.y_stretch;
    return c.lo[d] + 0.5 * L * (1.0 + std::tanh(b * (2.0 * xi / c.n[d] - 1.0)) / std::tanh(b));
  }
  return c.lo[d] + xi * L / c.n[d];
}
static double dcoord(const Config& c, int d, double xi) {  // dx/dxi
  double L = c.hi[d] - c.lo[d];
  if (d == 1 && c.y_stretch > 0.0) {
    double b = c.y_stretch;
    double ch = std::cosh(b * (2.0 * xi / c.n[d] - 1.0));
    return L * b / (c.n[d] * std::tanh(b) * ch * ch);
  }
  return L / c.n[d];
}

static void build_grid(const Config& c, Grid& g) {
  g.c = c;
  const double r3 = std::sqrt(3.0) / 6.0;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = c.n[d];
    g.p[d] = c.n[d] + 2 * G;
    g.h[d].resize(c.n[d]);
    g.xc[d].resize(c.n[d]);
    g.dface[d].resize(c.n[d] + 1);
    g.dgp[d].resize(2 * c.n[d]);
    for (int i = 0; i < c.n[d]; ++i) {
      g.h[d][i] = coord(c, d, i + 1.0) - coord(c, d, double(i));
      g.xc[d][i] = coord(c, d, i + 0.5);
      g.dgp[d][2 * i] = 1.0 / dcoord(c, d, i + 0.5 - r3);
      g.dgp[d][2 * i + 1] = 1.0 / dcoord(c, d, i + 0.5 + r3);
    }
    for (int f = 0; f <= c.n[d]; ++f) g.dface[d][f] = 1.0 / dcoord(c, d, double(f));
    if (!(d == 1 && c.y_stretch > 0.0)) {
      /* uniform axis: exact constants, so that every face sees identical scales */
      double h = (c.hi[d] - c.lo[d]) / c.n[d];
      for (int i = 0; i < c.n[d]; ++i) { g.h[d][i] = h; g.dgp[d][2 * i] = g.dgp[d][2 * i + 1] = 1.0 / h; }
      for (int f = 0; f <= c.n[d]; ++f) g.dface[d][f] = 1.0 / h;
    }
  }
}

/* Padded AoS array: pad[((k * py + j) * px + i) * 5 + comp]. */
static inline size_t pidx(const Grid& g, int i, int j, int k) {
  return ((size_t)(k + G) * g.p[1] + (j + G)) * g.p[0] + (i + G);
}
/* Caller layout: SoA [5][nz][ny][nx]. */
static inline size_t sidx(const Grid& g, int c, int i, int j, int k) {
  return (((size_t)c * g.n[2] + k) * g.n[1] + j) * g.n[0] + i;
}

/* Fill the padded array: interior copy, periodic wrap, wall mirror (R17):
 * ghost layer l mirrors interior layer l, velocity reversed, same pressure,
 * temperature 2 T_w - T_m (not below 0.1 T_w), density p / T.               */
static void fill_padded(const Grid& g, const double* q, std::vector<double>& pad) {
  pad.assign((size_t)g.p[0] * g.p[1] * g.p[2] * 5, 0.0);
  const double gm1 = g.c.gamma - 1.0;
#pragma omp parallel for schedule(static)
  for (int k = -G; k < g.n[2] + G; ++k)
    for (int j = -G; j < g.n[1] + G; ++j)
      for (int i = -G; i < g.n[0] + G; ++i) {
        int src[3] = {i, j, k};
        bool mirror = false;
        for (int d = 0; d < 3; ++d) {
          int N = g.n[d];
          if (src[d] >= 0 && src[d] < N) continue;
          if (g.c.bc[d] == 1) {
            mirror = true;
            src[d] = src[d] < 0 ? -src[d] - 1 : 2 * N - 1 - src[d];
          } else {
            src[d] = ((src[d] % N) + N) % N;
          }
        }
        double v[5];
        for (int c = 0; c < 5; ++c) v[c] = q[sidx(g, c, src[0], src[1], src[2])];
        if (mirror) {
          double rho = v[0];
          double U = v[1] / rho, V = v[2] / rho, W = v[3] / rho;
          double p = gm1 * (v[4] - 0.5 * rho * (U * U + V * V + W * W));
          double Tm = p / rho;
          double Tg = std::max(2.0 * g.c.T_wall - Tm, 0.1 * g.c.T_wall);
          double rg = p / Tg;
          v[0] = rg;
          v[1] = -rg * U;
          v[2] = -rg * V;
          v[3] = -rg * W;
          v[4] = p / gm1 + 0.5 * rg * (U * U + V * V + W * W);
        }
        double* o = &pad[pidx(g, i, j, k) * 5];
        for (int c = 0; c < 5; ++c) o[c] = v[c];
      }
}

/* Cyclic local frame of direction d: (n, t1, t2) = (x,y,z), (y,z,x), (z,x,y). */
static inline void frame_to_ijk(int d, int n, int t1, int t2, int& i, int& j, int& k) {
  if (d == 0) { i = n; j = t1; k = t2; }
  else if (d == 1) { j = n; k = t1; i = t2; }
  else { k = n; i = t1; j = t2; }
}
/* Conserved variables of a padded cell in the local frame of direction d. */
static inline void local_q(const Grid& g, const std::vector<double>& pad, int d, int n, int t1, int t2,
                           double out[5]) {
  int i, j, k;
  frame_to_ijk(d, n, t1, t2, i, j, k);
  const double* v = &pad[pidx(g, i, j, k) * 5];
  out[0] = v[0];
  out[1] = v[1 + d];
  out[2] = v[1 + (d + 1) % 3];
  out[3] = v[1 + (d + 2) % 3];
  out[4] = v[4];
}

static Gas<double> gas_of(const Config& c) {
  Gas<double> g;
  g.gamma = c.gamma;
  g.K = (5.0 - 3.0 * c.gamma) / (c.gamma - 1.0);
  g.mu_ref = c.mu_ref;
  g.T_ref = c.T_ref;
  g.mu_exp = c.mu_exp;
  g.Pr = c.prandtl;
  return g;
}

/* 2x2 Gauss quadrature (weights 1/4 of the face area) of the Gauss-point
 * integrals S1 = sum F(dt), S2 = sum F(dt/2); then F^n = (4 I(dt/2) - I(dt))/dt
 * and dF^n/dt = 4 (I(dt) - 2 I(dt/2))/dt^2 (Eq. (expansion-1)); momentum
 * rotated back from the local frame of direction d.  out[10]: F^n, dF^n/dt. */
static void face_assembly(const double S1[5], const double S2[5], double area, double dt, int d, double out[10]) {
  const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
  double Fn[5], dF[5];
  for (int k = 0; k < 5; ++k) {
    double I1 = 0.25 * area * S1[k];  // integral over [0, dt]
    double I2 = 0.25 * area * S2[k];  // integral over [0, dt/2]
    Fn[k] = (4.0 * I2 - I1) / dt;
    dF[k] = 4.0 * (I1 - 2.0 * I2) / (dt * dt);
  }
  const int gc[5] = {0, 1 + d, 1 + d1, 1 + d2, 4};
  for (int k = 0; k < 5; ++k) {
    out[gc[k]] = Fn[k];
    out[5 + gc[k]] = dF[k];
  }
}

/* Face fluxes of direction d for the whole grid.
 * Output fl[(f * N1 + a) * N2 + b][10]: F^n (5) and dF^n/dt (5), integrated over
 * the face, momentum in the global frame.  f = 0..n_d (face between cells f-1, f). */
static void direction_fluxes(const Grid& g, const std::vector<double>& pad, int d, double dt,
                             std::vector<double>& fl) {
  const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
  const int Nn = g.n[d], N1 = g.n[d1], N2 = g.n[d2];
  const Gas<double> gas = gas_of(g.c);
  fl.assign((size_t)(Nn + 1) * N1 * N2 * 10, 0.0);
  const int P1 = N1 + 4, P2 = N2 + 4;
#pragma omp parallel
  {
    std::vector<double> A((size_t)P1 * P2 * N_COUNT * 5);
    std::vector<double> B((size_t)N1 * P2 * 2 * T_COUNT * 5);
#pragma omp for schedule(dynamic)
    for (int f = 0; f <= Nn; ++f) {
      /* normal sweep on faces (f, a, b), a in [-2, N1+2), b in [-2, N2+2) */
      for (int a = -2; a < N1 + 2; ++a)
        for (int b = -2; b < N2 + 2; ++b) {
          double cells[6][5];
          for (int m = 0; m < 6; ++m) local_q(g, pad, d, f - 3 + m, a, b, cells[m]);
          double* o = &A[(((size_t)(a + 2) * P2 + (b + 2)) * N_COUNT) * 5];
          for (int k = 0; k < 5; ++k) {
            double c6[6];
            for (int m = 0; m < 6; ++m) c6[m] = cells[m][k];
            normal_sweep(c6, o[N_QL * 5 + k], o[N_QR * 5 + k], o[N_DLN * 5 + k], o[N_DRN * 5 + k],
                         o[N_D0 * 5 + k]);
          }
        }
      /* first tangential sweep along t1 to its two Gauss points */
      for (int a = 0; a < N1; ++a)
        for (int b = -2; b < N2 + 2; ++b) {
          double in[5][N_COUNT][5];
          for (int j = 0; j < 5; ++j)
            std::memcpy(in[j], &A[(((size_t)(a + j) * P2 + (b + 2)) * N_COUNT) * 5], sizeof(in[j]));
          for (int g1 = 0; g1 < 2; ++g1) {
            double(*o)[5] = reinterpret_cast<double(*)[5]>(&B[((((size_t)a * P2 + (b + 2)) * 2 + g1) * T_COUNT) * 5]);
            tangential_sweep_1(in, 1 + g1, o);
          }
        }
      /* second tangential sweep along t2, Gauss points, flux, face sum */
      for (int a = 0; a < N1; ++a)
        for (int b = 0; b < N2; ++b) {
          double S1[5] = {0, 0, 0, 0, 0}, S2[5] = {0, 0, 0, 0, 0};
          for (int g1 = 0; g1 < 2; ++g1) {
            double in[5][T_COUNT][5];
            for (int j = 0; j < 5; ++j)
              std::memcpy(in[j], &B[((((size_t)a * P2 + (b + j)) * 2 + g1) * T_COUNT) * 5], sizeof(in[j]));
            for (int g2 = 0; g2 < 2; ++g2) {
              GPInput<double> gp;
              tangential_sweep_2(in, 1 + g2, gp);
              double F1[5], F2[5];
              gp_flux_scaled(gp, g.dface[d][f], g.dgp[d1][2 * a + g1], g.dgp[d2][2 * b + g2], gas, dt, F1,
                             F2);
              for (int k = 0; k < 5; ++k) {
                S1[k] += F1[k];
                S2[k] += F2[k];
              }
            }
          }
          face_assembly(S1, S2, g.h[d1][a] * g.h[d2][b], dt, d, &fl[(((size_t)f * N1 + a) * N2 + b) * 10]);
        }
    }
  }
}

/* L and dL/dt of cell (i,j,k) from the integrated fluxes of its six faces
 * (Eq. (semi2)), with the body-force source (R19): S = (0, rho f, m . f),
 * dS/dt = (0, f L_rho, f . L_m).                                             */
static void cell_residual(const Grid& g, const double* q, int i, int j, int k, const double* fm[3],
                          const double* fp[3], double l[5], double dl[5]) {
  const double* f = g.c.body_force;
  double vol = g.h[0][i] * g.h[1][j] * g.h[2][k];
  for (int c = 0; c < 5; ++c) { l[c] = 0.0; dl[c] = 0.0; }
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 5; ++c) {
      l[c] -= (fp[d][c] - fm[d][c]) / vol;
      dl[c] -= (fp[d][5 + c] - fm[d][5 + c]) / vol;
    }
  double rho = q[sidx(g, 0, i, j, k)];
  double m[3] = {q[sidx(g, 1, i, j, k)], q[sidx(g, 2, i, j, k)], q[sidx(g, 3, i, j, k)]};
  double lrho = l[0];
  double lm[3];
  for (int a = 0; a < 3; ++a) {
    l[1 + a] += rho * f[a];
    lm[a] = l[1 + a];
  }
  l[4] += m[0] * f[0] + m[1] * f[1] + m[2] * f[2];
  for (int a = 0; a < 3; ++a) dl[1 + a] += f[a] * lrho;
  dl[4] += f[0] * lm[0] + f[1] * lm[1] + f[2] * lm[2];
}

/* L(Q) and dL/dt (Eq. (semi2) and its time derivative) with the body-force
 * source (R19): S = (0, rho f, rho U . f), dS/dt from the same cell's L.      */
static void residual(const Grid& g, const double* q, double dt, double* L, double* dL) {
  std::vector<double> pad;
  fill_padded(g, q, pad);
  std::vector<double> fl[3];
  for (int d = 0; d < 3; ++d) direction_fluxes(g, pad, d, dt, fl[d]);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        double l[5], dl[5];
        const double* fm[3];
        const double* fp[3];
        for (int d = 0; d < 3; ++d) {
          int d1 = (d + 1) % 3, d2 = (d + 2) % 3, ijk[3] = {i, j, k};
          size_t N1 = g.n[d1], N2 = g.n[d2];
          fm[d] = &fl[d][(((size_t)ijk[d] * N1 + ijk[d1]) * N2 + ijk[d2]) * 10];
          fp[d] = &fl[d][(((size_t)(ijk[d] + 1) * N1 + ijk[d1]) * N2 + ijk[d2]) * 10];
        }
        cell_residual(g, q, i, j, k, fm, fp, l, dl);
        for (int c = 0; c < 5; ++c) {
          L[sidx(g, c, i, j, k)] = l[c];
          dL[sidx(g, c, i, j, k)] = dl[c];
        }
      }
}

/* Integrated flux of the single face (f, a, b) of direction d, from scratch:
 * the same normal sweep, tangential sweeps, Gauss-point fluxes and assembly as
 * direction_fluxes, restricted to the 5x5 patch of faces this face needs.     */
static void single_face_flux(const Grid& g, const std::vector<double>& pad, int d, int f, int a, int b, double dt,
                             double out[10]) {
  const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
  const Gas<double> gas = gas_of(g.c);
  double A[5][5][N_COUNT][5];  // [t1 offset][t2 offset]
  for (int ja = 0; ja < 5; ++ja)
    for (int jb = 0; jb < 5; ++jb) {
      double cells[6][5];
      for (int m = 0; m < 6; ++m) local_q(g, pad, d, f - 3 + m, a - 2 + ja, b - 2 + jb, cells[m]);
      for (int k = 0; k < 5; ++k) {
        double c6[6];
        for (int m = 0; m < 6; ++m) c6[m] = cells[m][k];
        double* o = &A[ja][jb][0][0];
        normal_sweep(c6, o[N_QL * 5 + k], o[N_QR * 5 + k], o[N_DLN * 5 + k], o[N_DRN * 5 + k], o[N_D0 * 5 + k]);
      }
    }
  double Bt[5][2][T_COUNT][5];  // [t2 offset][g1]
  for (int jb = 0; jb < 5; ++jb) {
    double in[5][N_COUNT][5];
    for (int j = 0; j < 5; ++j) std::memcpy(in[j], A[j][jb], sizeof(in[j]));
    for (int g1 = 0; g1 < 2; ++g1) tangential_sweep_1(in, 1 + g1, Bt[jb][g1]);
  }
  double S1[5] = {0, 0, 0, 0, 0}, S2[5] = {0, 0, 0, 0, 0};
  for (int g1 = 0; g1 < 2; ++g1) {
    double in[5][T_COUNT][5];
    for (int j = 0; j < 5; ++j) std::memcpy(in[j], Bt[j][g1], sizeof(in[j]));
    for (int g2 = 0; g2 < 2; ++g2) {
      GPInput<double> gp;
      tangential_sweep_2(in, 1 + g2, gp);
      double F1[5], F2[5];
      gp_flux_scaled(gp, g.dface[d][f], g.dgp[d1][2 * a + g1], g.dgp[d2][2 * b + g2], gas, dt, F1, F2);
      for (int k = 0; k < 5; ++k) {
        S1[k] += F1[k];
        S2[k] += F2[k];
      }
    }
  }
  face_assembly(S1, S2, g.h[d1][a] * g.h[d2][b], dt, d, out);
}

/* L and dL/dt at a list of cells only (six single-face fluxes each). */
static void residual_at(const Grid& g, const double* q, double dt, int ncell, const int* ijk, double* L, double* dL) {
  std::vector<double> pad;
  fill_padded(g, q, pad);
#pragma omp parallel for schedule(dynamic)
  for (int c = 0; c < ncell; ++c) {
    const int i = ijk[3 * c], j = ijk[3 * c + 1], k = ijk[3 * c + 2];
    const int idx[3] = {i, j, k};
    double fmv[3][10], fpv[3][10];
    const double* fm[3];
    const double* fp[3];
    for (int d = 0; d < 3; ++d) {
      const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
      single_face_flux(g, pad, d, idx[d], idx[d1], idx[d2], dt, fmv[d]);
      single_face_flux(g, pad, d, idx[d] + 1, idx[d1], idx[d2], dt, fpv[d]);
      fm[d] = fmv[d];
      fp[d] = fpv[d];
    }
    cell_residual(g, q, i, j, k, fm, fp, &L[5 * c], &dL[5 * c]);
  }
}

/* CFL time step (R13): dt = CFL / max_cells max_d (|U_d| + c) / h_d. */
static double cfl_dt(const Grid& g, const double* q) {
  double smax = 0.0;
  const double gm = g.c.gamma;
#pragma omp parallel for reduction(max : smax) schedule(static)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        double rho = q[sidx(g, 0, i, j, k)];
        double U[3] = {q[sidx(g, 1, i, j, k)] / rho, q[sidx(g, 2, i, j, k)] / rho, q[sidx(g, 3, i, j, k)] / rho};
        double p = (gm - 1.0) * (q[sidx(g, 4, i, j, k)] - 0.5 * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
        double c = std::sqrt(gm * p / rho);
        double h[3] = {g.h[0][i], g.h[1][j], g.h[2][k]};
        for (int d = 0; d < 3; ++d) smax = std::max(smax, (std::fabs(U[d]) + c) / h[d]);
      }
  return g.c.cfl / smax;
}

/* One S2O4 step (Eq. (two-stage)); both stages use the windows [0, dt] and
 * [0, dt/2] measured from the start of the stage (R10).                     */
/* Stage 1 from Q^n, L(Q^n), dL/dt(Q^n): the intermediate state
 * Q* = Q^n + dt/2 L + dt^2/8 dL/dt and the part of Q^{n+1} known after it,
 * Q^n + dt L + dt^2/6 dL/dt.                                                */
static inline void s2o4_stage1(double qn, double L, double dL, double dt, double& qs, double& acc) {
  qs = qn + 0.5 * dt * L + 0.125 * dt * dt * dL;
  acc = qn + dt * L + dt * dt / 6.0 * dL;
}
/* Stage 2: Q^{n+1} = (Q^n + dt L + dt^2/6 dL/dt) + dt^2/3 dL/dt(Q*).          */
static inline double s2o4_stage2(double acc, double dLs, double dt) { return acc + dt * dt / 3.0 * dLs; }

static void s2o4_step(const Grid& g, double* q, double dt) {
  size_t N = (size_t)g.n[0] * g.n[1] * g.n[2] * 5;
  std::vector<double> L(N), dL(N), qs(N), acc(N);
  residual(g, q, dt, L.data(), dL.data());
  for (size_t m = 0; m < N; ++m) s2o4_stage1(q[m], L[m], dL[m], dt, qs[m], acc[m]);
  residual(g, qs.data(), dt, L.data(), dL.data());
  for (size_t m = 0; m < N; ++m) q[m] = s2o4_stage2(acc[m], dL[m], dt);
}

/* ------------------------------------------------------------------------ */
/* Statistics (Sec. 4.1): E_k and the total viscous dissipation              */
/* ------------------------------------------------------------------------ */
/* Velocity gradients: fourth-order central differences of U = m/rho at cell
 * centres (R20), taken in index space and scaled by d(index)/dx at the cell
 * centre, which on a uniform axis is 1/h and on the tanh-stretched y axis
 * the inverse of the map's derivative.  Neighbours beyond a periodic axis
 * wrap; beyond an isothermal no-slip wall they are the wall ghosts of R17,
 * whose velocity is the mirrored interior cell's, reversed.                  */
struct Stats {
  double Ek, eps_sol, eps_dil, eps_com;
  double total[5], max_abs[5], min_p, min_rho;
  int32_t nonfinite;
};

static void stats(const Grid& g, const double* q, double rho0, Stats& s) {
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const size_t N = (size_t)nx * ny * nz;
  std::vector<double> u(3 * N);
  double vol = 0.0, ek = 0.0, ens = 0.0, dil = 0.0;
  double tot[5] = {0, 0, 0, 0, 0}, mx[5] = {0, 0, 0, 0, 0};
  double minp = INFINITY, minr = INFINITY;
  int bad = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = ((size_t)k * ny + j) * nx + i;
        double v[5];
        for (int m = 0; m < 5; ++m) v[m] = q[sidx(g, m, i, j, k)];
        double dv = g.h[0][i] * g.h[1][j] * g.h[2][k];
        for (int m = 0; m < 3; ++m) u[m * N + c] = v[1 + m] / v[0];
        double ke = 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / v[0];
        double p = (g.c.gamma - 1.0) * (v[4] - ke);
        ek += ke * dv;
        vol += dv;
        for (int m = 0; m < 5; ++m) {
          tot[m] += v[m] * dv;
          mx[m] = std::max(mx[m], std::fabs(v[m]));
          if (!std::isfinite(v[m])) bad = 1;
        }
        minp = std::min(minp, p);
        minr = std::min(minr, v[0]);
      }
  std::vector<double> dcen[3];  // d(index)/dx at the cell centres
  for (int a = 0; a < 3; ++a) {
    dcen[a].resize(g.n[a]);
    for (int i = 0; i < g.n[a]; ++i) dcen[a][i] = 1.0 / dcoord(g.c, a, i + 0.5);
  }
  auto D = [&](int comp, int axis, int i, int j, int k) {
    auto at = [&](int o) {
      int ii = i, jj = j, kk = k;
      int* t = axis == 0 ? &ii : (axis == 1 ? &jj : &kk);
      const int n = g.n[axis];
      int m = *t + o;
      double sign = 1.0;
      if (m < 0 || m >= n) {
        if (g.c.bc[axis] == 1) {
          m = m < 0 ? -m - 1 : 2 * n - 1 - m;
          sign = -1.0;
        } else {
          m = (m % n + n) % n;
        }
      }
      *t = m;
      return sign * u[comp * N + ((size_t)kk * ny + jj) * nx + ii];
    };
    const int ia = axis == 0 ? i : (axis == 1 ? j : k);
    return (at(-2) - 8.0 * at(-1) + 8.0 * at(1) - at(2)) / 12.0 * dcen[axis][ia];
  };
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double gr[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) gr[a][b] = D(a, b, i, j, k);  // d U_a / d x_b
        double wx = gr[2][1] - gr[1][2], wy = gr[0][2] - gr[2][0], wz = gr[1][0] - gr[0][1];
        double div = gr[0][0] + gr[1][1] + gr[2][2];
        double dv = g.h[0][i] * g.h[1][j] * g.h[2][k];
        ens += (wx * wx + wy * wy + wz * wz) * dv;
        dil += div * div * dv;
      }
  s.Ek = ek / (rho0 * vol);
  s.eps_sol = g.c.mu_ref * ens / (rho0 * vol);
  s.eps_dil = 4.0 / 3.0 * g.c.mu_ref * dil / (rho0 * vol);
  s.eps_com = s.eps_sol + s.eps_dil;
  for (int m = 0; m < 5; ++m) { s.total[m] = tot[m]; s.max_abs[m] = mx[m]; }
  s.min_p = minp;
  s.min_rho = minr;
  s.nonfinite = bad;
}

}  // namespace hgo

/* ======================================================================== */
/* C interface for the tests (ctypes).                                      */
/* ======================================================================== */
using namespace hgo;

extern "C" {

typedef hgo::Config hgo_config;

/* Number of OpenMP threads the oracle will use (0: library default). */
void hgo_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int hgo_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* prim = (rho, U, V, W, lambda); side 0 full, +1 u>0, -1 u<0.
 * out: u[0..6], v[0..6], w[0..6], xi[0..2] = <xi^0>, <xi^2>, <xi^4> (24 doubles). */
void hgo_moments(const double prim[5], double K, int side, double out[24]) {
  State<double> s{prim[0], prim[1], prim[2], prim[3], prim[4]};
  Moments<double> m;
  maxwell_moments(s, K, side, m);
  for (int n = 0; n < 7; ++n) { out[n] = m.u[n]; out[7 + n] = m.v[n]; out[14 + n] = m.w[n]; }
  for (int e = 0; e < 3; ++e) out[21 + e] = m.xi[e];
}

/* <(coef . psi) u^a v^b w^c psi> for a state and side. */
void hgo_mom_apsi(const double prim[5], double K, int side, const double coef[5], int a, int b, int c,
                  double out[5]) {
  State<double> s{prim[0], prim[1], prim[2], prim[3], prim[4]};
  Moments<double> m;
  maxwell_moments(s, K, side, m);
  mom_apsi(m, coef, a, b, c, out);
}
void hgo_mom_psi(const double prim[5], double K, int side, int a, int b, int c, int e, double out[5]) {
  State<double> s{prim[0], prim[1], prim[2], prim[3], prim[4]};
  Moments<double> m;
  maxwell_moments(s, K, side, m);
  mom_psi(m, a, b, c, e, out);
}

void hgo_slope_solve(const double prim[5], double K, const double b[5], double a[5]) {
  State<double> s{prim[0], prim[1], prim[2], prim[3], prim[4]};
  slope_solve(s, K, b, a);
}

void hgo_time_slope(const double prim[5], double K, const double a[15], double A[5]) {
  State<double> s{prim[0], prim[1], prim[2], prim[3], prim[4]};
  Moments<double> m;
  maxwell_moments(s, K, 0, m);
  double aa[3][5];
  std::memcpy(aa, a, sizeof(aa));
  time_slope(s, m, K, aa, A);
}

void hgo_time_coefficients(double tau, double delta, double C[6]) { time_coefficients(tau, delta, C); }

/* Compatibility: Q0 from left/right conserved states. */
void hgo_q0(const double ql[5], const double qr[5], double gamma, double q0[5]) {
  double K = (5.0 - 3.0 * gamma) / (gamma - 1.0);
  State<double> sl = primitive(ql, gamma), sr = primitive(qr, gamma);
  Moments<double> a, b;
  maxwell_moments(sl, K, +1, a);
  maxwell_moments(sr, K, -1, b);
  double hl[5], hr[5];
  mom_psi(a, 0, 0, 0, 0, hl);
  mom_psi(b, 0, 0, 0, 0, hr);
  for (int k = 0; k < 5; ++k) q0[k] = sl.rho * hl[k] + sr.rho * hr[k];
}

/* Gauss-point flux: d[30] = dql (n,t1,t2) then dqr; gas[6] = gamma, mu_ref,
 * T_ref, mu_exp, Pr, unused.  Out F1 = F(dt1), F2 = F(dt2). */
void hgo_gp_flux(const double ql[5], const double qr[5], const double d[30], const double dq0n[5],
                 const double gas[6], double dt1, double dt2, double F1[5], double F2[5]) {
  Gas<double> g;
  g.gamma = gas[0];
  g.K = (5.0 - 3.0 * gas[0]) / (gas[0] - 1.0);
  g.mu_ref = gas[1];
  g.T_ref = gas[2];
  g.mu_exp = gas[3];
  g.Pr = gas[4];
  double dql[3][5], dqr[3][5];
  std::memcpy(dql, d, sizeof(dql));
  std::memcpy(dqr, d + 15, sizeof(dqr));
  gp_flux(ql, qr, dql, dqr, dq0n, g, dt1, dt2, F1, F2);
}

/* WENO pieces. where: 0 -> s = 1/2, 1 -> -sqrt3/6, 2 -> +sqrt3/6. */
void hgo_wenoz(const double v[5], int where, double out[2]) { wenoz(v, where, out[0], out[1]); }
double hgo_linear_value(const double v[5], int where) { return linear_value(v, where); }
void hgo_linear_weights(int where, double d[3]) { linear_weights(where, d); }
void hgo_candidates(const double v[5], double s, double val[3], double der[3]) { quad_candidates(v, s, val, der); }
/* WENO with the nonlinear weights replaced by the linear ones (for pins). */
void hgo_weno_linear(const double v[5], int where, double out[2]) {
  double d[3], pv[3], pd[3];
  linear_weights(where, d);
  quad_candidates(v, s_of(where), pv, pd);
  out[0] = d[0] * pv[0] + d[1] * pv[1] + d[2] * pv[2];
  derivative_linear_weights(where, d);
  out[1] = d[0] * pd[0] + d[1] * pd[1] + d[2] * pd[2];
}
void hgo_derivative_linear_weights(int where, double d[3]) { derivative_linear_weights(where, d); }
void hgo_normal_sweep(const double c[6], double out[5]) { normal_sweep(c, out[0], out[1], out[2], out[3], out[4]); }

/* Whole-grid operations.  q is SoA [5][nz][ny][nx]. */
void hgo_residual(const hgo_config* cfg, const double* q, double dt, double* L, double* dL) {
  Grid g;
  build_grid(*cfg, g);
  residual(g, q, dt, L, dL);
}
/* Integrated flux F^n, dF^n/dt (global momentum frame) of face (f, a, b) of
 * direction d: f the face index along d (face f between cells f-1 and f), a
 * and b the cell indices along d+1 and d+2. */
void hgo_face_flux(const hgo_config* cfg, const double* q, double dt, int d, int f, int a, int b, double out[10]) {
  Grid g;
  build_grid(*cfg, g);
  std::vector<double> pad;
  fill_padded(g, q, pad);
  single_face_flux(g, pad, d, f, a, b, dt, out);
}

/* L, dL/dt at ncell cells ijk[3 * c + (0,1,2)]; outputs L[5 * c + comp]. */
void hgo_residual_at(const hgo_config* cfg, const double* q, double dt, int ncell, const int* ijk, double* L,
                     double* dL) {
  Grid g;
  build_grid(*cfg, g);
  residual_at(g, q, dt, ncell, ijk, L, dL);
}
double hgo_cfl_dt(const hgo_config* cfg, const double* q) {
  Grid g;
  build_grid(*cfg, g);
  return cfl_dt(g, q);
}
/* Advance nsteps; dt_fixed <= 0 uses the CFL rule each step. Returns the last
 * dt.  With flags bit 0 the streamwise force follows the constant-mass-flux
 * controller (Sec. 4.2 fixes the force by a constant streamwise momentum flux;
 * the rule is reading R24): target m_t = volume mean of rho U of the initial
 * state, rho_b its mean density, and after each step with error e = m - m_t,
 * f <- f - (2 e^{n+1} - e^n) / (rho_b dt), the step that brings the error to
 * zero over the next step if the wall drag stays what the last step showed.
 * The force in effect after the last step is returned in *force_out.        */
double hgo_step_force(const hgo_config* cfg, double* q, int nsteps, double dt_fixed, double* force_out) {
  Grid g;
  build_grid(*cfg, g);
  const bool control = (cfg->flags & 1) != 0;
  // volume means of rho and rho U
  auto means = [&](double& rho_m, double& m_m) {
    double vs = 0.0, rs = 0.0, ms = 0.0;
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          double v = g.h[0][i] * g.h[1][j] * g.h[2][k];
          vs += v;
          rs += v * q[sidx(g, 0, i, j, k)];
          ms += v * q[sidx(g, 1, i, j, k)];
        }
    rho_m = rs / vs;
    m_m = ms / vs;
  };
  double rho_b = 0.0, m_t = 0.0;
  if (control) means(rho_b, m_t);
  double m_prev = m_t;
  double dt = dt_fixed;
  for (int s = 0; s < nsteps; ++s) {
    dt = dt_fixed > 0.0 ? dt_fixed : cfl_dt(g, q);
    s2o4_step(g, q, dt);
    if (control) {
      double r, m;
      means(r, m);
      g.c.body_force[0] -= (2.0 * (m - m_t) - (m_prev - m_t)) / (rho_b * dt);
      m_prev = m;
    }
  }
  if (force_out) *force_out = g.c.body_force[0];
  return dt;
}
double hgo_step(const hgo_config* cfg, double* q, int nsteps, double dt_fixed) {
  return hgo_step_force(cfg, q, nsteps, dt_fixed, nullptr);
}
/* The grid step's two stages (s2o4_stage1, s2o4_stage2) on a scalar linear
 * ODE q' = lam q, whose L = lam q and dL/dt = lam^2 q are exact (for the
 * amplification-polynomial pin): returns q^{n+1}.                            */
double hgo_s2o4_scalar(double q, double lam, double dt) {
  double qs, acc;
  s2o4_stage1(q, lam * q, lam * lam * q, dt, qs, acc);
  return s2o4_stage2(acc, lam * lam * qs, dt);
}
/* out: Ek, eps_sol, eps_dil, eps_com, total[5], max_abs[5], min_p, min_rho, nonfinite */
void hgo_stats(const hgo_config* cfg, const double* q, double rho0, double out[17]) {
  Grid g;
  build_grid(*cfg, g);
  Stats s;
  stats(g, q, rho0, s);
  out[0] = s.Ek; out[1] = s.eps_sol; out[2] = s.eps_dil; out[3] = s.eps_com;
  for (int m = 0; m < 5; ++m) { out[4 + m] = s.total[m]; out[9 + m] = s.max_abs[m]; }
  out[14] = s.min_p; out[15] = s.min_rho; out[16] = s.nonfinite;
}
/* Cell geometry for tests: widths h[axis][n] and centres. */
void hgo_geometry(const hgo_config* cfg, int axis, double* h, double* xc, double* dface, double* dgp) {
  Grid g;
  build_grid(*cfg, g);
  for (int i = 0; i < g.n[axis]; ++i) {
    h[i] = g.h[axis][i];
    xc[i] = g.xc[axis][i];
    dgp[2 * i] = g.dgp[axis][2 * i];
    dgp[2 * i + 1] = g.dgp[axis][2 * i + 1];
  }
  for (int f = 0; f <= g.n[axis]; ++f) dface[f] = g.dface[axis][f];
}

/* Floating-point operations of the method for one face of an interior,
 * uniform-grid interface with viscosity, counted on a representative state:
 * out[0] normal sweep per face, out[1] first tangential sweep per (face, GP
 * line), out[2] second tangential sweep per GP, out[3] flux per GP, out[4]
 * face assembly (Gauss sum, F and dF/dt), out[5..11] the per-GP-flux
 * breakdown add, mul, div, sqrt, exp, erfc, pow.                           */
void hgo_count_flops(double out[12]) {
  using C = Counted;
  /* a smooth, generic state: no zero data, so no branch is skipped */
  double cells[6][5];
  for (int m = 0; m < 6; ++m) {
    double x = 0.3 * m;
    double rho = 1.0 + 0.1 * std::sin(x), U = 0.3 + 0.05 * std::cos(x), V = 0.2 - 0.04 * x, W = -0.1 + 0.02 * x * x;
    double p = 2.0 + 0.1 * std::cos(2 * x);
    cells[m][0] = rho; cells[m][1] = rho * U; cells[m][2] = rho * V; cells[m][3] = rho * W;
    cells[m][4] = p / 0.4 + 0.5 * rho * (U * U + V * V + W * W);
  }
  auto total = [](const OpCount& o) {
    return (double)(o.add + o.mul + o.div + o.sqrt + o.exp + o.erfc + o.pow);
  };
  /* normal sweep: 5 components */
  g_ops = OpCount();
  for (int k = 0; k < 5; ++k) {
    C c6[6], a, b, cc, d, e;
    for (int m = 0; m < 6; ++m) c6[m] = cells[m][k];
    normal_sweep(c6, a, b, cc, d, e);
  }
  out[0] = total(g_ops);
  /* first tangential sweep for one Gauss point */
  g_ops = OpCount();
  {
    C in[5][N_COUNT][5], o[T_COUNT][5];
    for (int j = 0; j < 5; ++j)
      for (int q = 0; q < N_COUNT; ++q)
        for (int k = 0; k < 5; ++k) in[j][q][k] = cells[j][k] * (1.0 + 0.01 * q) + 0.001 * j * j;
    tangential_sweep_1(in, 1, o);
  }
  out[1] = total(g_ops);
  g_ops = OpCount();
  {
    C in[5][T_COUNT][5];
    GPInput<C> o;
    for (int j = 0; j < 5; ++j)
      for (int q = 0; q < T_COUNT; ++q)
        for (int k = 0; k < 5; ++k) in[j][q][k] = cells[j][k] * (1.0 + 0.01 * q) + 0.001 * j * j;
    tangential_sweep_2(in, 1, o);
  }
  out[2] = total(g_ops);
  /* flux at one Gauss point with scaling */
  g_ops = OpCount();
  {
    GPInput<C> in;
    for (int k = 0; k < 5; ++k) {
      in.ql[k] = cells[2][k];
      in.qr[k] = cells[3][k] * 1.001;
      in.dq0n[k] = 0.01 * (k + 1);
      for (int d = 0; d < 3; ++d) {
        in.dql[d][k] = 0.02 * (k + 1) * (d + 1);
        in.dqr[d][k] = 0.021 * (k + 1) * (d + 1);
      }
    }
    Gas<C> gas;
    gas.gamma = 1.4; gas.K = 2.0; gas.mu_ref = 1e-3; gas.T_ref = 1.0; gas.mu_exp = 0.0; gas.Pr = 0.72;
    C F1[5], F2[5];
    gp_flux_scaled(in, C(10.0), C(10.0), C(10.0), gas, C(1e-3), F1, F2);
  }
  out[3] = total(g_ops);
  out[5] = g_ops.add; out[6] = g_ops.mul; out[7] = g_ops.div; out[8] = g_ops.sqrt;
  out[9] = g_ops.exp; out[10] = g_ops.erfc; out[11] = g_ops.pow;
  /* face assembly: 4-point sums (2 x 15 adds), area, F and dF/dt (counted by hand:
   * per component 2 sums of 4 -> 6 adds; I1, I2: 2 mul each incl. area; F: 1 mul,
   * 1 add, 1 div; dF: 1 mul, 1 add, 1 mul, 1 mul, 1 div) */
  out[4] = 5.0 * (6 + 4 + 3 + 5) + 1;
}

}  // extern "C"
