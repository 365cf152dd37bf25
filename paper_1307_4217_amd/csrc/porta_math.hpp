// porta_math.hpp -- per-update arithmetic of the BESSER short-characteristics
// step (Stepan & Trujillo Bueno 2013, Sect. 3), written for gfx950 and usable
// from host code as well (the host build only serves unit tests of this file).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace porta {

// ---------------------------------------------------------------------------
// exp(-t) for t >= 0.  On the GPU the FP32 form maps to v_exp_f32.
// ---------------------------------------------------------------------------
__host__ __device__ inline float exp_neg(float t) {
#ifdef __HIP_DEVICE_COMPILE__
  return __expf(-t);
#else
  return std::exp(-t);
#endif
}
__host__ __device__ inline double exp_neg(double t) { return exp(-t); }

// Reciprocal: the FP32 form is the hardware v_rcp_f32 (1 ulp), the FP64 form
// an IEEE division.
__host__ __device__ inline float recip(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
__host__ __device__ inline double recip(double x) { return 1.0 / x; }

// ---------------------------------------------------------------------------
// Coefficients of Eq. fsbez (Sect. 3.3):
//   e = exp(-tau), psi'_M, psi'_O (linear K'I), omega_M, omega_O, omega_C
//   (quadratic Bezier source function with control point c_M).
// Below a threshold the closed forms cancel; a Taylor series about tau = 0 is
// used instead (Table 1 gives the FP64 thresholds 0.14 / 0.18 for the omegas).
// FP32 switches at tau = 1.2 (one series for all six, below); FP64 uses eight
// terms of each coefficient's own series below the paper's thresholds (0.1 for
// the psi').
// ---------------------------------------------------------------------------
template <class T>
struct Coefs {
  T e, psiM, psiO, omM, omO, omC;
  T em1;             // 1 - e to the relative precision of T, formed on request (EM1 of
                     // coefficients), for an update written as I_M - em1 I_M: e itself,
                     // rounded next to 1 in FP32, is off by up to 3e-8 for thin steps, a
                     // bias that a chain of thousands of steps would add up
  T pmt, omt, oct;   // psi'_M / tau, omega_M / tau, omega_C / tau (for the tau-derivatives)
};

// Horner evaluation of tau * sum_{n<NT} c_n tau^n.
template <class T, int NT>
__host__ __device__ inline T series(T tau, const T (&c)[NT]) {
  T acc = c[NT - 1];
#pragma unroll
  for (int n = NT - 2; n >= 0; --n) acc = acc * tau + c[n];
  return acc * tau;
}

// FP32 below tau = 1.2: all six from one series.  With the exponential remainders
//   E_n(t) = sum_k (-t)^k / (k + n)!,   E_n = 1/n! - t E_{n+1},   e = 1 - t E_1,
// the series of the coefficients regroup as
//   psi'_O = t E_2,   psi'_M = t (E_1 - E_2),   omega_O = 2 t E_3,
//   omega_M = t (E_1 - 2 E_2 + 2 E_3),   omega_C = t (2 E_2 - 4 E_3),
// (from 1/(n!(n+2)) = 1/(n+1)! - 1/(n+2)!, 1/(n!(n+3)) = 1/(n+1)! - 2/(n+2)! + 2/(n+3)!
// and 2/(n!(n+2)(n+3)) = 2/(n+2)! - 4/(n+3)!), so ten terms of E_3 and the downward
// recurrence (stable for t < 1.2) give every coefficient within 1e-6 relative.
template <bool EM1 = false>
__host__ __device__ inline Coefs<float> coefficients(float tau) {
  Coefs<float> c;
  if (tau < 1.2f) {
    const float kE3[10] = {1.0f / 6, -1.0f / 24, 1.0f / 120, -1.0f / 720, 1.0f / 5040,
                           -1.0f / 40320, 1.0f / 362880, -1.0f / 3628800, 1.0f / 39916800,
                           -1.0f / 479001600};
    float E3 = kE3[9];
#pragma unroll
    for (int n = 8; n >= 0; --n) E3 = E3 * tau + kE3[n];
    const float E2 = 0.5f - tau * E3;
    const float E1 = 1.0f - tau * E2;
    c.e = 1.0f - tau * E1;
    if constexpr (EM1) c.em1 = tau * E1;
    c.pmt = E1 - E2;
    c.omt = E1 + 2.0f * (E3 - E2);
    c.oct = 2.0f * E2 - 4.0f * E3;
    c.psiO = tau * E2;
    c.psiM = tau * c.pmt;
    c.omO = (2.0f * tau) * E3;
    c.omM = tau * c.omt;
    c.omC = tau * c.oct;
  } else {
    c.e = exp_neg(tau);
    if constexpr (EM1) c.em1 = 1.0f - c.e;
    const float it = recip(tau), it2 = it * it;
    const float g = c.e + tau - 1.0f;               // e + tau - 1
    c.psiO = g * it;
    c.psiM = (1.0f - c.e * (1.0f + tau)) * it;
    c.omM = (2.0f - c.e * (tau * tau + 2.0f * tau + 2.0f)) * it2;
    c.omO = 1.0f - 2.0f * g * it2;
    c.omC = 2.0f * (tau - 2.0f + c.e * (tau + 2.0f)) * it2;
    c.pmt = c.psiM * it;
    c.omt = c.omM * it;
    c.oct = c.omC * it;
  }
  return c;
}

template <bool EM1 = false>
__host__ __device__ inline Coefs<double> coefficients(double tau) {
  // eight terms, identical to the rows of Table 1 for the omegas
  const double kPM[8] = {1.0 / 2, -1.0 / 3, 1.0 / 8, -1.0 / 30, 1.0 / 144, -1.0 / 840,
                         1.0 / 5760, -1.0 / 45360};
  const double kPO[8] = {1.0 / 2, -1.0 / 6, 1.0 / 24, -1.0 / 120, 1.0 / 720, -1.0 / 5040,
                         1.0 / 40320, -1.0 / 362880};
  const double kOM[8] = {1.0 / 3, -1.0 / 4, 1.0 / 10, -1.0 / 36, 1.0 / 168, -1.0 / 960,
                         1.0 / 6480, -1.0 / 50400};
  const double kOO[8] = {1.0 / 3, -1.0 / 12, 1.0 / 60, -1.0 / 360, 1.0 / 2520, -1.0 / 20160,
                         1.0 / 181440, -1.0 / 1814400};
  const double kOC[8] = {1.0 / 3, -1.0 / 6, 1.0 / 20, -1.0 / 90, 1.0 / 504, -1.0 / 3360,
                         1.0 / 25920, -1.0 / 226800};
  Coefs<double> c;
  c.e = exp_neg(tau);
  if constexpr (EM1) c.em1 = 1.0 - c.e;   // FP64: the same bias is 1e-16 per step
  const double it = 1.0 / tau, it2 = it * it;
  if (tau < 0.1) {
    c.psiM = series(tau, kPM);
    c.psiO = series(tau, kPO);
  } else {
    c.psiM = (1.0 - c.e * (1.0 + tau)) * it;
    c.psiO = (c.e + tau - 1.0) * it;
  }
  if (tau < 0.14)
    c.omM = series(tau, kOM);
  else
    c.omM = (2.0 - c.e * (tau * tau + 2.0 * tau + 2.0)) * it2;
  if (tau < 0.18) {
    c.omO = series(tau, kOO);
    c.omC = series(tau, kOC);
  } else {
    c.omO = 1.0 - 2.0 * (c.e + tau - 1.0) * it2;
    c.omC = 2.0 * (tau - 2.0 + c.e * (tau + 2.0)) * it2;
  }
  c.pmt = c.psiM * it;
  c.omt = c.omM * it;
  c.oct = c.omC * it;
  return c;
}

// ---------------------------------------------------------------------------
// BESSER control point of the upwind interval (Sect. 3.2, steps 1-9), in the
// scale-free form with D_M = y_O - y_M, D_P = y_P - y_O and r = h_M / h_P:
//   parabolic c_M = y_O - (r^2 D_P + D_M) / (2 (1 + r)),
//   parabolic c_P = y_O + (r D_P + D_M / r) / (2 (1 + r)).
// Only the ratio of the optical paths enters, so c_M is the same for every
// frequency when all opacities share one profile.
// ---------------------------------------------------------------------------
__host__ __device__ inline double besser_cm(double yM, double yO, double yP, double r) {
  const double dM = yO - yM, dP = yP - yO;
  if (dM * dP <= 0.0) return yO;                       // extremum at O (step 2)
  const double inv = 0.5 / (1.0 + r);
  const double cM = yO - (r * r * dP + dM) * inv;      // steps 3-4
  if ((cM - yM) * (cM - yO) > 0.0) return yM;          // overshoot in MO (steps 5-6)
  const double cP = yO + (r * dP + dM / r) * inv;
  if ((cP - yO) * (cP - yP) > 0.0)                     // overshoot in OP (step 7)
    return yO - r * dP;                                // c_P = y_P; steps 8-9
  return cM;
}

// Control point of the parabola through M, O, P: steps 1, 3 and 4 without the
// monotonicity tests (the choice of the DELOPAR solver), in the same ratio form.
__host__ __device__ inline double parabolic_cm(double yM, double yO, double yP, double r) {
  const double dM = yO - yM, dP = yP - yO;
  return yO - (r * r * dP + dM) * (0.5 / (1.0 + r));
}

// The control point of either rule from one evaluation of steps 1, 3 and 4: the
// parabolic rule returns there, BESSER goes on with its tests (same result as
// besser_cm).
__host__ __device__ inline double control_cm(double yM, double yO, double yP, double r,
                                             bool parabolic) {
  const double dM = yO - yM, dP = yP - yO;
  const double inv = 0.5 / (1.0 + r);
  const double cM = yO - (r * r * dP + dM) * inv;
  if (parabolic) return cM;
  if (dM * dP <= 0.0) return yO;
  if ((cM - yM) * (cM - yO) > 0.0) return yM;
  const double cP = yO + (r * dP + dM / r) * inv;
  if ((cP - yO) * (cP - yP) > 0.0) return yO - r * dP;
  return cM;
}

// The same control point in the sweep precision, for interpolation on the grid.
template <class T>
__host__ __device__ inline T besser_cm_t(T yM, T yO, T yP, T r) {
  const T dM = yO - yM, dP = yP - yO;
  if (dM * dP <= T(0)) return yO;
  const T inv = T(0.5) / (T(1) + r);
  const T cM = yO - (r * r * dP + dM) * inv;
  if ((cM - yM) * (cM - yO) > T(0)) return yM;
  const T cP = yO + (r * dP + dM / r) * inv;
  if ((cP - yO) * (cP - yP) > T(0)) return yO - r * dP;
  return cM;
}

// Monotonic quadratic Bezier interpolation through three equidistant nodes at
// -1, 0, +1, evaluated at t in [-1/2, 1/2].  Each interval takes the BESSER
// control point (Sect. 3.2) of the triple read towards it, so the value does not
// depend on the reading direction and reduces to the Lagrange parabola when
// nothing is clamped.
//
// With equal spacing (ratio 1) the BESSER branches collapse.  Let d1 = y0 - ym,
// d2 = yp - y0.  If d1 and d2 differ in sign the control point is y0.  Otherwise
// the parabola's tangent point y0 +- (d1 + d2)/4 overshoots ym exactly when
// |d2| > 3|d1| (clamped to ym = y0 - d1) and its mirror overshoots yp exactly
// when |d1| > 3|d2| (giving y0 - d2 on the upwind side), so both control points
// are y0 -+ q with q = sign(d1) min(|d1|, |d2|, |d1 + d2|/4).  The spline value is
// then linear in (ym, y0, yp, q) with weights that depend on t alone:
//   t >= 0:  (1-t)^2 y0 + 2t(1-t)(y0 + q) + t^2 yp
//   t <  0:  t^2 ym + 2(1+t)(-t)(y0 - q) + (1+t)^2 y0
// i.e. a ym + (1 - t^2) y0 + c yp + 2t(1 - |t|) q with a = t^2 [t<0], c = t^2 [t>=0].
template <class T>
struct BezW {
  T a, b, c, e;
};

template <class T>
__host__ __device__ inline BezW<T> bez_weights(T t) {
  const T t2 = t * t;
  BezW<T> w;
  w.a = (t < T(0)) ? t2 : T(0);
  w.b = T(1) - t2;
  w.c = (t < T(0)) ? T(0) : t2;
  w.e = T(2) * t * (T(1) - fabs(t));
  return w;
}

template <class T>
__host__ __device__ inline T bez_eval(const BezW<T>& w, T ym, T y0, T yp) {
  const T d1 = y0 - ym, d2 = yp - y0;
  const T m = fmin(fmin(fabs(d1), fabs(d2)), T(0.25) * fabs(d1 + d2));
  // a zero difference gives m = 0, so only opposite strict signs need the test
  const T q = ((d1 > T(0)) == (d2 > T(0))) ? copysign(m, d1) : T(0);
  return w.a * ym + w.b * y0 + w.c * yp + w.e * q;
}

// bez_eval with its partial derivatives g = d/d(ym, y0, yp), on the branches the value
// takes: q = c - y0 is the clamped offset of the control point, which is 0 (with no
// dependence) where the two differences do not share a strict sign (the extremum rule
// of the control point), else d1, d2 or (d1 + d2)/4, whichever is smallest in size.
template <class T>
__host__ __device__ inline T bez_eval_grad(const BezW<T>& w, T ym, T y0, T yp, T g[3]) {
  const T d1 = y0 - ym, d2 = yp - y0;
  T q = T(0), q1 = T(0), q2 = T(0);   // q and its partials in d1, d2
  if (d1 * d2 > T(0)) {
    const T a1 = fabs(d1), a2 = fabs(d2), a3 = T(0.25) * fabs(d1 + d2);
    if (a1 <= a2 && a1 <= a3) {
      q = d1;
      q1 = T(1);
    } else if (a2 <= a3) {
      q = d2;
      q2 = T(1);
    } else {
      q = T(0.25) * (d1 + d2);
      q1 = q2 = T(0.25);
    }
  }
  g[0] = w.a - w.e * q1;
  g[1] = w.b + w.e * (q1 - q2);
  g[2] = w.c + w.e * q2;
  return w.a * ym + w.b * y0 + w.c * yp + w.e * q;
}

template <class T>
__host__ __device__ inline T bezier3(T ym, T y0, T yp, T t) {
  return bez_eval(bez_weights(t), ym, y0, yp);
}

// BESSER control point together with its partial derivatives
// d = (dc/dy_M, dc/dy_O, dc/dy_P, dc/dr), following the same branches.
__host__ __device__ inline double besser_cm_grad(double yM, double yO, double yP, double r,
                                                 double d[4]) {
  const double dM = yO - yM, dP = yP - yO;
  d[0] = d[1] = d[2] = d[3] = 0.0;
  if (dM * dP <= 0.0) {
    d[1] = 1.0;
    return yO;
  }
  const double inv = 0.5 / (1.0 + r);
  const double cM = yO - (r * r * dP + dM) * inv;
  if ((cM - yM) * (cM - yO) > 0.0) {
    d[0] = 1.0;
    return yM;
  }
  const double cP = yO + (r * dP + dM / r) * inv;
  if ((cP - yO) * (cP - yP) > 0.0) {
    d[1] = 1.0 + r;
    d[2] = -r;
    d[3] = -dP;
    return yO - r * dP;
  }
  d[0] = inv;
  d[1] = 1.0 - (1.0 - r * r) * inv;
  d[2] = -r * r * inv;
  d[3] = -2.0 * (r * r * dP + 2.0 * r * dP - dM) * inv * inv;
  return cM;
}

// The parabolic control point with d = (dc/dy_M, dc/dy_O, dc/dy_P, dc/dr).
__host__ __device__ inline double parabolic_cm_grad(double yM, double yO, double yP, double r,
                                                    double d[4]) {
  const double dM = yO - yM, dP = yP - yO;
  const double inv = 0.5 / (1.0 + r);
  d[0] = inv;
  d[1] = 1.0 - (1.0 - r * r) * inv;
  d[2] = -r * r * inv;
  d[3] = -2.0 * (r * r * dP + 2.0 * r * dP - dM) * inv * inv;
  return yO - (r * r * dP + dM) * inv;
}

// dL/dtau from the adjoints of the six coefficients, with the derivatives
// written through the coefficients themselves (pmt = psi'_M/t, omt = omega_M/t,
// oct = omega_C/t, formed with the coefficients):
//   de/dt = -e,                 dpsi'_M/dt = e - pmt,   dpsi'_O/dt = pmt,
//   domega_M/dt = e - 2 omt,    domega_C/dt = 2 (pmt - oct),
//   domega_O/dt = 2 (omt + oct - pmt)   (from omega_M+omega_O+omega_C = 1-e).
template <class T>
__host__ __device__ inline T coef_tau_grad(const Coefs<T>& c, T gE, T gPM, T gPO, T gOM, T gOO,
                                           T gOC) {
  return -c.e * gE + (c.e - c.pmt) * gPM + c.pmt * gPO + (c.e - T(2) * c.omt) * gOM +
         T(2) * (c.omt + c.oct - c.pmt) * gOO + T(2) * (c.pmt - c.oct) * gOC;
}

// ---------------------------------------------------------------------------
// Solve (1 + K') x = b for a Stokes 4-vector, K' with the symmetric
// dichroism block e = (e_Q, e_U, e_V) and the antisymmetric dispersion block
// r = (r_Q, r_U, r_V):
//   K' = [[0, eQ, eU, eV], [eQ, 0, rV, -rU], [eU, -rV, 0, rQ], [eV, rU, -rQ, 0]].
// Eliminating x_0 leaves (B - e e^T) x_v = b_v - b_0 e with B y = y + y x r,
// whose inverse is B^-1 y = (y - y x r + (y.r) r) / (1 + r.r); the rank-one
// term is removed with the Sherman-Morrison formula.
// ---------------------------------------------------------------------------
template <class T>
__host__ __device__ inline void binv(const T y[3], const T r[3], T inv_den, T out[3]) {
  const T yr = y[0] * r[0] + y[1] * r[1] + y[2] * r[2];
  out[0] = (y[0] - (y[1] * r[2] - y[2] * r[1]) + yr * r[0]) * inv_den;
  out[1] = (y[1] - (y[2] * r[0] - y[0] * r[2]) + yr * r[1]) * inv_den;
  out[2] = (y[2] - (y[0] * r[1] - y[1] * r[0]) + yr * r[2]) * inv_den;
}

template <class T>
__host__ __device__ inline void solve_stokes(const T e[3], const T r[3], const T b[4], T x[4]) {
  const T inv_den = recip(T(1) + r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  const T c[3] = {b[1] - b[0] * e[0], b[2] - b[0] * e[1], b[3] - b[0] * e[2]};
  T u[3], v[3];
  binv(c, r, inv_den, u);
  binv(e, r, inv_den, v);
  const T eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
  const T ev = e[0] * v[0] + e[1] * v[1] + e[2] * v[2];
  const T f = eu * recip(T(1) - ev);
  x[1] = u[0] + f * v[0];
  x[2] = u[1] + f * v[1];
  x[3] = u[2] + f * v[2];
  x[0] = b[0] - (e[0] * x[1] + e[1] * x[2] + e[2] * x[3]);
}

// The same solve for the family 1 + p K' with K' fixed per node and ray and the
// scalar p = psi'_O varying with frequency.  With X = e x r,
//   B^-1 c = (c - p c x r + p^2 (c.r) r) / (1 + p^2 r.r),
//   v = B^-1 (p e) = p (e - p X + p^2 (e.r) r) / (1 + p^2 r.r),
//   (p e).v = p^2 (e.e + p^2 (e.r)^2) / (1 + p^2 r.r)      (since e.X = 0),
// so the products of e and r are formed once (StokesOp) and each frequency needs
// two reciprocals (StokesFreq) shared by the system and its transpose, which is the
// same with r -> -r (SGN = -1).
template <class T>
struct StokesOp {
  T e[3], r[3], X[3], C[3];   // e, r, e x r, (e.r) r
  T rr, ee, er2;              // r.r, e.e, (e.r)^2
};

template <class T>
__host__ __device__ inline StokesOp<T> stokes_op(const T e[3], const T r[3]) {
  StokesOp<T> k;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    k.e[i] = e[i];
    k.r[i] = r[i];
  }
  k.X[0] = e[1] * r[2] - e[2] * r[1];
  k.X[1] = e[2] * r[0] - e[0] * r[2];
  k.X[2] = e[0] * r[1] - e[1] * r[0];
  const T er = e[0] * r[0] + e[1] * r[1] + e[2] * r[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) k.C[i] = er * r[i];
  k.rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  k.ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
  k.er2 = er * er;
  return k;
}

template <class T>
struct StokesFreq {
  T p, p2, inv_den, fden;     // p, p^2, 1/(1 + p^2 r.r), 1/(1 - (p e).v)
};

template <class T>
__host__ __device__ inline StokesFreq<T> stokes_freq(const StokesOp<T>& k, T p) {
  StokesFreq<T> F;
  F.p = p;
  F.p2 = p * p;
  F.inv_den = recip(T(1) + F.p2 * k.rr);
  F.fden = recip(T(1) - F.p2 * F.inv_den * (k.ee + F.p2 * k.er2));
  return F;
}

// x = (1 + p K')^-1 b (SGN = 1) or (1 + p K')^-T b (SGN = -1).
template <int SGN, class T>
__host__ __device__ inline void stokes_solve(const StokesOp<T>& k, const StokesFreq<T>& F,
                                             const T b[4], T x[4]) {
  const T q = SGN > 0 ? F.p : -F.p;
  const T pb0 = F.p * b[0];
  const T c[3] = {b[1] - pb0 * k.e[0], b[2] - pb0 * k.e[1], b[3] - pb0 * k.e[2]};
  const T cx[3] = {c[1] * k.r[2] - c[2] * k.r[1], c[2] * k.r[0] - c[0] * k.r[2],
                   c[0] * k.r[1] - c[1] * k.r[0]};
  const T p2cr = F.p2 * (c[0] * k.r[0] + c[1] * k.r[1] + c[2] * k.r[2]);
  const T s = F.p * F.inv_den;
  T u[3], v[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u[i] = (c[i] - q * cx[i] + p2cr * k.r[i]) * F.inv_den;
    v[i] = s * (k.e[i] - q * k.X[i] + F.p2 * k.C[i]);
  }
  const T f = F.p * (k.e[0] * u[0] + k.e[1] * u[1] + k.e[2] * u[2]) * F.fden;
  x[1] = u[0] + f * v[0];
  x[2] = u[1] + f * v[1];
  x[3] = u[2] + f * v[2];
  x[0] = b[0] - F.p * (k.e[0] * x[1] + k.e[1] * x[2] + k.e[2] * x[3]);
}

// K' x for the same layout (eta = e, rho = r).
template <class T>
__host__ __device__ inline void kprime_apply(const T e[3], const T r[3], const T x[4], T y[4]) {
  y[0] = e[0] * x[1] + e[1] * x[2] + e[2] * x[3];
  y[1] = e[0] * x[0] + r[2] * x[2] - r[1] * x[3];
  y[2] = e[1] * x[0] - r[2] * x[1] + r[0] * x[3];
  y[3] = e[2] * x[0] + r[1] * x[1] - r[0] * x[2];
}

// ---------------------------------------------------------------------------
// Per-ray projection tables built from the spherical tensors T^K_Q(i, Omega)
// of Eq. 1 (reference direction of Stokes Q along (mu cos chi, mu sin chi,
// -sin theta)):
//   emis[i][c]: eps_i = sum_c emis[i][c] e_c for the six real multipole
//               components e = (eps00, eps20, Re eps21, Im eps21, Re eps22,
//               Im eps22), i.e. eps_i = sum_KQ w^K T^K_Q(i) eps^K_Q summed
//               over +-Q with eps^K_-Q = (-1)^Q conj(eps^K_Q);
//   proj[c][i]: J_c = sum_i proj[c][i] I_i for c = J00, J10, Re J11, Im J11,
//               J20, Re J21, Im J21, Re J22, Im J22.
// ---------------------------------------------------------------------------
struct RayConsts {
  double mu;        // signed direction cosine
  double sx, sy;    // horizontal direction components sin(theta) cos/sin(chi)
  double weight;    // quadrature weight (all rays sum to 1)
  double emis[4][6];
  double proj[9][4];
};

__host__ __device__ inline void ray_consts(double mu, double chi, double weight, double w2,
                                           RayConsts& rc) {
  const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  const double c1 = cos(chi), s1 = sin(chi), c2 = cos(2.0 * chi), s2 = sin(2.0 * chi);
  const double r3h = 0.5 * sqrt(3.0);            // sqrt(3)/2
  const double r3q = 0.25 * sqrt(3.0);           // sqrt(3)/4
  const double k20 = 1.0 / (2.0 * sqrt(2.0));
  rc.mu = mu;
  rc.sx = st * c1;
  rc.sy = st * s1;
  rc.weight = weight;
  // T^K_Q for Q >= 0 as (re, im): index 0 -> K=0; 1 -> (1,0); 2 -> (1,1);
  // 3 -> (2,0); 4 -> (2,1); 5 -> (2,2).
  double tr[4][6] = {}, ti[4][6] = {};
  // Stokes I
  tr[0][0] = 1.0;
  tr[0][3] = k20 * (3.0 * mu * mu - 1.0);
  tr[0][4] = -r3h * st * mu * c1;  ti[0][4] = -r3h * st * mu * s1;
  tr[0][5] = r3q * st * st * c2;   ti[0][5] = r3q * st * st * s2;
  // Stokes Q
  tr[1][3] = -3.0 * k20 * st * st;
  tr[1][4] = -r3h * st * mu * c1;  ti[1][4] = -r3h * st * mu * s1;
  tr[1][5] = -r3q * (1.0 + mu * mu) * c2;  ti[1][5] = -r3q * (1.0 + mu * mu) * s2;
  // Stokes U: -i (sqrt3/2) sin(theta) e^{i chi}, -i (sqrt3/2) mu e^{2 i chi}
  tr[2][4] = r3h * st * s1;        ti[2][4] = -r3h * st * c1;
  tr[2][5] = r3h * mu * s2;        ti[2][5] = -r3h * mu * c2;
  // Stokes V
  tr[3][1] = sqrt(1.5) * mu;
  tr[3][2] = -r3h * st * c1;       ti[3][2] = -r3h * st * s1;
  for (int i = 0; i < 4; ++i) {
    rc.emis[i][0] = tr[i][0];
    rc.emis[i][1] = w2 * tr[i][3];
    rc.emis[i][2] = 2.0 * w2 * tr[i][4];    // 2 Re(T e) = 2 (Tr er - Ti ei)
    rc.emis[i][3] = -2.0 * w2 * ti[i][4];
    rc.emis[i][4] = 2.0 * w2 * tr[i][5];
    rc.emis[i][5] = -2.0 * w2 * ti[i][5];
    rc.proj[0][i] = tr[i][0];
    rc.proj[1][i] = tr[i][1];
    rc.proj[2][i] = tr[i][2];
    rc.proj[3][i] = ti[i][2];
    rc.proj[4][i] = tr[i][3];
    rc.proj[5][i] = tr[i][4];
    rc.proj[6][i] = ti[i][4];
    rc.proj[7][i] = tr[i][5];
    rc.proj[8][i] = ti[i][5];
  }
}

// ---------------------------------------------------------------------------
// Two-level statistical equilibrium for K = 2 with Hanle rotation, written as
// a real 5x5 system in x = (S20, Re S21, Im S21, Re S22, Im S22).  With
// a = 1 + delta (1 - eps), h = (1 - eps) H_u, g = sqrt(6)/2 and the right-hand
// side R_Q = (1 - eps) w2 conj(J^2_Q):
//   a S_Q + i h sum_Q' <Q|b.J|Q'> S_Q' = R_Q, using S_-Q = (-1)^Q conj(S_Q).
// Rows Q = 0, 1 (re, im), 2 (re, im).
// ---------------------------------------------------------------------------
__host__ __device__ inline void hanle_system(double a, double h, double bx, double by,
                                             double bz, double A[5][5]) {
  const double g = 0.5 * sqrt(6.0);
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) A[i][j] = 0.0;
  // Q = 0
  A[0][0] = a;
  A[0][1] = -2.0 * h * g * by;
  A[0][2] = -2.0 * h * g * bx;
  // Q = 1, real part
  A[1][0] = h * g * by;
  A[1][1] = a;
  A[1][2] = -h * bz;
  A[1][3] = -h * by;
  A[1][4] = -h * bx;
  // Q = 1, imaginary part
  A[2][0] = h * g * bx;
  A[2][1] = h * bz;
  A[2][2] = a;
  A[2][3] = h * bx;
  A[2][4] = -h * by;
  // Q = 2, real part
  A[3][1] = h * by;
  A[3][2] = -h * bx;
  A[3][3] = a;
  A[3][4] = -2.0 * h * bz;
  // Q = 2, imaginary part
  A[4][1] = h * bx;
  A[4][2] = h * by;
  A[4][3] = 2.0 * h * bz;
  A[4][4] = a;
}

// Gaussian elimination with partial pivoting.  Every index is a compile-time constant
// (the pivot row is swapped in by selects over the candidate rows), so on the GPU the
// matrix stays in registers rather than in per-lane scratch memory.
template <int N>
__host__ __device__ inline void solve_pivot(double A[N][N], double b[N]) {
#pragma unroll
  for (int c = 0; c < N; ++c) {
    int piv = c;
    double best = fabs(A[c][c]);
#pragma unroll
    for (int r = c + 1; r < N; ++r) {
      const double v = fabs(A[r][c]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
#pragma unroll
    for (int r = c + 1; r < N; ++r) {
      const bool sw = piv == r;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const double t = A[c][k];
        A[c][k] = sw ? A[r][k] : t;
        A[r][k] = sw ? t : A[r][k];
      }
      const double t = b[c];
      b[c] = sw ? b[r] : t;
      b[r] = sw ? t : b[r];
    }
    const double inv = 1.0 / A[c][c];
#pragma unroll
    for (int r = c + 1; r < N; ++r) {
      const double f = A[r][c] * inv;
#pragma unroll
      for (int k = c; k < N; ++k) A[r][k] -= f * A[c][k];
      b[r] -= f * b[c];
    }
  }
#pragma unroll
  for (int r = N - 1; r >= 0; --r) {
    double s = b[r];
#pragma unroll
    for (int k = r + 1; k < N; ++k) s -= A[r][k] * b[k];
    b[r] = s / A[r][r];
  }
}

}  // namespace porta
