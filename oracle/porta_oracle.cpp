/*
 * porta_oracle.cpp -- plain, slow FP64 CPU oracle of the PORTA hot path.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or constant with the GPU library and the GPU library never calls it.
 *
 * What it computes (Stepan & Trujillo Bueno 2013, arXiv:1307.4217):
 *   - the short-characteristics formal solution of the Stokes-vector transfer
 *     equation (Sect. 3, Eqs. rte, fsint) with the BESSER monotonic quadratic
 *     Bezier source-function interpolation (Sect. 3.2, steps 1-9) and the
 *     linear treatment of K'I (Sect. 3.3, Eqs. fsbez, kappa, omega_M/O/C,
 *     psi'_M/O, Table 1 for small optical depths), swept over a 3-D grid
 *     that is periodic in x and y (Sect. 3.1, Appendix A);
 *   - the diagonal Lambda* of Sect. 3.3 (Eq. 14);
 *   - the radiation-field tensors J^K_Q of Eq. 1 on the discrete quadrature;
 *   - one Jacobi update of the statistical equilibrium of a two-level
 *     J_l = 0 -> J_u = 1 atom with Hanle rotation (Sect. 2, Eq. nonlte;
 *     Sect. 5 for the Jacobi scheme and the convergence measure R_c);
 *   - long characteristics along the same rays (brute force check), and through
 *     the trilinear medium cut at every face crossing (reference for the
 *     vertical-face variant);
 *   - complex-step directional derivatives of the emergent Stokes vector;
 *   - the reverse-mode gradient of a loss on the emergent Stokes vector with
 *     respect to every transfer coefficient (recorded node updates, walked
 *     backward plane by plane).
 *
 * Readings where the paper is silent (same numbering as the design notes):
 *   A1 M and P always lie on the neighbouring horizontal grid planes.
 *   A3 emission and absorption coefficients are interpolated, S = eps/eta_I
 *      and K' = K/eta_I - 1 are formed at M, O and P afterwards.
 *   A4 tau_MO = (eta_I(M) + eta_I(O))/2 * |Delta s|.
 *   A5 on the last plane of a ray (no downwind point) c_M = (y_M + y_O)/2.
 *   A6 series thresholds: omega_M 0.14, omega_O and omega_C 0.18 (Table 1),
 *      psi'_M and psi'_O 0.1.
 *   A7 Lambda* is the response of I_O to a unit S_O (Stokes I only): omega_O +
 *      c omega_C with c the control point of that unit source (1 with BESSER,
 *      (1 + tau_MO/tau_OP)/2 with the parabolic rule, 1/2 on the last plane, A5);
 *      zero on the boundary plane.
 *   A8 K = 2 multipoles are updated by plain Lambda iteration.
 *   A9/O7 T^K_Q(i, Omega) with reference direction gamma = 0, see tkq().
 *
 * Everything is double precision; the sweep is templated on the scalar so
 * that std::complex<double> inputs p + i h v give the exact directional
 * derivative Im(I(p + i h v))/h of the branch taken by the real evaluation.
 */
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cd = std::complex<double>;

inline double rp(double v) { return v; }
inline double rp(const cd& v) { return v.real(); }

/* A physical complex number; each part may itself carry a complex-step
 * perturbation when T = std::complex<double>. */
template <class T>
struct Cx {
  T re, im;
};
/* Real part of the product a b. */
template <class T>
inline T cmul_re(const Cx<double>& a, const Cx<T>& b) {
  return a.re * b.re - a.im * b.im;
}

/* -------------------------------------------------------------------------- */
/* Problem description (the oracle's own definition of the inputs).           */
/* -------------------------------------------------------------------------- */
}  // namespace

extern "C" {
typedef struct {
  int nx, ny, nz;
  double lx, ly;
  const double* z;      /* nz heights, strictly increasing */
  int nmu, nchi, nfreq;
  const double* mu;     /* nmu inclination cosines in (0,1] (one hemisphere) */
  const double* wmu;    /* nmu weights, sum 1 */
  const double* phi;    /* nfreq profile values relative to line centre */
  const double* wfreq;  /* nfreq frequency quadrature weights */
  double i_bottom;      /* Stokes I entering at the bottom for upward rays */
  double w2;            /* w^(2) of the transition */
  int interp;           /* 0 bilinear, 1 9-point monotonic Bezier */
  int control;          /* control point along the ray: 0 BESSER (Sect. 3.2, steps 1-9),
                           1 parabolic (steps 1, 3, 4 only: the DELOPAR choice) */
  int faces;            /* where M and P lie: 0 on the neighbouring horizontal planes
                           (reading A1); 1 on the first face of the grid the ray crosses,
                           horizontal or vertical (Sect. 3.1), with bilinear interpolation
                           on that face; needs interp = 0 */
} oracle_problem;
}

namespace {

/* Ray enumeration: rays [0, nmu*nchi) go upward (mu > 0), the rest downward;
 * inside a hemisphere the inclination index is slow and the azimuth fast.
 * Azimuths follow the trapezoid rule with nodes (m + 1/2) 2 pi / nchi; the
 * weight of a ray is wmu/2/nchi so that all weights sum to one. */
struct Ray {
  double mu, sint, chi, sx, sy, w;
  bool up;
};

Ray make_ray(const oracle_problem& pb, int r) {
  const int nh = pb.nmu * pb.nchi;
  const int hemi = r / nh;
  const int a = (r % nh) / pb.nchi;
  const int m = r % pb.nchi;
  Ray ray;
  ray.up = (hemi == 0);
  ray.mu = ray.up ? pb.mu[a] : -pb.mu[a];
  ray.sint = std::sqrt(std::max(0.0, 1.0 - pb.mu[a] * pb.mu[a]));
  ray.chi = (m + 0.5) * 2.0 * M_PI / pb.nchi;
  ray.sx = ray.sint * std::cos(ray.chi);
  ray.sy = ray.sint * std::sin(ray.chi);
  ray.w = 0.5 * pb.wmu[a] / pb.nchi;
  return ray;
}

/* Index of (K, Q) in a 9-slot table: K=0 -> 0; K=1, Q=-1..1 -> 1..3; K=2, Q=-2..2 -> 4..8 */
inline int kq(int K, int Q) { return K == 0 ? 0 : (K == 1 ? 2 + Q : 6 + Q); }

/* Spherical tensors T^K_Q(i, Omega) of Eq. 1 (i = I, Q, U, V), polarization
 * reference: Q > 0 along e_a = (mu cos chi, mu sin chi, -sin theta). */
void tkq(double mu, double chi, Cx<double> t[4][9]) {
  for (int i = 0; i < 4; ++i)
    for (int s = 0; s < 9; ++s) t[i][s] = Cx<double>{0.0, 0.0};
  const double st = std::sqrt(std::max(0.0, 1.0 - mu * mu));
  const double r2 = std::sqrt(2.0), r3 = std::sqrt(3.0);
  auto ph = [&](int q, double amp) {  // amp * e^{i q chi}
    return Cx<double>{amp * std::cos(q * chi), amp * std::sin(q * chi)};
  };
  auto iph = [&](int q, double amp) {  // i * amp * e^{i q chi}
    return Cx<double>{-amp * std::sin(q * chi), amp * std::cos(q * chi)};
  };
  /* Stokes I */
  t[0][kq(0, 0)] = Cx<double>{1.0, 0.0};
  t[0][kq(2, 0)] = Cx<double>{(3.0 * mu * mu - 1.0) / (2.0 * r2), 0.0};
  t[0][kq(2, 1)] = ph(1, -0.5 * r3 * st * mu);
  t[0][kq(2, -1)] = ph(-1, +0.5 * r3 * st * mu);
  t[0][kq(2, 2)] = ph(2, 0.25 * r3 * st * st);
  t[0][kq(2, -2)] = ph(-2, 0.25 * r3 * st * st);
  /* Stokes Q */
  t[1][kq(2, 0)] = Cx<double>{-3.0 / (2.0 * r2) * st * st, 0.0};
  t[1][kq(2, 1)] = ph(1, -0.5 * r3 * st * mu);
  t[1][kq(2, -1)] = ph(-1, +0.5 * r3 * st * mu);
  t[1][kq(2, 2)] = ph(2, -0.25 * r3 * (1.0 + mu * mu));
  t[1][kq(2, -2)] = ph(-2, -0.25 * r3 * (1.0 + mu * mu));
  /* Stokes U */
  t[2][kq(2, 1)] = iph(1, -0.5 * r3 * st);
  t[2][kq(2, -1)] = iph(-1, -0.5 * r3 * st);
  t[2][kq(2, 2)] = iph(2, -0.5 * r3 * mu);
  t[2][kq(2, -2)] = iph(-2, +0.5 * r3 * mu);
  /* Stokes V */
  t[3][kq(1, 0)] = Cx<double>{std::sqrt(1.5) * mu, 0.0};
  t[3][kq(1, 1)] = ph(1, -0.5 * r3 * st);
  t[3][kq(1, -1)] = ph(-1, +0.5 * r3 * st);
}

/* -------------------------------------------------------------------------- */
/* Sect. 3.3: coefficients of Eq. fsbez.                                      */
/* -------------------------------------------------------------------------- */
template <class T>
struct Coef {
  T e, psiM, psiO, omM, omO, omC;
};

constexpr double kThreshOmegaM = 0.14;  // Table 1
constexpr double kThreshOmegaOC = 0.18; // Table 1
constexpr double kThreshPsi = 0.10;     // reading A6

template <class T>
Coef<T> coefficients(const T& tau) {
  using std::exp;
  Coef<T> c;
  const double t = rp(tau);
  c.e = exp(-tau);
  /* at tau = 0 the series branch gives e = 1 and all other coefficients 0 */
  const T t2 = tau * tau;
  /* Taylor series about tau = 0, 8 terms each, n = 0..7 */
  T sM(0.0), sO(0.0), sC(0.0), pM(0.0), pO(0.0);
  {
    double fact = 1.0;  // n!
    T tp = tau;         // tau^{n+1}
    for (int n = 0; n < 8; ++n) {
      if (n > 0) fact *= n;
      const double sg = (n % 2 == 0) ? 1.0 : -1.0;
      sM += sg * tp / (fact * (n + 3));
      sO += sg * 2.0 * tp / (fact * (n + 1) * (n + 2) * (n + 3));   // 2 tau^{n+1}/(n+3)!
      sC += sg * 2.0 * tp / (fact * (n + 2) * (n + 3));
      pM += sg * tp / (fact * (n + 2));
      pO += sg * tp / (fact * (n + 1) * (n + 2));                   // tau^{n+1}/(n+2)!
      tp = tp * tau;
    }
  }
  if (t < kThreshPsi) {
    c.psiM = pM;
    c.psiO = pO;
  } else {
    c.psiM = (1.0 - c.e * (1.0 + tau)) / tau;
    c.psiO = (c.e + tau - 1.0) / tau;
  }
  if (t < kThreshOmegaM)
    c.omM = sM;
  else
    c.omM = (2.0 - c.e * (t2 + 2.0 * tau + 2.0)) / t2;
  if (t < kThreshOmegaOC) {
    c.omO = sO;
    c.omC = sC;
  } else {
    c.omO = 1.0 - 2.0 * (c.e + tau - 1.0) / t2;
    c.omC = 2.0 * (tau - 2.0 + c.e * (tau + 2.0)) / t2;
  }
  return c;
}

/* -------------------------------------------------------------------------- */
/* Sect. 3.2: BESSER control point c_M of the upwind interval MO.             */
/* -------------------------------------------------------------------------- */
template <class T>
T besser_cm(const T& yM, const T& yO, const T& yP, const T& hM, const T& hP) {
  if (!(rp(hM) > 0.0)) return yO;       // zero-length MO interval: c_M is irrelevant
  if (!(rp(hP) > 0.0)) {                // limit h_P -> 0 of steps 3-6
    if (rp(yO - yM) * rp(yP - yO) <= 0.0) return yO;
    return yM;
  }
  /* step 1 */
  const T dM = (yO - yM) / hM;
  const T dP = (yP - yO) / hP;
  /* step 2: not monotonic -> local extremum at O */
  if (rp(dM) * rp(dP) <= 0.0) return yO;
  /* step 3: derivative at O (Eq. deriv) */
  T yd = (hM * dP + hP * dM) / (hM + hP);
  /* step 4 */
  T cM = yO - 0.5 * hM * yd;
  T cP = yO + 0.5 * hP * yd;
  /* steps 5-6: overshoot in MO */
  const double lo = std::min(rp(yM), rp(yO)), hi = std::max(rp(yM), rp(yO));
  if (rp(cM) < lo || rp(cM) > hi) return yM;
  /* step 7: overshoot in OP */
  const double lo2 = std::min(rp(yO), rp(yP)), hi2 = std::max(rp(yO), rp(yP));
  if (rp(cP) < lo2 || rp(cP) > hi2) {
    cP = yP;
    /* step 8: new derivative at O */
    yd = (cP - yO) / (0.5 * hP);
    /* step 9: keep the derivative at O continuous */
    cM = yO - 0.5 * hM * yd;
  }
  return cM;
}

/* The control point of the parabola through M, O, P (steps 1, 3 and 4 of Sect. 3.2
 * without the monotonicity tests): the formal solver then interpolates the source
 * function parabolically, as DELOPAR does (Sect. 3). */
template <class T>
T parabolic_cm(const T& yM, const T& yO, const T& yP, const T& hM, const T& hP) {
  if (!(rp(hM) > 0.0)) return yO;
  if (!(rp(hP) > 0.0)) return 0.5 * (yM + yO);   // no downwind point: the chord's midpoint
  const T dM = (yO - yM) / hM;
  const T dP = (yP - yO) / hP;
  const T yd = (hM * dP + hP * dM) / (hM + hP);
  return yO - 0.5 * hM * yd;
}

template <class T>
T control_point(int control, const T& yM, const T& yO, const T& yP, const T& hM, const T& hP) {
  return control == 1 ? parabolic_cm(yM, yO, yP, hM, hP) : besser_cm(yM, yO, yP, hM, hP);
}

/* One-dimensional monotonic quadratic Bezier interpolation through three
 * equidistant nodes at -1, 0, +1, evaluated at t in [-1/2, 1/2].  The control
 * point of each interval is the BESSER c_M of the triple read towards that
 * interval, so the result does not depend on the reading direction. */
template <class T>
T bezier1d(const T& ym, const T& y0, const T& yp, double t) {
  const T one(1.0);
  if (t >= 0.0) {
    const T c = besser_cm(yp, y0, ym, one, one);
    return (1.0 - t) * (1.0 - t) * y0 + 2.0 * t * (1.0 - t) * c + t * t * yp;
  }
  const T c = besser_cm(ym, y0, yp, one, one);
  const double u = 1.0 + t;
  return (1.0 - u) * (1.0 - u) * ym + 2.0 * u * (1.0 - u) * c + u * u * y0;
}

inline int wrap(long i, int n) {
  long r = i % n;
  return (int)(r < 0 ? r + n : r);
}

/* Interpolation of a horizontal plane (x fastest) at a point given in cell
 * units; x and y are periodic.  Mode 0: bilinear from the 4 surrounding
 * nodes.  Mode 1: 9 nodes around the nearest node, monotonic Bezier along x
 * for each of the three rows, then along y. */
template <class T>
T interp_plane(const T* f, int nx, int ny, double fx, double fy, int mode) {
  if (mode == 0) {
    const double fi = std::floor(fx), fj = std::floor(fy);
    const double tx = fx - fi, ty = fy - fj;
    const int i0 = wrap((long)fi, nx), i1 = wrap((long)fi + 1, nx);
    const int j0 = wrap((long)fj, ny), j1 = wrap((long)fj + 1, ny);
    return (1.0 - tx) * (1.0 - ty) * f[j0 * nx + i0] + tx * (1.0 - ty) * f[j0 * nx + i1] +
           (1.0 - tx) * ty * f[j1 * nx + i0] + tx * ty * f[j1 * nx + i1];
  }
  const double fi = std::floor(fx + 0.5), fj = std::floor(fy + 0.5);
  const double tx = fx - fi, ty = fy - fj;
  T row[3];
  for (int dj = -1; dj <= 1; ++dj) {
    const int j = wrap((long)fj + dj, ny);
    const T* r = f + (size_t)j * nx;
    row[dj + 1] = bezier1d(r[wrap((long)fi - 1, nx)], r[wrap((long)fi, nx)],
                           r[wrap((long)fi + 1, nx)], tx);
  }
  return bezier1d(row[0], row[1], row[2], ty);
}

/* Emission vector component i from the multipoles (eps00, eps20, Re eps21,
 * Im eps21, Re eps22, Im eps22): eps_i = Re sum_{KQ} w^(K) T^K_Q(i) eps^K_Q,
 * summed over all Q with eps^K_{-Q} = (-1)^Q conj(eps^K_Q); no K = 1 terms. */
template <class T>
T emission(const Cx<double> t[4][9], int i, const T e[6], double w2) {
  Cx<T> ek[9];
  for (int s = 0; s < 9; ++s) ek[s] = Cx<T>{T(0.0), T(0.0)};
  ek[kq(0, 0)] = Cx<T>{e[0], T(0.0)};
  ek[kq(2, 0)] = Cx<T>{e[1], T(0.0)};
  ek[kq(2, 1)] = Cx<T>{e[2], e[3]};
  ek[kq(2, 2)] = Cx<T>{e[4], e[5]};
  ek[kq(2, -1)] = Cx<T>{-e[2], e[3]};   // -(conj eps21)
  ek[kq(2, -2)] = Cx<T>{e[4], -e[5]};   // conj eps22
  T sum(0.0);
  for (int K = 0; K <= 2; ++K)
    for (int Q = -K; Q <= K; ++Q) {
      const double wk = (K == 0) ? 1.0 : (K == 2 ? w2 : 0.0);
      if (wk == 0.0) continue;
      sum += wk * cmul_re(t[i][kq(K, Q)], ek[kq(K, Q)]);
    }
  return sum;
}

/* K' = K/eta_I - 1 from (eta_Q, eta_U, eta_V, rho_Q, rho_U, rho_V) and eta_I. */
template <class T>
void kprime(const T eta[6], const T& etaI, T k[4][4]) {
  const T eQ = eta[0] / etaI, eU = eta[1] / etaI, eV = eta[2] / etaI;
  const T rQ = eta[3] / etaI, rU = eta[4] / etaI, rV = eta[5] / etaI;
  const T z(0.0);
  const T m[4][4] = {{z, eQ, eU, eV}, {eQ, z, rV, -rU}, {eU, -rV, z, rQ}, {eV, rU, -rQ, z}};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) k[a][b] = m[a][b];
}

/* Gaussian elimination with partial pivoting on the real parts. */
template <class T, int N>
void gauss_solve(T A[N][N], T b[N], T x[N]) {
  for (int c = 0; c < N; ++c) {
    int piv = c;
    for (int r = c + 1; r < N; ++r)
      if (std::fabs(rp(A[r][c])) > std::fabs(rp(A[piv][c]))) piv = r;
    if (piv != c) {
      for (int k = 0; k < N; ++k) std::swap(A[c][k], A[piv][k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < N; ++r) {
      const T f = A[r][c] / A[c][c];
      for (int k = c; k < N; ++k) A[r][k] -= f * A[c][k];
      b[r] -= f * b[c];
    }
  }
  for (int r = N - 1; r >= 0; --r) {
    T s = b[r];
    for (int k = r + 1; k < N; ++k) s -= A[r][k] * x[k];
    x[r] = s / A[r][r];
  }
}

template <class T>
struct FieldsT {
  const T* kappa;  // [N]
  const T* prop;   // [6][N]
  const T* emis;   // [6][N]
};

/* Sect. 3.1: the point where the short characteristic through node O = (i, j, k)
 * first meets a face of the grid, going upwind (dir = -1, the point M) or downwind
 * (dir = +1, the point P): the horizontal plane next to k, or a vertical plane x =
 * const or y = const of the nodes next to O, whichever the ray reaches first (ties
 * go to the horizontal plane).  On a horizontal plane the four nodes around the
 * point are those of the bilinear interpolation in x and y; on a vertical plane they
 * are the nodes of that plane around it, bilinear in y (or x) and z, two of them on
 * plane k itself.  Returns false where the ray leaves the grid through its top or
 * bottom plane without crossing a face (no point P on the last plane). */
struct FacePoint {
  size_t node[4];
  double w[4];
  double ds;   /* distance from O */
};

bool first_face(const oracle_problem& pb, const Ray& ray, int i, int j, int k, int dir,
                FacePoint& fp) {
  const int nx = pb.nx, ny = pb.ny, nz = pb.nz;
  const size_t np = (size_t)nx * ny;
  const double dx = pb.lx / nx, dy = pb.ly / ny;
  const double ux = dir * ray.sx, uy = dir * ray.sy, uz = dir * ray.mu;   // direction of travel
  const int kz = k + (uz > 0.0 ? 1 : -1);
  if (kz < 0 || kz >= nz) return false;
  const double sz = std::fabs(pb.z[kz] - pb.z[k]) / std::fabs(uz);
  const double inf = std::numeric_limits<double>::infinity();
  const double sx = ux != 0.0 ? dx / std::fabs(ux) : inf;
  const double sy = uy != 0.0 ? dy / std::fabs(uy) : inf;
  auto at = [&](int ii, int jj, int kk) {
    return (size_t)kk * np + (size_t)wrap(jj, ny) * nx + (size_t)wrap(ii, nx);
  };
  if (sz <= sx && sz <= sy) {
    fp.ds = sz;
    const double fx = i + sz * ux / dx, fy = j + sz * uy / dy;
    const double fi = std::floor(fx), fj = std::floor(fy);
    const double tx = fx - fi, ty = fy - fj;
    const int i0 = (int)fi, j0 = (int)fj;
    fp.node[0] = at(i0, j0, kz);     fp.w[0] = (1.0 - tx) * (1.0 - ty);
    fp.node[1] = at(i0 + 1, j0, kz); fp.w[1] = tx * (1.0 - ty);
    fp.node[2] = at(i0, j0 + 1, kz); fp.w[2] = (1.0 - tx) * ty;
    fp.node[3] = at(i0 + 1, j0 + 1, kz); fp.w[3] = tx * ty;
    return true;
  }
  const bool xface = sx <= sy;
  const double s = xface ? sx : sy;
  fp.ds = s;
  const double tz = s * std::fabs(uz) / std::fabs(pb.z[kz] - pb.z[k]);   // fraction from k to kz
  if (xface) {
    const int ic = i + (ux > 0.0 ? 1 : -1);
    const double fy = j + s * uy / dy, fj = std::floor(fy), ty = fy - fj;
    const int j0 = (int)fj;
    fp.node[0] = at(ic, j0, k);      fp.w[0] = (1.0 - ty) * (1.0 - tz);
    fp.node[1] = at(ic, j0 + 1, k);  fp.w[1] = ty * (1.0 - tz);
    fp.node[2] = at(ic, j0, kz);     fp.w[2] = (1.0 - ty) * tz;
    fp.node[3] = at(ic, j0 + 1, kz); fp.w[3] = ty * tz;
  } else {
    const int jc = j + (uy > 0.0 ? 1 : -1);
    const double fx = i + s * ux / dx, fi = std::floor(fx), tx = fx - fi;
    const int i0 = (int)fi;
    fp.node[0] = at(i0, jc, k);      fp.w[0] = (1.0 - tx) * (1.0 - tz);
    fp.node[1] = at(i0 + 1, jc, k);  fp.w[1] = tx * (1.0 - tz);
    fp.node[2] = at(i0, jc, kz);     fp.w[2] = (1.0 - tx) * tz;
    fp.node[3] = at(i0 + 1, jc, kz); fp.w[3] = tx * tz;
  }
  return true;
}

template <class T>
T face_interp(const T* f, const FacePoint& fp) {
  return fp.w[0] * f[fp.node[0]] + fp.w[1] * f[fp.node[1]] + fp.w[2] * f[fp.node[2]] +
         fp.w[3] * f[fp.node[3]];
}

/* One step of the formal solution: the Stokes vector at node O = (i, j) of plane k
 * of the ray, from the upwind plane k - s already held in I ([4][N], one Stokes
 * component after the other).  Writes I_O into I and, if lam is given, Lambda* at O. */
template <class T>
void node_update(const oracle_problem& pb, const FieldsT<T>& f, const Ray& ray,
                 const Cx<double> t[4][9], double phi, int k, int i, int j, T* I, double* lam) {
  const int nx = pb.nx, ny = pb.ny, nz = pb.nz;
  const size_t np = (size_t)nx * ny;
  const size_t N = np * nz;
  const double dx = pb.lx / nx, dy = pb.ly / ny;
  const int s = ray.up ? 1 : -1;
  const int kup = k - s, kdn = k + s;
  const size_t pO = (size_t)k * np + (size_t)j * nx + i;
  /* M and P on the first face crossed (faces = 1, Sect. 3.1) */
  FacePoint fpM{}, fpP{};
  const bool faces = pb.faces != 0;
  const bool hasP = faces ? first_face(pb, ray, i, j, k, +1, fpP) : (kdn >= 0 && kdn < nz);
  if (faces) first_face(pb, ray, i, j, k, -1, fpM);
  const double dsM = faces ? fpM.ds : (pb.z[k] - pb.z[kup]) / ray.mu;
  const double dsP = faces ? (hasP ? fpP.ds : 0.0) : (hasP ? (pb.z[kdn] - pb.z[k]) / ray.mu : 0.0);
  /* or M on the upwind plane, P on the downwind plane (reading A1) */
  const double fxM = i - dsM * ray.sx / dx, fyM = j - dsM * ray.sy / dy;
  const double fxP = i + dsP * ray.sx / dx, fyP = j + dsP * ray.sy / dy;
  auto atM = [&](const T* arr) {
    if (faces) return face_interp(arr, fpM);
    return interp_plane(arr + (size_t)kup * np, nx, ny, fxM, fyM, pb.interp);
  };
  auto atP = [&](const T* arr) {
    if (faces) return face_interp(arr, fpP);
    return interp_plane(arr + (size_t)kdn * np, nx, ny, fxP, fyP, pb.interp);
  };
  /* absorption and emission at M, O, P (reading A3) */
  T kapM = atM(f.kappa), kapO = f.kappa[pO], kapP(0.0);
  T etaM[6], etaO[6], epsM[6], epsO[6], epsP[6];
  for (int c = 0; c < 6; ++c) {
    etaM[c] = atM(f.prop + c * N);
    etaO[c] = f.prop[c * N + pO];
    epsM[c] = atM(f.emis + c * N);
    epsO[c] = f.emis[c * N + pO];
    epsP[c] = T(0.0);
  }
  if (hasP) {
    kapP = atP(f.kappa);
    for (int c = 0; c < 6; ++c) epsP[c] = atP(f.emis + c * N);
  }
  /* Stokes vector at M, interpolated from the upwind plane */
  T IM[4];
  for (int st = 0; st < 4; ++st) IM[st] = atM(I + st * N);
  /* monochromatic coefficients: eta_I(nu) = kappa * phi, eps(nu) = eps * phi */
  const T etaIM = kapM * phi, etaIO = kapO * phi, etaIP = kapP * phi;
  T eM[6], eO[6], eP[6], nM[6], nO[6];
  for (int c = 0; c < 6; ++c) {
    eM[c] = epsM[c] * phi; eO[c] = epsO[c] * phi; eP[c] = epsP[c] * phi;
    nM[c] = etaM[c] * phi; nO[c] = etaO[c] * phi;
  }
  /* optical paths (reading A4) */
  const T tauMO = 0.5 * (etaIM + etaIO) * std::fabs(dsM);
  const T tauOP = 0.5 * (etaIO + etaIP) * std::fabs(dsP);
  /* source vectors S = eps / eta_I */
  T SM[4], SO[4], SP[4], cM[4];
  for (int st = 0; st < 4; ++st) {
    SM[st] = emission(t, st, eM, pb.w2) / etaIM;
    SO[st] = emission(t, st, eO, pb.w2) / etaIO;
    SP[st] = hasP ? emission(t, st, eP, pb.w2) / etaIP : T(0.0);
    cM[st] = hasP ? control_point(pb.control, SM[st], SO[st], SP[st], tauMO, tauOP)
                  : 0.5 * (SM[st] + SO[st]);   // reading A5
  }
  T KM[4][4], KO[4][4];
  kprime(nM, etaIM, KM);
  kprime(nO, etaIO, KO);
  const Coef<T> cf = coefficients(tauMO);
  /* Eq. fsbez right-hand side */
  T b[4];
  for (int a = 0; a < 4; ++a) {
    T acc = cf.e * IM[a];
    for (int c = 0; c < 4; ++c) acc -= cf.psiM * KM[a][c] * IM[c];
    acc += cf.omM * SM[a] + cf.omO * SO[a] + cf.omC * cM[a];
    b[a] = acc;
  }
  /* Eq. kappa: kappa^{-1} = 1 + psi'_O K'_O; solve kappa^{-1} I_O = b */
  T A[4][4];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c) A[a][c] = (a == c ? T(1.0) : T(0.0)) + cf.psiO * KO[a][c];
  T IO[4];
  gauss_solve<T, 4>(A, b, IO);
  for (int st = 0; st < 4; ++st) I[st * N + pO] = IO[st];
  /* Eq. 14: I_O for S_O = 1 and zero elsewhere, i.e. omega_O + omega_C c_M with c_M
   * the control point of that unit source (1 for BESSER, whose step 2 finds the
   * extremum at O; (1 + tau_MO/tau_OP)/2 for the parabola; 1/2 on the last plane,
   * reading A5) */
  if (lam) {
    const double cunit =
        hasP ? rp(control_point(pb.control, T(0.0), T(1.0), T(0.0), tauMO, tauOP)) : 0.5;
    lam[pO] = rp(cf.omO + cunit * cf.omC);
  }
}

/* Boundary plane of a ray (entering intensity; Lambda* = 0 there). */
template <class T>
void boundary_plane(const oracle_problem& pb, const Ray& ray, T* I, double* lam) {
  const size_t np = (size_t)pb.nx * pb.ny;
  const size_t N = np * pb.nz;
  const int kb = ray.up ? 0 : pb.nz - 1;
  for (size_t p = 0; p < np; ++p) {
    I[0 * N + kb * np + p] = T(ray.up ? pb.i_bottom : 0.0);
    I[1 * N + kb * np + p] = I[2 * N + kb * np + p] = I[3 * N + kb * np + p] = T(0.0);
    if (lam) lam[kb * np + p] = 0.0;
  }
}

/* The sweep when M may lie on a vertical face (faces = 1): a node then depends on
 * nodes of its own plane, and with x and y periodic these dependencies close around
 * the box.  Each plane (in upwind order) is therefore the fixed point of its node
 * equations, reached by passes over the plane in the ray's horizontal upwind order
 * (each pass carries the intensity once around the box) until a pass changes no
 * Stokes value by more than 1e-15 of the largest; the plane starts from zero.  A plane
 * that does not converge in kMaxPasses passes is set to NaN. */
constexpr int kMaxPasses = 200000;

template <class T>
void sweep_faces(const oracle_problem& pb, const FieldsT<T>& f, const Ray& ray,
                 const Cx<double> t[4][9], double phi, T* I, double* lam) {
  const int nx = pb.nx, ny = pb.ny, nz = pb.nz;
  const size_t np = (size_t)nx * ny, N = np * nz;
  const int s = ray.up ? 1 : -1;
  const int kb = ray.up ? 0 : nz - 1;
  const bool xup = ray.sx >= 0.0, yup = ray.sy >= 0.0;   // upwind neighbours at lower index
  for (int step = 1; step < nz; ++step) {
    const int k = kb + s * step;
    for (size_t q = 0; q < np; ++q)
      for (int st = 0; st < 4; ++st) I[st * N + (size_t)k * np + q] = T(0.0);
    bool done = false;
    for (int pass = 0; pass < kMaxPasses && !done; ++pass) {
      double change = 0.0, scale = 0.0;
      for (int jj = 0; jj < ny; ++jj)
        for (int ii = 0; ii < nx; ++ii) {
          const int i = xup ? ii : nx - 1 - ii, j = yup ? jj : ny - 1 - jj;
          const size_t pO = (size_t)k * np + (size_t)j * nx + i;
          double old[4];
          for (int st = 0; st < 4; ++st) old[st] = rp(I[st * N + pO]);
          node_update(pb, f, ray, t, phi, k, i, j, I, lam);
          for (int st = 0; st < 4; ++st) {
            const double v = rp(I[st * N + pO]);
            change = std::max(change, std::fabs(v - old[st]));
            scale = std::max(scale, std::fabs(v));
          }
        }
      done = pass > 0 && change <= 1e-15 * scale;
    }
    if (!done)
      for (size_t q = 0; q < np; ++q)
        for (int st = 0; st < 4; ++st)
          I[st * N + (size_t)k * np + q] = T(std::numeric_limits<double>::quiet_NaN());
  }
}

/* Formal solution for one ray and one frequency over the whole grid.
 * Writes I ([4][N], one Stokes component after the other) and Lambda* (N). */
template <class T>
void sweep_one(const oracle_problem& pb, const FieldsT<T>& f, const Ray& ray, int jf,
               T* I, double* lam) {
  Cx<double> t[4][9];
  tkq(ray.mu, ray.chi, t);
  const int s = ray.up ? 1 : -1;
  const int kb = ray.up ? 0 : pb.nz - 1;   // boundary plane
  boundary_plane(pb, ray, I, lam);
  if (pb.faces) {
    sweep_faces(pb, f, ray, t, pb.phi[jf], I, lam);
    return;
  }
  for (int step = 1; step < pb.nz; ++step) {
    const int k = kb + s * step;
    for (int j = 0; j < pb.ny; ++j)
      for (int i = 0; i < pb.nx; ++i) node_update(pb, f, ray, t, pb.phi[jf], k, i, j, I, lam);
  }
}

/* -------------------------------------------------------------------------- */
/* Reverse-mode differentiation of the formal solution.                       */
/* -------------------------------------------------------------------------- */
/* A real number that records every operation applied to it on the calling
 * thread's tape, so that one backward pass over the tape gives the derivative of
 * a result with respect to each input (reverse-mode automatic differentiation).
 * Inputs ("leaves") carry ids 0 .. nleaf-1 and are not on the tape; the k-th
 * recorded operation has id nleaf + k; id -1 marks a constant. */
struct Tape {
  struct Op {
    int a, b;        // ids of the operands (-1: none or constant)
    double da, db;   // partial derivatives of the result with respect to them
  };
  std::vector<Op> ops;
  int nleaf = 0;
};
static thread_local Tape* g_tape __attribute__((tls_model("initial-exec"))) = nullptr;

struct Rv {
  double v = 0.0;
  int id = -1;
  Rv() = default;
  Rv(double x) : v(x), id(-1) {}
};
inline double rp(const Rv& x) { return x.v; }

inline Rv record(double v, int a, double da, int b, double db) {
  Rv r(v);
  if (a < 0 && b < 0) return r;
  g_tape->ops.push_back({a, b, da, db});
  r.id = g_tape->nleaf + (int)g_tape->ops.size() - 1;
  return r;
}
inline Rv operator+(const Rv& x, const Rv& y) { return record(x.v + y.v, x.id, 1.0, y.id, 1.0); }
inline Rv operator-(const Rv& x, const Rv& y) { return record(x.v - y.v, x.id, 1.0, y.id, -1.0); }
inline Rv operator*(const Rv& x, const Rv& y) { return record(x.v * y.v, x.id, y.v, y.id, x.v); }
inline Rv operator/(const Rv& x, const Rv& y) {
  const double q = x.v / y.v;
  return record(q, x.id, 1.0 / y.v, y.id, -q / y.v);
}
inline Rv operator-(const Rv& x) { return record(-x.v, x.id, -1.0, -1, 0.0); }
inline Rv& operator+=(Rv& x, const Rv& y) { return x = x + y; }
inline Rv& operator-=(Rv& x, const Rv& y) { return x = x - y; }
inline Rv exp(const Rv& x) {
  const double e = std::exp(x.v);
  return record(e, x.id, e, -1, 0.0);
}

/* Backward pass over the tape: adj_out holds dL/d(result) for each recorded
 * operation on entry (indexed id - nleaf); the derivatives reaching the inputs are
 * added to leafadj (indexed by id). */
void backward(const Tape& tape, std::vector<double>& adj, double* leafadj) {
  auto send = [&](int id, double v) {
    if (id < 0) return;
    if (id < tape.nleaf)
      leafadj[id] += v;
    else
      adj[id - tape.nleaf] += v;
  };
  for (long k = (long)tape.ops.size() - 1; k >= 0; --k) {
    const double a = adj[k];
    if (a == 0.0) continue;
    const Tape::Op& op = tape.ops[k];
    send(op.a, a * op.da);
    send(op.b, a * op.db);
  }
}

double freq_norm(const oracle_problem& pb) {
  double s = 0.0;
  for (int j = 0; j < pb.nfreq; ++j) s += pb.wfreq[j] * pb.phi[j];
  return s;
}

/* Eq. 1 on the discrete quadrature: add w_Omega W_j sum_i T^K_Q(i) I_i to J,
 * and w_Omega W_j Lambda* to the angle-frequency averaged Lambda*. */
void accumulate_j(const Ray& ray, double Wj, const double* I,
                  size_t sp, size_t sc, const double* lam, size_t N, double* jkq) {
  /* I_i at point p is I[p * sp + i * sc] */
  Cx<double> t[4][9];
  tkq(ray.mu, ray.chi, t);
  const double w = ray.w * Wj;
  for (size_t p = 0; p < N; ++p) {
    Cx<double> J[9];
    for (int s = 0; s < 9; ++s) J[s] = Cx<double>{0.0, 0.0};
    for (int K = 0; K <= 2; ++K)
      for (int Q = 0; Q <= K; ++Q)
        for (int st = 0; st < 4; ++st) {
          const Cx<double>& tt = t[st][kq(K, Q)];
          J[kq(K, Q)].re += tt.re * I[p * sp + st * sc];
          J[kq(K, Q)].im += tt.im * I[p * sp + st * sc];
        }
    jkq[0 * N + p] += w * J[kq(0, 0)].re;
    jkq[1 * N + p] += w * J[kq(1, 0)].re;
    jkq[2 * N + p] += w * J[kq(1, 1)].re;
    jkq[3 * N + p] += w * J[kq(1, 1)].im;
    jkq[4 * N + p] += w * J[kq(2, 0)].re;
    jkq[5 * N + p] += w * J[kq(2, 1)].re;
    jkq[6 * N + p] += w * J[kq(2, 1)].im;
    jkq[7 * N + p] += w * J[kq(2, 2)].re;
    jkq[8 * N + p] += w * J[kq(2, 2)].im;
    if (lam) jkq[9 * N + p] += w * lam[p];
  }
}

bool valid_problem(const oracle_problem* pb) {
  if (!pb || pb->nx < 1 || pb->ny < 1 || pb->nz < 2 || pb->nmu < 1 || pb->nchi < 1 ||
      pb->nfreq < 1 || !pb->z || !pb->mu || !pb->wmu || !pb->phi || !pb->wfreq ||
      (pb->interp != 0 && pb->interp != 1) || (pb->control != 0 && pb->control != 1) ||
      (pb->faces != 0 && pb->faces != 1) || (pb->faces == 1 && pb->interp != 0))
    return false;
  for (int k = 1; k < pb->nz; ++k)
    if (!(pb->z[k] > pb->z[k - 1])) return false;
  for (int a = 0; a < pb->nmu; ++a)
    if (!(pb->mu[a] > 0.0 && pb->mu[a] <= 1.0)) return false;
  return true;
}

int nthreads_of(int req) {
#ifdef _OPENMP
  return req > 0 ? req : omp_get_max_threads();
#else
  (void)req;
  return 1;
#endif
}

/* Long characteristics: integrate along the straight ray from the boundary to
 * every grid point, interpolating only the material (never I) at the plane
 * crossings, with the same BESSER step per segment. */
void lc_one(const oracle_problem& pb, const FieldsT<double>& f, const Ray& ray, int jf,
            double* Iout) {
  const int nx = pb.nx, ny = pb.ny, nz = pb.nz;
  const size_t np = (size_t)nx * ny, N = np * nz;
  const double dx = pb.lx / nx, dy = pb.ly / ny;
  const double phi = pb.phi[jf];
  Cx<double> t[4][9];
  tkq(ray.mu, ray.chi, t);
  const int s = ray.up ? 1 : -1;
  const int kb = ray.up ? 0 : nz - 1;
  struct Node {
    double kap, eta[6], eps[6];
    double ds;  // path length from the previous node
  };
  std::vector<Node> path;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t pO = (size_t)k * np + (size_t)j * nx + i;
        const int nsteps = s * (k - kb);  // planes between boundary and O
        /* nodes from the boundary crossing (m = 0) to O (m = nsteps), plus the
         * downwind crossing beyond O when it exists */
        const int kend = k + s;
        const bool hasP = (kend >= 0 && kend < nz);
        const int nnodes = nsteps + 1 + (hasP ? 1 : 0);
        path.assign(nnodes, Node());
        for (int m = 0; m < nnodes; ++m) {
          const int kk = kb + s * m;
          const double dist = (pb.z[kk] - pb.z[k]) / ray.mu;  // signed path from O
          const double fx = i + dist * ray.sx / dx, fy = j + dist * ray.sy / dy;
          Node& nd = path[m];
          nd.kap = interp_plane(f.kappa + (size_t)kk * np, nx, ny, fx, fy, pb.interp);
          for (int c = 0; c < 6; ++c) {
            nd.eta[c] = interp_plane(f.prop + c * N + (size_t)kk * np, nx, ny, fx, fy, pb.interp);
            nd.eps[c] = interp_plane(f.emis + c * N + (size_t)kk * np, nx, ny, fx, fy, pb.interp);
          }
          nd.ds = (m == 0) ? 0.0 : std::fabs((pb.z[kk] - pb.z[kk - s]) / ray.mu);
        }
        double Ic[4] = {ray.up ? pb.i_bottom : 0.0, 0.0, 0.0, 0.0};
        for (int m = 1; m <= nsteps; ++m) {
          const Node &nM = path[m - 1], &nO = path[m];
          const bool hp = (m + 1 < nnodes);
          const Node* nP = hp ? &path[m + 1] : nullptr;
          const double tauMO = 0.5 * (nM.kap + nO.kap) * phi * nO.ds;
          const double tauOP = hp ? 0.5 * (nO.kap + nP->kap) * phi * nP->ds : 0.0;
          double SM[4], SO[4], SP[4], cM[4], eM[6], eO[6], eP[6], hM[6], hO[6];
          for (int c = 0; c < 6; ++c) {
            eM[c] = nM.eps[c] * phi; eO[c] = nO.eps[c] * phi; eP[c] = hp ? nP->eps[c] * phi : 0.0;
            hM[c] = nM.eta[c] * phi; hO[c] = nO.eta[c] * phi;
          }
          for (int st = 0; st < 4; ++st) {
            SM[st] = emission(t, st, eM, pb.w2) / (nM.kap * phi);
            SO[st] = emission(t, st, eO, pb.w2) / (nO.kap * phi);
            SP[st] = hp ? emission(t, st, eP, pb.w2) / (nP->kap * phi) : 0.0;
            cM[st] = hp ? control_point(pb.control, SM[st], SO[st], SP[st], tauMO, tauOP)
                        : 0.5 * (SM[st] + SO[st]);
          }
          double KM[4][4], KO[4][4];
          kprime(hM, nM.kap * phi, KM);
          kprime(hO, nO.kap * phi, KO);
          const Coef<double> cf = coefficients(tauMO);
          double b[4], A[4][4], x[4];
          for (int a = 0; a < 4; ++a) {
            double acc = cf.e * Ic[a];
            for (int c = 0; c < 4; ++c) acc -= cf.psiM * KM[a][c] * Ic[c];
            b[a] = acc + cf.omM * SM[a] + cf.omO * SO[a] + cf.omC * cM[a];
            for (int c = 0; c < 4; ++c) A[a][c] = (a == c ? 1.0 : 0.0) + cf.psiO * KO[a][c];
          }
          gauss_solve<double, 4>(A, b, x);
          for (int st = 0; st < 4; ++st) Ic[st] = x[st];
        }
        for (int st = 0; st < 4; ++st) Iout[4 * pO + st] = Ic[st];
      }
}

/* Trilinear interpolation of a node field at a point in cell units (fx, fy; x and y
 * periodic) and height z (inside [z_0, z_{nz-1}]). */
double trilinear(const oracle_problem& pb, const double* f, double fx, double fy, double z) {
  const int nx = pb.nx, ny = pb.ny, nz = pb.nz;
  const size_t np = (size_t)nx * ny;
  int kk = 0;
  while (kk < nz - 2 && pb.z[kk + 1] <= z) ++kk;
  const double tz = std::min(1.0, std::max(0.0, (z - pb.z[kk]) / (pb.z[kk + 1] - pb.z[kk])));
  const double fi = std::floor(fx), fj = std::floor(fy);
  const double tx = fx - fi, ty = fy - fj;
  const int i0 = wrap((long)fi, nx), i1 = wrap((long)fi + 1, nx);
  const int j0 = wrap((long)fj, ny), j1 = wrap((long)fj + 1, ny);
  double v = 0.0;
  for (int dk = 0; dk < 2; ++dk) {
    const double* g = f + (size_t)(kk + dk) * np;
    const double pl = (1.0 - tx) * (1.0 - ty) * g[j0 * nx + i0] + tx * (1.0 - ty) * g[j0 * nx + i1] +
                      (1.0 - tx) * ty * g[j1 * nx + i0] + tx * ty * g[j1 * nx + i1];
    v += (dk ? tz : 1.0 - tz) * pl;
  }
  return v;
}

/* Long characteristics through the trilinear medium: the straight ray from the
 * boundary to node O is cut at every face of the grid it crosses (x, y and z planes;
 * beyond O, at the first face crossed downwind, the point P of the last step), each
 * piece is split into nsub equal parts, the transfer coefficients at the cuts are the
 * trilinear interpolation of the node values, and Eq. fsbez with BESSER control
 * points is applied piece by piece.  As nsub grows this tends to the exact solution
 * of the transfer equation in that medium. */
void lc_fine_one(const oracle_problem& pb, const FieldsT<double>& f, const Ray& ray, int jf,
                 int nsub, double* Iout) {
  const int nx = pb.nx, ny = pb.ny, nz = pb.nz;
  const size_t np = (size_t)nx * ny, N = np * nz;
  const double dx = pb.lx / nx, dy = pb.ly / ny;
  const double phi = pb.phi[jf];
  Cx<double> t[4][9];
  tkq(ray.mu, ray.chi, t);
  const int kb = ray.up ? 0 : nz - 1;
  const double amu = std::fabs(ray.mu);
  std::vector<double> cuts, pts;
  struct Pt {
    double kap, eta[6], eps[6];
  };
  std::vector<Pt> path;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t pO = (size_t)k * np + (size_t)j * nx + i;
        if (k == kb) {
          Iout[4 * pO] = ray.up ? pb.i_bottom : 0.0;
          Iout[4 * pO + 1] = Iout[4 * pO + 2] = Iout[4 * pO + 3] = 0.0;
          continue;
        }
        /* distances upwind from O (positive) of the face crossings, O at 0 */
        const double send = std::fabs(pb.z[k] - pb.z[kb]) / amu;
        cuts.assign(1, 0.0);
        for (int kk = k; kk != kb;) {
          kk += ray.up ? -1 : 1;
          cuts.push_back(std::fabs(pb.z[k] - pb.z[kk]) / amu);
        }
        if (ray.sx != 0.0)
          for (int m = 1; m * dx / std::fabs(ray.sx) < send; ++m) cuts.push_back(m * dx / std::fabs(ray.sx));
        if (ray.sy != 0.0)
          for (int m = 1; m * dy / std::fabs(ray.sy) < send; ++m) cuts.push_back(m * dy / std::fabs(ray.sy));
        std::sort(cuts.begin(), cuts.end());
        std::vector<double> u;
        for (double c : cuts)
          if (u.empty() || c - u.back() > 1e-12 * send) u.push_back(c);
        u.back() = send;
        /* the downwind piece: first face crossed beyond O, if inside the grid */
        FacePoint fpP;
        const bool hasP = first_face(pb, ray, i, j, k, +1, fpP);
        pts.clear();
        for (size_t a = u.size() - 1; a >= 1; --a)
          for (int q = 0; q < nsub; ++q) pts.push_back(u[a] - (u[a] - u[a - 1]) * q / nsub);
        pts.push_back(0.0);
        if (hasP) pts.push_back(-fpP.ds / nsub);
        path.resize(pts.size());
        for (size_t a = 0; a < pts.size(); ++a) {
          const double sd = pts[a];
          const double fx = i - sd * ray.sx / dx, fy = j - sd * ray.sy / dy;
          const double z = pb.z[k] - sd * ray.mu;
          Pt& pt = path[a];
          pt.kap = trilinear(pb, f.kappa, fx, fy, z);
          for (int c = 0; c < 6; ++c) {
            pt.eta[c] = trilinear(pb, f.prop + c * N, fx, fy, z);
            pt.eps[c] = trilinear(pb, f.emis + c * N, fx, fy, z);
          }
        }
        const size_t nO = pts.size() - (hasP ? 2 : 1);   // index of O
        double Ic[4] = {ray.up ? pb.i_bottom : 0.0, 0.0, 0.0, 0.0};
        for (size_t m = 1; m <= nO; ++m) {
          const Pt &nM = path[m - 1], &nO_ = path[m];
          const bool hp = m + 1 < path.size();
          const Pt* nP = hp ? &path[m + 1] : nullptr;
          const double dsM = pts[m - 1] - pts[m], dsP = hp ? pts[m] - pts[m + 1] : 0.0;
          const double tauMO = 0.5 * (nM.kap + nO_.kap) * phi * dsM;
          const double tauOP = hp ? 0.5 * (nO_.kap + nP->kap) * phi * dsP : 0.0;
          double SM[4], SO[4], SP[4], cM[4], eM[6], eO[6], eP[6], hM[6], hO[6];
          for (int c = 0; c < 6; ++c) {
            eM[c] = nM.eps[c] * phi; eO[c] = nO_.eps[c] * phi; eP[c] = hp ? nP->eps[c] * phi : 0.0;
            hM[c] = nM.eta[c] * phi; hO[c] = nO_.eta[c] * phi;
          }
          for (int st = 0; st < 4; ++st) {
            SM[st] = emission(t, st, eM, pb.w2) / (nM.kap * phi);
            SO[st] = emission(t, st, eO, pb.w2) / (nO_.kap * phi);
            SP[st] = hp ? emission(t, st, eP, pb.w2) / (nP->kap * phi) : 0.0;
            cM[st] = hp ? control_point(pb.control, SM[st], SO[st], SP[st], tauMO, tauOP)
                        : 0.5 * (SM[st] + SO[st]);
          }
          double KM[4][4], KO[4][4];
          kprime(hM, nM.kap * phi, KM);
          kprime(hO, nO_.kap * phi, KO);
          const Coef<double> cf = coefficients(tauMO);
          double b[4], A[4][4], x[4];
          for (int a = 0; a < 4; ++a) {
            double acc = cf.e * Ic[a];
            for (int c = 0; c < 4; ++c) acc -= cf.psiM * KM[a][c] * Ic[c];
            b[a] = acc + cf.omM * SM[a] + cf.omO * SO[a] + cf.omC * cM[a];
            for (int c = 0; c < 4; ++c) A[a][c] = (a == c ? 1.0 : 0.0) + cf.psiO * KO[a][c];
          }
          gauss_solve<double, 4>(A, b, x);
          for (int st = 0; st < 4; ++st) Ic[st] = x[st];
        }
        for (int st = 0; st < 4; ++st) Iout[4 * pO + st] = Ic[st];
      }
}

}  // namespace

extern "C" {

/* Formal solution of the selected rays and frequencies.
 *   jkq   [10][N] accumulated (J00, J10, Re/Im J11, J20, Re/Im J21, Re/Im J22, Lambda-bar)
 *   itop  [nray_sel][nfreq_sel][ny][nx][4]: I at the top plane (upward rays; zero for others)
 *   ifull [nray_sel][nfreq_sel][N][4]:       I everywhere
 *   lamf  [nray_sel][nfreq_sel][N]:          Lambda* everywhere
 * Any output may be NULL.  Returns 0, or -1 for an invalid problem. */
int oracle_fs_sweep(const oracle_problem* pb, const double* kappa, const double* prop,
                    const double* emis, int nray_sel, const int* rays, int nfreq_sel,
                    const int* freqs, double* jkq, double* itop, double* ifull, double* lamf,
                    int nthreads) {
  if (!valid_problem(pb) || !kappa || !prop || !emis || nray_sel < 0 || nfreq_sel < 0) return -1;
  const size_t np = (size_t)pb->nx * pb->ny, N = np * pb->nz;
  const int nrays = 2 * pb->nmu * pb->nchi;
  for (int r = 0; r < nray_sel; ++r)
    if (rays[r] < 0 || rays[r] >= nrays) return -1;
  for (int q = 0; q < nfreq_sel; ++q)
    if (freqs[q] < 0 || freqs[q] >= pb->nfreq) return -1;
  const double fnorm = freq_norm(*pb);
  const FieldsT<double> f{kappa, prop, emis};
  const int nt = nthreads_of(nthreads);
  const long npairs = (long)nray_sel * nfreq_sel;
  std::vector<std::vector<double>> jpart(jkq ? nt : 0);
  if (itop) std::memset(itop, 0, sizeof(double) * npairs * np * 4);
#pragma omp parallel num_threads(nt)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double> I(4 * N), lam(N);
    if (jkq) jpart[tid].assign(10 * N, 0.0);
#pragma omp for schedule(static)
    for (long pair = 0; pair < npairs; ++pair) {
      const int r = rays[pair / nfreq_sel], jf = freqs[pair % nfreq_sel];
      const Ray ray = make_ray(*pb, r);
      sweep_one<double>(*pb, f, ray, jf, I.data(), lam.data());
      if (jkq)
        accumulate_j(ray, pb->wfreq[jf] * pb->phi[jf] / fnorm, I.data(), 1, N, lam.data(),
                     N, jpart[tid].data());
      if (itop && ray.up)
        for (size_t q = 0; q < np; ++q)
          for (int st = 0; st < 4; ++st)
            itop[(pair * np + q) * 4 + st] = I[st * N + (size_t)(pb->nz - 1) * np + q];
      if (ifull)
        for (size_t q = 0; q < N; ++q)
          for (int st = 0; st < 4; ++st) ifull[(pair * N + q) * 4 + st] = I[st * N + q];
      if (lamf) std::memcpy(lamf + pair * N, lam.data(), sizeof(double) * N);
    }
  }
  if (jkq)
    for (int t = 0; t < nt; ++t)
      for (size_t q = 0; q < 10 * N; ++q) jkq[q] += jpart[t][q];
  return 0;
}

/* Complex-step variant: the inputs are (kappa + i h dkappa, prop + i h dprop,
 * emis + i h demis); returns the real and imaginary parts of I at the top
 * plane, [nray_sel][nfreq_sel][ny][nx][4], so Im/h is the exact directional
 * derivative of the emergent Stokes vector along (dkappa, dprop, demis). */
int oracle_fs_sweep_cs(const oracle_problem* pb, const double* kappa, const double* prop,
                       const double* emis, const double* dkappa, const double* dprop,
                       const double* demis, double h, int nray_sel, const int* rays,
                       int nfreq_sel, const int* freqs, double* itop_re, double* itop_im,
                       int nthreads) {
  if (!valid_problem(pb) || pb->faces || !kappa || !prop || !emis || !dkappa || !dprop ||
      !demis)
    return -1;
  const size_t np = (size_t)pb->nx * pb->ny, N = np * pb->nz;
  std::vector<cd> ck(N), cp(6 * N), ce(6 * N);
  for (size_t p = 0; p < N; ++p) ck[p] = cd(kappa[p], h * dkappa[p]);
  for (size_t p = 0; p < 6 * N; ++p) {
    cp[p] = cd(prop[p], h * dprop[p]);
    ce[p] = cd(emis[p], h * demis[p]);
  }
  const FieldsT<cd> f{ck.data(), cp.data(), ce.data()};
  const long npairs = (long)nray_sel * nfreq_sel;
  std::memset(itop_re, 0, sizeof(double) * npairs * np * 4);
  std::memset(itop_im, 0, sizeof(double) * npairs * np * 4);
  const int nt = nthreads_of(nthreads);
#pragma omp parallel num_threads(nt)
  {
    std::vector<cd> I(4 * N);
#pragma omp for schedule(static)
    for (long pair = 0; pair < npairs; ++pair) {
      const int r = rays[pair / nfreq_sel], jf = freqs[pair % nfreq_sel];
      const Ray ray = make_ray(*pb, r);
      if (!ray.up) continue;
      sweep_one<cd>(*pb, f, ray, jf, I.data(), nullptr);
      const size_t top = (size_t)(pb->nz - 1) * np;
      for (size_t q = 0; q < np; ++q)
        for (int st = 0; st < 4; ++st) {
          itop_re[(pair * np + q) * 4 + st] = I[st * N + top + q].real();
          itop_im[(pair * np + q) * 4 + st] = I[st * N + top + q].imag();
        }
    }
  }
  return 0;
}

/* Reverse-mode derivative of L = sum over the selected (ray, frequency) pairs, top
 * nodes and Stokes parameters of seed * I_top, with respect to every transfer
 * coefficient (the function differentiated is the formal solution of Sect. 3.3,
 * Eqs. fsbez and kappa, with its BESSER control points and Table 1 branches).  For
 * each upward (ray, frequency) pair the forward sweep stores the whole Stokes field;
 * the planes are then walked from the top down, and on each plane every node update
 * (node_update, the same code as the forward solution) is recorded on a tape whose
 * inputs are the upwind plane's Stokes vectors and the coefficients of the upwind,
 * own and downwind planes; one backward pass per node sends dL/dI_O to those inputs,
 * so dL/dI reaches the upwind plane before that plane is walked.  Branches (control
 * point, series or closed form, pivots) are those of the forward evaluation.
 *   seed   [nray_sel][nfreq_sel][ny][nx][4]  (entries of downward rays are ignored)
 *   g_kappa [N], g_prop [6][N], g_emis [6][N] are added to.
 * Returns 0, or -1 for an invalid problem. */
int oracle_fs_adjoint(const oracle_problem* pb, const double* kappa, const double* prop,
                      const double* emis, int nray_sel, const int* rays, int nfreq_sel,
                      const int* freqs, const double* seed, double* g_kappa, double* g_prop,
                      double* g_emis, int nthreads) {
  if (!valid_problem(pb) || pb->faces || !kappa || !prop || !emis || !seed || !g_kappa ||
      !g_prop || !g_emis || nray_sel < 0 || nfreq_sel < 0)
    return -1;
  const int nrays = 2 * pb->nmu * pb->nchi;
  for (int r = 0; r < nray_sel; ++r)
    if (rays[r] < 0 || rays[r] >= nrays) return -1;
  for (int q = 0; q < nfreq_sel; ++q)
    if (freqs[q] < 0 || freqs[q] >= pb->nfreq) return -1;
  const int nx = pb->nx, ny = pb->ny, nz = pb->nz;
  const size_t np = (size_t)nx * ny, N = np * nz;
  const FieldsT<double> f{kappa, prop, emis};
  const int nt = nthreads_of(nthreads);
  const long npairs = (long)nray_sel * nfreq_sel;
  /* gradient rows: 0 kappa, 1..6 propagation matrix, 7..12 emissivities */
  std::vector<std::vector<double>> gpart(nt);
#pragma omp parallel num_threads(nt)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    std::vector<double>& g = gpart[tid];
    g.assign(13 * N, 0.0);
    std::vector<double> I(4 * N), lamI(4 * N);
    std::vector<Rv> Ir(4 * N), kr(N), pr(6 * N), er(6 * N);
    Tape tape;
    g_tape = &tape;
    /* leaf ids of one plane step: Stokes vectors of the upwind plane [4][np], then the
     * 13 coefficients of the upwind, own and downwind planes [3][13][np] */
    tape.nleaf = (int)(43 * np);
    std::vector<double> leafadj(43 * np), adj;
    auto leaf_coef = [&](int pl, int c, size_t q) { return (int)((4 + 13 * pl + c) * np + q); };
#pragma omp for schedule(static)
    for (long pair = 0; pair < npairs; ++pair) {
      const int r = rays[pair / nfreq_sel], jf = freqs[pair % nfreq_sel];
      const Ray ray = make_ray(*pb, r);
      if (!ray.up) continue;
      sweep_one<double>(*pb, f, ray, jf, I.data(), nullptr);
      for (size_t p = 0; p < 4 * N; ++p) Ir[p] = Rv(I[p]);
      for (size_t p = 0; p < N; ++p) kr[p] = Rv(kappa[p]);
      for (size_t p = 0; p < 6 * N; ++p) {
        pr[p] = Rv(prop[p]);
        er[p] = Rv(emis[p]);
      }
      const FieldsT<Rv> fr{kr.data(), pr.data(), er.data()};
      std::fill(lamI.begin(), lamI.end(), 0.0);
      for (size_t q = 0; q < np; ++q)
        for (int st = 0; st < 4; ++st)
          lamI[st * N + (size_t)(nz - 1) * np + q] = seed[(pair * np + q) * 4 + st];
      Cx<double> t[4][9];
      tkq(ray.mu, ray.chi, t);
      for (int k = nz - 1; k >= 1; --k) {
        for (size_t q = 0; q < np; ++q) {
          for (int st = 0; st < 4; ++st) Ir[st * N + (size_t)(k - 1) * np + q].id = (int)(st * np + q);
          for (int pl = 0; pl < 3; ++pl) {
            const int kk = k - 1 + pl;
            if (kk >= nz) continue;
            const size_t pk = (size_t)kk * np + q;
            kr[pk].id = leaf_coef(pl, 0, q);
            for (int c = 0; c < 6; ++c) {
              pr[c * N + pk].id = leaf_coef(pl, 1 + c, q);
              er[c * N + pk].id = leaf_coef(pl, 7 + c, q);
            }
          }
        }
        std::fill(leafadj.begin(), leafadj.end(), 0.0);
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i) {
            const size_t pO = (size_t)k * np + (size_t)j * nx + i;
            tape.ops.clear();
            node_update<Rv>(*pb, fr, ray, t, pb->phi[jf], k, i, j, Ir.data(), nullptr);
            adj.assign(tape.ops.size(), 0.0);
            for (int st = 0; st < 4; ++st) {
              const int id = Ir[st * N + pO].id;
              const double l = lamI[st * N + pO];
              if (id >= tape.nleaf)
                adj[id - tape.nleaf] += l;
              else if (id >= 0)
                leafadj[id] += l;
            }
            backward(tape, adj, leafadj.data());
          }
        for (size_t q = 0; q < np; ++q) {
          for (int st = 0; st < 4; ++st)
            lamI[st * N + (size_t)(k - 1) * np + q] += leafadj[st * np + q];
          for (int pl = 0; pl < 3; ++pl) {
            const int kk = k - 1 + pl;
            if (kk >= nz) continue;
            const size_t pk = (size_t)kk * np + q;
            for (int c = 0; c < 13; ++c) g[c * N + pk] += leafadj[leaf_coef(pl, c, q)];
          }
        }
      }
    }
  }
  for (int th = 0; th < nt; ++th)
    for (size_t p = 0; p < N; ++p) {
      g_kappa[p] += gpart[th][p];
      for (int c = 0; c < 6; ++c) {
        g_prop[c * N + p] += gpart[th][(1 + c) * N + p];
        g_emis[c * N + p] += gpart[th][(7 + c) * N + p];
      }
    }
  return 0;
}

/* Long-characteristics solution at every point, [nray_sel][nfreq_sel][N][4]. */
int oracle_lc_sweep(const oracle_problem* pb, const double* kappa, const double* prop,
                    const double* emis, int nray_sel, const int* rays, int nfreq_sel,
                    const int* freqs, double* ifull) {
  if (!valid_problem(pb) || pb->faces || !ifull) return -1;
  const size_t N = (size_t)pb->nx * pb->ny * pb->nz;
  const FieldsT<double> f{kappa, prop, emis};
  for (int r = 0; r < nray_sel; ++r)
    for (int q = 0; q < nfreq_sel; ++q)
      lc_one(*pb, f, make_ray(*pb, rays[r]), freqs[q], ifull + ((size_t)r * nfreq_sel + q) * N * 4);
  return 0;
}

/* Long characteristics through the trilinear medium (lc_fine_one) at every point,
 * [nray_sel][nfreq_sel][N][4]; nsub >= 1 parts per piece between face crossings. */
int oracle_lc_fine_sweep(const oracle_problem* pb, const double* kappa, const double* prop,
                         const double* emis, int nray_sel, const int* rays, int nfreq_sel,
                         const int* freqs, int nsub, double* ifull, int nthreads) {
  if (!valid_problem(pb) || !ifull || nsub < 1) return -1;
  const size_t N = (size_t)pb->nx * pb->ny * pb->nz;
  const FieldsT<double> f{kappa, prop, emis};
  const long npairs = (long)nray_sel * nfreq_sel;
  const int nt = nthreads_of(nthreads);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (long pair = 0; pair < npairs; ++pair)
    lc_fine_one(*pb, f, make_ray(*pb, rays[pair / nfreq_sel]), freqs[pair % nfreq_sel], nsub,
                ifull + (size_t)pair * N * 4);
  return 0;
}

/* Eq. 1 from a stored block of Stokes vectors, [nray][nf][N][4], for the rays
 * ray0..ray0+nray-1 and frequencies f0..f0+nf-1; lam [nray][nf][N] or NULL. */
int oracle_jkq_accumulate(const oracle_problem* pb, int ray0, int nray, int f0, int nf,
                          const double* stokes, const double* lam, double* jkq) {
  if (!valid_problem(pb) || !stokes || !jkq) return -1;
  const int nrays = 2 * pb->nmu * pb->nchi;
  if (ray0 < 0 || nray < 0 || ray0 + nray > nrays || f0 < 0 || nf < 0 || f0 + nf > pb->nfreq)
    return -1;
  const size_t N = (size_t)pb->nx * pb->ny * pb->nz;
  const double fnorm = freq_norm(*pb);
  for (int r = 0; r < nray; ++r) {
    const Ray ray = make_ray(*pb, ray0 + r);
    for (int q = 0; q < nf; ++q) {
      const int jf = f0 + q;
      const size_t off = ((size_t)r * nf + q) * N;
      accumulate_j(ray, pb->wfreq[jf] * pb->phi[jf] / fnorm, stokes + 4 * off, 4, 1,
                   lam ? lam + off : nullptr, N, jkq);
    }
  }
  return 0;
}

/* The two-level (J_l = 0 -> J_u = 1) statistical equilibrium written as
 * L(rho) rho = f (Sect. 2, Eq. nonlte), with the source-function multipoles
 * S^K_Q standing for the unknowns, stored [6][N] in the order
 * S00, S20, Re S21, Im S21, Re S22, Im S22:
 *   K = 0:  S00 - (1-eps) J00                                     = f_0
 *   K = 2:  [1 + delta (1-eps)] S2_Q + i (1-eps) H sum_Q' Kmat_QQ'(b) S2_Q'
 *              - (1-eps) w2 conj(J2_Q)                             = f2_Q   (Q = -2..2)
 * with Kmat the matrix of b.J in the rank-2 representation; f = (eps B, 0, ...)
 * for the problem itself, another right-hand side on the coarse grids of the
 * multigrid iteration (Sect. 5, Eq. mgcsfy).  Components with Q < 0 follow from
 * X_{-Q} = (-1)^Q conj(X_Q) for S, J and f alike. */
namespace {

struct SeeAtom {
  double eps_c, delta2, w2, planck;
  const double* hanle;
  const double* bhat;
};

/* Five K = 2 components Q = -2..2 from the three stored Q >= 0 ones. */
void unfold_k2(double x0, double re1, double im1, double re2, double im2, cd out[5]) {
  out[2] = cd(x0, 0.0);
  out[3] = cd(re1, im1);
  out[4] = cd(re2, im2);
  out[1] = -std::conj(out[3]);
  out[0] = std::conj(out[4]);
}

/* The 5x5 matrix acting on S2_Q at point p. */
void k2_matrix(const SeeAtom& at, size_t N, size_t p, cd A[5][5]) {
  const double H = at.hanle ? at.hanle[p] : 0.0;
  const double bx = at.bhat ? at.bhat[0 * N + p] : 0.0, by = at.bhat ? at.bhat[1 * N + p] : 0.0,
               bz = at.bhat ? at.bhat[2 * N + p] : 1.0;
  const double om = 1.0 - at.eps_c;
  for (int a = 0; a < 5; ++a)
    for (int c = 0; c < 5; ++c) A[a][c] = 0.0;
  for (int qi = 0; qi < 5; ++qi) {
    const int Q = qi - 2;
    A[qi][qi] += 1.0 + at.delta2 * om;
    A[qi][qi] += cd(0.0, om * H) * cd(bz * Q, 0.0);   // b_z Q on the diagonal
  }
  for (int qpi = 0; qpi < 5; ++qpi) {
    const int Qp = qpi - 2;
    if (Qp + 1 <= 2) {  // <Q'+1| b.J |Q'>
      const cd v = 0.5 * cd(bx, -by) * std::sqrt(6.0 - Qp * (Qp + 1.0));
      A[qpi + 1][qpi] += cd(0.0, om * H) * v;
    }
    if (Qp - 1 >= -2) {  // <Q'-1| b.J |Q'>
      const cd v = 0.5 * cd(bx, by) * std::sqrt(6.0 - Qp * (Qp - 1.0));
      A[qpi - 1][qpi] += cd(0.0, om * H) * v;
    }
  }
}

void f_at(const SeeAtom& at, const double* rhs, size_t N, size_t p, double& f0, cd f2[5]) {
  if (rhs) {
    f0 = rhs[p];
    unfold_k2(rhs[1 * N + p], rhs[2 * N + p], rhs[3 * N + p], rhs[4 * N + p], rhs[5 * N + p], f2);
  } else {
    f0 = at.eps_c * at.planck;
    for (int q = 0; q < 5; ++q) f2[q] = 0.0;
  }
}

}  // namespace

/* One Jacobi update at every point:
 *   K = 0 (Jacobi with Lambda-bar):
 *     S00 <- [(1-eps)(J00 - Lbar S00_old) + f_0] / [1 - (1-eps) Lbar]
 *   K = 2 (Lambda iteration with Hanle rotation): solve the K = 2 equations above
 *     for S2 with J2 from the last formal solution.
 * rhs [6][N] or NULL for (eps B, 0, ...).  emis_new (= kappa * S_new) may be NULL;
 * rc = max |dS00| / |S00_new|. */
int oracle_see_update(int n, const double* jkq, const double* s_old, double eps_c, double delta2,
                      double w2, double planck, const double* hanle, const double* bhat,
                      const double* rhs, const double* kappa, double* s_new, double* emis_new,
                      double* rc) {
  if (n < 0 || !jkq || !s_old || !s_new) return -1;
  const size_t N = (size_t)n;
  const SeeAtom at{eps_c, delta2, w2, planck, hanle, bhat};
  double rmax = 0.0;
  for (size_t p = 0; p < N; ++p) {
    const double J00 = jkq[0 * N + p], Lb = jkq[9 * N + p];
    const double so = s_old[p];
    double f0;
    cd f2[5];
    f_at(at, rhs, N, p, f0, f2);
    const double s00 = ((1.0 - eps_c) * (J00 - Lb * so) + f0) / (1.0 - (1.0 - eps_c) * Lb);
    cd J2[5];
    unfold_k2(jkq[4 * N + p], jkq[5 * N + p], jkq[6 * N + p], jkq[7 * N + p], jkq[8 * N + p], J2);
    cd A[5][5], b[5], x[5];
    k2_matrix(at, N, p, A);
    for (int qi = 0; qi < 5; ++qi) b[qi] = (1.0 - eps_c) * w2 * std::conj(J2[qi]) + f2[qi];
    /* complex Gaussian elimination with partial pivoting */
    for (int c = 0; c < 5; ++c) {
      int piv = c;
      for (int r = c + 1; r < 5; ++r)
        if (std::abs(A[r][c]) > std::abs(A[piv][c])) piv = r;
      if (piv != c) {
        for (int k = 0; k < 5; ++k) std::swap(A[c][k], A[piv][k]);
        std::swap(b[c], b[piv]);
      }
      for (int r = c + 1; r < 5; ++r) {
        const cd fct = A[r][c] / A[c][c];
        for (int k = c; k < 5; ++k) A[r][k] -= fct * A[c][k];
        b[r] -= fct * b[c];
      }
    }
    for (int r = 4; r >= 0; --r) {
      cd sacc = b[r];
      for (int k = r + 1; k < 5; ++k) sacc -= A[r][k] * x[k];
      x[r] = sacc / A[r][r];
    }
    s_new[0 * N + p] = s00;
    s_new[1 * N + p] = x[2].real();
    s_new[2 * N + p] = x[3].real();
    s_new[3 * N + p] = x[3].imag();
    s_new[4 * N + p] = x[4].real();
    s_new[5 * N + p] = x[4].imag();
    if (emis_new && kappa)
      for (int c = 0; c < 6; ++c) emis_new[c * N + p] = kappa[p] * s_new[c * N + p];
    const double rel = std::fabs(s00 - so) / std::fabs(s00);
    if (rel > rmax) rmax = rel;
  }
  if (rc) *rc = rmax;
  return 0;
}

/* The left-hand side L(rho) rho of the equations above at every point, [6][N],
 * for the multipoles s and the radiation field jkq of their formal solution. */
int oracle_see_operator(int n, const double* jkq, const double* s, double eps_c, double delta2,
                        double w2, const double* hanle, const double* bhat, double* out) {
  if (n < 0 || !jkq || !s || !out) return -1;
  const size_t N = (size_t)n;
  const SeeAtom at{eps_c, delta2, w2, 0.0, hanle, bhat};
  for (size_t p = 0; p < N; ++p) {
    out[p] = s[p] - (1.0 - eps_c) * jkq[p];
    cd S2[5], J2[5], A[5][5];
    unfold_k2(s[1 * N + p], s[2 * N + p], s[3 * N + p], s[4 * N + p], s[5 * N + p], S2);
    unfold_k2(jkq[4 * N + p], jkq[5 * N + p], jkq[6 * N + p], jkq[7 * N + p], jkq[8 * N + p], J2);
    k2_matrix(at, N, p, A);
    cd y[5];
    for (int a = 0; a < 5; ++a) {
      y[a] = -(1.0 - eps_c) * w2 * std::conj(J2[a]);
      for (int c = 0; c < 5; ++c) y[a] += A[a][c] * S2[c];
    }
    out[1 * N + p] = y[2].real();
    out[2 * N + p] = y[3].real();
    out[3 * N + p] = y[3].imag();
    out[4 * N + p] = y[4].real();
    out[5 * N + p] = y[4].imag();
  }
  return 0;
}

/* ---- single-step helpers, exported for the pin tests ---------------------- */

void oracle_coefficients(double tau, double* out6) {
  const Coef<double> c = coefficients(tau);
  out6[0] = c.e; out6[1] = c.psiM; out6[2] = c.psiO;
  out6[3] = c.omM; out6[4] = c.omO; out6[5] = c.omC;
}

double oracle_besser_cm(double yM, double yO, double yP, double hM, double hP) {
  return besser_cm(yM, yO, yP, hM, hP);
}

double oracle_parabolic_cm(double yM, double yO, double yP, double hM, double hP) {
  return parabolic_cm(yM, yO, yP, hM, hP);
}

double oracle_bezier1d(double ym, double y0, double yp, double t) {
  return bezier1d(ym, y0, yp, t);
}

double oracle_interp_plane(const double* f, int nx, int ny, double fx, double fy, int mode) {
  return interp_plane(f, nx, ny, fx, fy, mode);
}

/* T^K_Q(i, Omega) for all 9 (K, Q) slots (K=0; K=1, Q=-1..1; K=2, Q=-2..2). */
void oracle_tkq(double mu, double chi, double* re36, double* im36) {
  Cx<double> t[4][9];
  tkq(mu, chi, t);
  for (int i = 0; i < 4; ++i)
    for (int s = 0; s < 9; ++s) {
      re36[9 * i + s] = t[i][s].re;
      im36[9 * i + s] = t[i][s].im;
    }
}

/* Emission vector (eps_I, eps_Q, eps_U, eps_V) of one ray from the 6 multipoles. */
void oracle_emission(double mu, double chi, const double* e6, double w2, double* out4) {
  Cx<double> t[4][9];
  tkq(mu, chi, t);
  for (int i = 0; i < 4; ++i) out4[i] = emission(t, i, e6, w2);
}

void oracle_solve4(const double* A16, const double* b4, double* x4) {
  double A[4][4], b[4], x[4];
  for (int a = 0; a < 4; ++a) {
    b[a] = b4[a];
    for (int c = 0; c < 4; ++c) A[a][c] = A16[4 * a + c];
  }
  gauss_solve<double, 4>(A, b, x);
  for (int a = 0; a < 4; ++a) x4[a] = x[a];
}

}  // extern "C"
