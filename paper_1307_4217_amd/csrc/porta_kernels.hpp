// porta_kernels.hpp -- HIP kernels of the forward path for gfx950: table
// preparation, the plane step of the short-characteristics sweep, the
// ray/frequency reduction of J^K_Q and the stand-alone J accumulation (the
// statistical-equilibrium update is in porta_see.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "porta_math.hpp"

namespace porta {

constexpr int kMaxMu = 64;
constexpr int kUploadChunk = 240;   // doubles per upload launch (kernel-argument copy)

// ---------------------------------------------------------------------------
// Small host -> device uploads travel inside the kernel arguments, which the
// runtime copies at launch time; the host buffer can be reused at once and
// the copy is ordered on the caller's stream.
// ---------------------------------------------------------------------------
struct UploadChunk {
  double v[kUploadChunk];
  double* dst;
  int n;
};

__global__ void k_upload(const UploadChunk c) {
  const int t = threadIdx.x;
  if (t < c.n) c.dst[t] = c.v[t];
}

// Opt-in validity check of the transfer coefficients: flag[0] = 1 if some eta_I is
// not finite or not > 0, or some propagation-matrix or emission entry is not finite.
// Every writer stores the same value, so the unordered stores agree.
__global__ void k_zero_flag(int* flag) {
  if (threadIdx.x == 0) flag[0] = 0;
}

template <class T>
__global__ void __launch_bounds__(256) k_check_fields(const T* __restrict__ kappa,
                                                      const T* __restrict__ prop,
                                                      const T* __restrict__ emis, size_t N,
                                                      int* flag) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < N;
       p += (size_t)gridDim.x * blockDim.x) {
    bool bad = !(kappa[p] > T(0)) || !isfinite(kappa[p]);
#pragma unroll
    for (int c = 0; c < 6; ++c) bad = bad || !isfinite(prop[c * N + p]) || !isfinite(emis[c * N + p]);
    if (bad) flag[0] = 1;
  }
}

__global__ void k_fill_f64(double* __restrict__ p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Ray constants (direction, weight, emission and J projection tables) and the
// normalized frequency weights, from the uploaded quadrature.
template <class T>
__global__ void k_prepare(const double* __restrict__ mu, const double* __restrict__ wmu, int nmu,
                          int nchi, double w2, const double* __restrict__ phi,
                          const double* __restrict__ wfreq, int nfreq,
                          RayConsts* __restrict__ rays, T* __restrict__ phiT,
                          double* __restrict__ wn) {
  __shared__ double norm;
  const int nh = nmu * nchi;
  for (int r = threadIdx.x; r < 2 * nh; r += blockDim.x) {
    const int a = (r % nh) / nchi, m = r % nchi;
    const double m0 = mu[a];
    const double chi = (m + 0.5) * (2.0 * M_PI / nchi);
    ray_consts(r < nh ? m0 : -m0, chi, 0.5 * wmu[a] / nchi, w2, rays[r]);
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int j = 0; j < nfreq; ++j) s += wfreq[j] * phi[j];
    norm = s;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nfreq; j += blockDim.x) {
    wn[j] = wfreq[j] * phi[j] / norm;
    phiT[j] = (T)phi[j];
  }
}

// ---------------------------------------------------------------------------
// Vector loads and stores of one Stokes vector.
// ---------------------------------------------------------------------------
__device__ inline void load4(const float* p, float v[4]) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}
__device__ inline void load4(const double* p, double v[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ inline void store4(float* p, const float v[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ inline void store4(double* p, const double v[4]) {
  *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  *reinterpret_cast<double2*>(p + 2) = make_double2(v[2], v[3]);
}
// The same with the non-temporal hint: a plane state that the next launch reads from
// HBM anyway (the planes of a launch exceed the caches) need not take L2 lines from
// the upwind rows and coefficients that neighbouring tiles read again.
typedef float porta_f4 __attribute__((ext_vector_type(4)));
typedef double porta_d2 __attribute__((ext_vector_type(2)));
__device__ inline void store4_nt(float* p, const float v[4]) {
  const porta_f4 q = {v[0], v[1], v[2], v[3]};
  __builtin_nontemporal_store(q, reinterpret_cast<porta_f4*>(p));
}
__device__ inline void store4_nt(double* p, const double v[4]) {
  const porta_d2 a = {v[0], v[1]}, b = {v[2], v[3]};
  __builtin_nontemporal_store(a, reinterpret_cast<porta_d2*>(p));
  __builtin_nontemporal_store(b, reinterpret_cast<porta_d2*>(p + 2));
}

__device__ inline int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Bilinear stencil on a periodic plane for a point displaced by (u, v) cells
// from node (i, j).  For one ray and one pair of planes the displacement is
// the same at every node, so every thread of a plane sees the same weights.
struct Stencil {
  int i00, i10, i01, i11;
  double w00, w10, w01, w11;
};

__device__ inline Stencil make_stencil(int i, int j, int nx, int ny, double u, double v) {
  // reduce the displacement to one period first so the integer shift stays in range
  u -= nx * floor(u / nx);
  v -= ny * floor(v / ny);
  const double fu = floor(u), fv = floor(v);
  const double tx = u - fu, ty = v - fv;
  const int i0 = wrapi(i + (int)fu, nx), i1 = (i0 + 1 == nx) ? 0 : i0 + 1;
  const int j0 = wrapi(j + (int)fv, ny), j1 = (j0 + 1 == ny) ? 0 : j0 + 1;
  Stencil s;
  s.i00 = j0 * nx + i0;
  s.i10 = j0 * nx + i1;
  s.i01 = j1 * nx + i0;
  s.i11 = j1 * nx + i1;
  s.w00 = (1.0 - tx) * (1.0 - ty);
  s.w10 = tx * (1.0 - ty);
  s.w01 = (1.0 - tx) * ty;
  s.w11 = tx * ty;
  return s;
}

template <class T>
__device__ inline double bil(const T* __restrict__ f, const Stencil& s) {
  return s.w00 * (double)f[s.i00] + s.w10 * (double)f[s.i10] + s.w01 * (double)f[s.i01] +
         s.w11 * (double)f[s.i11];
}

// Transposed stencil: the nodes (i', j') whose stencil for the same displacement
// (u, v) contains node (i, j), with the weight that node received.  Used by the
// adjoint to turn the scatter of the forward interpolation into a gather.
__device__ inline Stencil make_tstencil(int i, int j, int nx, int ny, double u, double v) {
  u -= nx * floor(u / nx);
  v -= ny * floor(v / ny);
  const double fu = floor(u), fv = floor(v);
  const double tx = u - fu, ty = v - fv;
  const int i0 = wrapi(i - (int)fu, nx), i1 = (i0 == 0) ? nx - 1 : i0 - 1;
  const int j0 = wrapi(j - (int)fv, ny), j1 = (j0 == 0) ? ny - 1 : j0 - 1;
  Stencil s;
  s.i00 = j0 * nx + i0;
  s.i10 = j0 * nx + i1;
  s.i01 = j1 * nx + i0;
  s.i11 = j1 * nx + i1;
  s.w00 = (1.0 - tx) * (1.0 - ty);
  s.w10 = tx * (1.0 - ty);
  s.w01 = (1.0 - tx) * ty;
  s.w11 = tx * ty;
  return s;
}

// 3x3 stencil around the node nearest to the displaced point (mode B), with the
// fractional offsets tx, ty in [-1/2, 1/2) from that node.
struct Stencil9 {
  int col[3];     // x indices of columns -1, 0, +1 (periodic)
  int row[3];     // offsets j * nx of rows -1, 0, +1 (periodic)
  double tx, ty;
};

__device__ inline Stencil9 make_stencil9(int i, int j, int nx, int ny, double u, double v) {
  u -= nx * floor(u / nx);
  v -= ny * floor(v / ny);
  const double fu = floor(u + 0.5), fv = floor(v + 0.5);
  Stencil9 s;
  s.tx = u - fu;
  s.ty = v - fv;
  const int ic = wrapi(i + (int)fu, nx), jc = wrapi(j + (int)fv, ny);
  s.col[0] = (ic == 0) ? nx - 1 : ic - 1;
  s.col[1] = ic;
  s.col[2] = (ic + 1 == nx) ? 0 : ic + 1;
  s.row[0] = ((jc == 0) ? ny - 1 : jc - 1) * nx;
  s.row[1] = jc * nx;
  s.row[2] = ((jc + 1 == ny) ? 0 : jc + 1) * nx;
  return s;
}

// Monotonic Bezier interpolation on a plane: along x for each of the three rows,
// then along y.
template <class T>
__device__ inline double bez9(const T* __restrict__ f, const Stencil9& s) {
  const BezW<double> wx = bez_weights(s.tx), wy = bez_weights(s.ty);
  double r[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const T* row = f + s.row[b];
    r[b] = bez_eval(wx, (double)row[s.col[0]], (double)row[s.col[1]], (double)row[s.col[2]]);
  }
  return bez_eval(wy, r[0], r[1], r[2]);
}

// Frequency-independent part of the update of node p on plane kO for one ray:
// transfer coefficients interpolated at M (plane kM) and P (plane kP, if any),
// source vectors S = eps/eta_I at M, O, P, K' at M and O, the line-centre
// optical paths and the BESSER control points (Sect. 3.1-3.3).
struct PointSetup {
  Stencil sM;
  double dsM, dsP;
  double kapM, kapO, kapP, ikM, ikO, ikP;
  double epsM[6], epsO[6], epsP[6], etaM[6], etaO[6];
  double SM[4], SO[4], SP[4], cM[4];
  double tau0M, tau0P, ratio;
  bool hasP;
};

template <int MODE, class T>
__device__ inline void setup_point(const T* __restrict__ kappa, const T* __restrict__ prop,
                                   const T* __restrict__ emis, size_t N, int nx, int ny, int np,
                                   int kO, int kM, int kP, double dzM, double dzP, double inv_dx,
                                   double inv_dy, const RayConsts& rc, int p, bool parabolic,
                                   PointSetup& ps, Stencil9& sM9) {
  const int i = p % nx, j = p / nx;
  const double inv_mu = 1.0 / fabs(rc.mu);
  ps.dsM = dzM * inv_mu;
  const double uM = -ps.dsM * rc.sx * inv_dx, vM = -ps.dsM * rc.sy * inv_dy;
  const size_t bM = (size_t)kM * np, bO = (size_t)kO * np + p;
  if (MODE == 0) {
    ps.sM = make_stencil(i, j, nx, ny, uM, vM);
    ps.kapM = bil(kappa + bM, ps.sM);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      ps.epsM[c] = bil(emis + c * N + bM, ps.sM);
      ps.etaM[c] = bil(prop + c * N + bM, ps.sM);
    }
  } else {
    ps.sM = Stencil{0, 0, 0, 0, 1.0, 0.0, 0.0, 0.0};
    sM9 = make_stencil9(i, j, nx, ny, uM, vM);
    ps.kapM = bez9(kappa + bM, sM9);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      ps.epsM[c] = bez9(emis + c * N + bM, sM9);
      ps.etaM[c] = bez9(prop + c * N + bM, sM9);
    }
  }
  ps.kapO = (double)kappa[bO];
  ps.ikM = 1.0 / ps.kapM;
  ps.ikO = 1.0 / ps.kapO;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    ps.epsO[c] = (double)emis[c * N + bO];
    ps.etaO[c] = (double)prop[c * N + bO];
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    double em = 0.0, eo = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      em += rc.emis[s][c] * ps.epsM[c];
      eo += rc.emis[s][c] * ps.epsO[c];
    }
    ps.SM[s] = em * ps.ikM;
    ps.SO[s] = eo * ps.ikO;
  }
  ps.tau0M = 0.5 * (ps.kapM + ps.kapO) * ps.dsM;   // line-centre tau_MO
  ps.hasP = kP >= 0;
  if (ps.hasP) {
    ps.dsP = dzP * inv_mu;
    const double uP = ps.dsP * rc.sx * inv_dx, vP = ps.dsP * rc.sy * inv_dy;
    const size_t bP = (size_t)kP * np;
    if (MODE == 0) {
      const Stencil sP = make_stencil(i, j, nx, ny, uP, vP);
      ps.kapP = bil(kappa + bP, sP);
#pragma unroll
      for (int c = 0; c < 6; ++c) ps.epsP[c] = bil(emis + c * N + bP, sP);
    } else {
      const Stencil9 sP = make_stencil9(i, j, nx, ny, uP, vP);
      ps.kapP = bez9(kappa + bP, sP);
#pragma unroll
      for (int c = 0; c < 6; ++c) ps.epsP[c] = bez9(emis + c * N + bP, sP);
    }
    ps.ikP = 1.0 / ps.kapP;
    ps.tau0P = 0.5 * (ps.kapO + ps.kapP) * ps.dsP;
    ps.ratio = ps.tau0M / ps.tau0P;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double ep = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) ep += rc.emis[s][c] * ps.epsP[c];
      ps.SP[s] = ep * ps.ikP;
      ps.cM[s] = control_cm(ps.SM[s], ps.SO[s], ps.SP[s], ps.ratio, parabolic);
    }
  } else {
    // no downwind plane: linear control point
    ps.dsP = ps.kapP = ps.ikP = ps.tau0P = ps.ratio = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      ps.SP[s] = 0.0;
      ps.cM[s] = 0.5 * (ps.SM[s] + ps.SO[s]);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) ps.epsP[c] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Add the frequency-integrated Stokes vectors of a batch of rays on one plane
// to J^K_Q (Eq. 1) and Lbar, in a fixed ray order (no atomics).  On the
// boundary plane the Stokes vector is (ibound, 0, 0, 0) at every frequency.
// ---------------------------------------------------------------------------
__device__ inline void jreduce_point(double* __restrict__ jkq, const double* __restrict__ jpart,
                                     const RayConsts* __restrict__ rays, int ray0, int nrb,
                                     int np, size_t N, size_t plane_off, int p, int boundary,
                                     double ibound) {
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int rb = 0; rb < nrb; ++rb) {
    const RayConsts& rc = rays[ray0 + rb];
    double ib[4], lam;
    if (boundary) {
      ib[0] = ibound;
      ib[1] = ib[2] = ib[3] = 0.0;
      lam = 0.0;
    } else {
      const double* jp = jpart + (size_t)rb * 5 * np + p;
      ib[0] = jp[0];
      ib[1] = jp[(size_t)np];
      ib[2] = jp[2 * (size_t)np];
      ib[3] = jp[3 * (size_t)np];
      lam = jp[4 * (size_t)np];
    }
    const double w = rc.weight;
#pragma unroll
    for (int c = 0; c < 9; ++c)
      acc[c] += w * (rc.proj[c][0] * ib[0] + rc.proj[c][1] * ib[1] + rc.proj[c][2] * ib[2] +
                     rc.proj[c][3] * ib[3]);
    acc[9] += w * lam;
  }
#pragma unroll
  for (int c = 0; c < 10; ++c) jkq[c * N + plane_off + p] += acc[c];
}

__global__ void __launch_bounds__(256)
    k_jreduce(double* __restrict__ jkq, const double* __restrict__ jpart,
              const RayConsts* __restrict__ rays, int ray0, int nrb, int np, size_t N,
              size_t plane_off, int boundary, double ibound) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  jreduce_point(jkq, jpart, rays, ray0, nrb, np, N, plane_off, p, boundary, ibound);
}

// ---------------------------------------------------------------------------
// One plane of the sweep for a batch of rays of one hemisphere and every
// frequency.  Thread = (node of plane k, ray of the batch); the frequency
// loop runs inside the thread so that the frequency-independent work
// (interpolation of the coefficients at M and P, S and K' at M and O, the
// BESSER control points) is done once per node and ray.
//
// Plane state layout: [ray in batch][frequency][node][Stokes].
// ---------------------------------------------------------------------------
template <class T>
struct PlaneArgs {
  const T* kappa;
  const T* prop;
  const T* emis;
  const RayConsts* rays;
  const T* phi;
  const double* wn;
  const T* iprev;    // upwind plane state, or nullptr when the upwind plane is the boundary
  T* inext;          // state of plane k
  double* jpart;     // [ray in batch][5][node]: sum_j W_j I_i and sum_j W_j Lambda*, or nullptr
  // J of the previous plane (reduced by the blocks of the first ray of the batch)
  double* jkq;               // [10][N] or nullptr
  const double* jpart_prev;  // partial sums of the previous plane, or nullptr (boundary plane)
  size_t prev_off;           // offset of the previous plane in jkq
  size_t N;
  int nx, ny, np, nfreq;
  int kO, kM, kP;    // plane of O, upwind plane, downwind plane (-1: none)
  double dzM, dzP;   // |z_kO - z_kM|, |z_kP - z_kO|
  double inv_dx, inv_dy;
  int ray0;
  int xcd_remap;     // tiles per XCD per round (0: hardware order), see xcd_tile
  int parabolic;     // control point: 0 BESSER, 1 parabola through M, O, P
  T ibound;          // Stokes I on the boundary plane of this hemisphere
};

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X, each with
// its own L2.  With chunk R > 0 the tiles are renumbered so that every XCD takes
// R consecutive tiles per round (neighbouring rows of one ray then share an L2)
// while the eight XCDs still advance through the grid together.
__device__ inline void xcd_tile(int chunk, int& bx, int& by) {
  bx = blockIdx.x;
  by = blockIdx.y;
  if (chunk <= 0) return;
  const int T = gridDim.x * gridDim.y;
  const int L = blockIdx.y * gridDim.x + blockIdx.x;
  const int round = 8 * chunk;
  const int Tmain = (T / round) * round;
  int Lp = L;
  if (L < Tmain) {
    const int x = L % 8, k = L / 8;
    Lp = (k / chunk) * round + x * chunk + (k % chunk);
  }
  bx = Lp % gridDim.x;
  by = Lp / gridDim.x;
}

constexpr int kMaxFreq = 4096;   // frequencies held in LDS by the sweep kernels

template <class T>
__device__ inline void load_upwind(const T* __restrict__ q, const Stencil& s, T v[4][4]) {
  load4(q + 4 * (size_t)s.i00, v[0]);
  load4(q + 4 * (size_t)s.i10, v[1]);
  load4(q + 4 * (size_t)s.i01, v[2]);
  load4(q + 4 * (size_t)s.i11, v[3]);
}

// Upwind Stokes vector of one frequency by the 9-point monotonic Bezier (mode B).
template <class T>
__device__ inline void upwind_bez9(const T* __restrict__ q, const Stencil9& s,
                                   const BezW<T>& wx, const BezW<T>& wy, T IM[4]) {
  T v[3][3][4];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) load4(q + 4 * (size_t)(s.row[b] + s.col[a]), v[b][a]);
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    T r[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) r[b] = bez_eval(wx, v[b][0][st], v[b][1][st], v[b][2][st]);
    IM[st] = bez_eval(wy, r[0], r[1], r[2]);
  }
}

// Occupancy targets: three waves per SIMD for the FP32 bilinear sweep (168 VGPRs,
// with the next frequency's corners in flight and no spill in the loop; four or five
// waves were slower), two for the others (the 9-point mode would otherwise drop to
// one).
template <class T, int MODE>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(MODE == 0 && sizeof(T) == 4 ? 3 : 2)))
k_sweep_plane(const PlaneArgs<T> a) {
  // per-frequency weights and profile, read from LDS inside the frequency loop so that
  // no vector-memory wait (which on gfx9 also covers earlier stores) sits in the loop
  extern __shared__ double s_tab[];
  double* s_wn = s_tab;
  T* s_phi = reinterpret_cast<T*>(s_tab + a.nfreq);
  for (int t = threadIdx.x; t < a.nfreq; t += blockDim.x) {
    s_wn[t] = a.wn[t];
    s_phi[t] = a.phi[t];
  }
  __syncthreads();
  int bx, rb;
  xcd_tile(a.xcd_remap, bx, rb);
  const int p = bx * blockDim.x + threadIdx.x;
  const bool active = p < a.np;
  const int pp = active ? p : 0;   // inactive lanes only take part in the barriers
  if (active && rb == 0 && a.jkq)
    jreduce_point(a.jkq, a.jpart_prev, a.rays, a.ray0, gridDim.y, a.np, a.N, a.prev_off, p,
                  a.jpart_prev == nullptr, (double)a.ibound);
  const RayConsts& rc = a.rays[a.ray0 + rb];
  PointSetup ps;
  Stencil9 sM9;
  setup_point<MODE>(a.kappa, a.prop, a.emis, a.N, a.nx, a.ny, a.np, a.kO, a.kM, a.kP, a.dzM,
                    a.dzP, a.inv_dx, a.inv_dy, rc, pp, a.parabolic != 0, ps, sM9);
  const BezW<T> bwx = bez_weights(MODE == 1 ? (T)sM9.tx : T(0));
  const BezW<T> bwy = bez_weights(MODE == 1 ? (T)sM9.ty : T(0));
  const Stencil& sM = ps.sM;
  const double ikM = ps.ikM, ikO = ps.ikO;
  const double* etaM = ps.etaM;
  const double* etaO = ps.etaO;
  const double* SM = ps.SM;
  const double* SO = ps.SO;
  const double* cM = ps.cM;
  const double tau0M = ps.tau0M;
  // Lambda* = omega_O + omega_C c_M for a unit source at O alone (Eq. 14): c_M is 1 for
  // BESSER, (1 + ratio)/2 for the parabola, 1/2 without a downwind point
  const double lamfac = ps.hasP ? control_cm(0.0, 1.0, 0.0, ps.ratio, a.parabolic != 0) : 0.5;

  // frequency-independent pieces in the sweep precision
  const T eMv[3] = {(T)(etaM[0] * ikM), (T)(etaM[1] * ikM), (T)(etaM[2] * ikM)};
  const T rMv[3] = {(T)(etaM[3] * ikM), (T)(etaM[4] * ikM), (T)(etaM[5] * ikM)};
  const T eOv[3] = {(T)(etaO[0] * ikO), (T)(etaO[1] * ikO), (T)(etaO[2] * ikO)};
  const T rOv[3] = {(T)(etaO[3] * ikO), (T)(etaO[4] * ikO), (T)(etaO[5] * ikO)};
  const StokesOp<T> KO = stokes_op(eOv, rOv);
  T SMt[4], SOt[4], cMt[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    SMt[s] = (T)SM[s];
    SOt[s] = (T)SO[s];
    cMt[s] = (T)cM[s];
  }
  const T tau0 = (T)tau0M;
  const T w00 = (T)sM.w00, w10 = (T)sM.w10, w01 = (T)sM.w01, w11 = (T)sM.w11;
  const T lf = (T)lamfac;

  const size_t fstride = (size_t)a.np * 4;
  const T* ip = a.iprev ? a.iprev + (size_t)rb * a.nfreq * fstride : nullptr;
  T* op = a.inext + (size_t)rb * a.nfreq * fstride + (size_t)pp * 4;
  double jacc0 = 0.0, jacc1 = 0.0, jacc2 = 0.0, jacc3 = 0.0, lacc = 0.0;

  if (!active) return;   // no barrier follows

  // one update (Eq. fsbez solved with Eq. kappa) at frequency f from the upwind
  // Stokes vector IM
  auto update = [&](int f, T i0, T i1, T i2, T i3) __attribute__((always_inline)) {
    const T IM[4] = {i0, i1, i2, i3};
    const T tau = tau0 * s_phi[f];
    const Coefs<T> cf = coefficients(tau);
    T KI[4];
    kprime_apply(eMv, rMv, IM, KI);
    T b[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
      b[s] = cf.e * IM[s] - cf.psiM * KI[s] + cf.omM * SMt[s] + cf.omO * SOt[s] + cf.omC * cMt[s];
    T x[4];
    stokes_solve<1>(KO, stokes_freq(KO, cf.psiO), b, x);
    store4_nt(op + (size_t)f * fstride, x);
    const double W = s_wn[f];
    jacc0 += W * (double)x[0];
    jacc1 += W * (double)x[1];
    jacc2 += W * (double)x[2];
    jacc3 += W * (double)x[3];
    lacc += W * (double)(cf.omO + lf * cf.omC);
  };
  // bilinear upwind component s from the four corner values
#define PORTA_BILIN(v, s) (w00 * v[0][s] + w10 * v[1][s] + w01 * v[2][s] + w11 * v[3][s])

  if (!ip) {
    // the upwind plane is the boundary
    for (int f = 0; f < a.nfreq; ++f) update(f, a.ibound, T(0), T(0), T(0));
  } else if (MODE == 1) {
    for (int f = 0; f < a.nfreq; ++f) {
      T IM[4];
      upwind_bez9(ip + (size_t)f * fstride, sM9, bwx, bwy, IM);
      update(f, IM[0], IM[1], IM[2], IM[3]);
    }
  } else {
    if constexpr (sizeof(T) == 4) {
      // the corners of frequency f + 1 are loaded during the arithmetic of frequency f
      // (in FP64 the second buffer does not fit without spilling)
      T vA[4][4], vB[4][4];
      load_upwind(ip, sM, vA);
      for (int f = 0; f < a.nfreq; f += 2) {
        if (f + 1 < a.nfreq) load_upwind(ip + (size_t)(f + 1) * fstride, sM, vB);
        update(f, PORTA_BILIN(vA, 0), PORTA_BILIN(vA, 1), PORTA_BILIN(vA, 2),
               PORTA_BILIN(vA, 3));
        if (f + 1 >= a.nfreq) break;
        if (f + 2 < a.nfreq) load_upwind(ip + (size_t)(f + 2) * fstride, sM, vA);
        update(f + 1, PORTA_BILIN(vB, 0), PORTA_BILIN(vB, 1), PORTA_BILIN(vB, 2),
               PORTA_BILIN(vB, 3));
      }
    } else {
      T v[4][4];
      for (int f = 0; f < a.nfreq; ++f) {
        load_upwind(ip + (size_t)f * fstride, sM, v);
        update(f, PORTA_BILIN(v, 0), PORTA_BILIN(v, 1), PORTA_BILIN(v, 2), PORTA_BILIN(v, 3));
      }
    }
  }
#undef PORTA_BILIN
  if (a.jpart) {
    double* jp = a.jpart + (size_t)rb * 5 * a.np + p;
    jp[0] = jacc0;
    jp[(size_t)a.np] = jacc1;
    jp[2 * (size_t)a.np] = jacc2;
    jp[3 * (size_t)a.np] = jacc3;
    jp[4 * (size_t)a.np] = lacc;
  }
}

// Eq. 1 from a stored block of Stokes vectors [nray][nf][N][4].
template <class T>
__global__ void __launch_bounds__(256)
    k_jkq_accumulate(double* __restrict__ jkq, const T* __restrict__ stokes,
                     const T* __restrict__ lam, const RayConsts* __restrict__ rays,
                     const double* __restrict__ wn, int ray0, int nray, int f0, int nf, size_t N) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int r = 0; r < nray; ++r) {
    double ib[4] = {0, 0, 0, 0}, lb = 0.0;
    for (int q = 0; q < nf; ++q) {
      const double W = wn[f0 + q];
      const size_t off = ((size_t)r * nf + q) * N + p;
      T v[4];
      load4(stokes + 4 * off, v);
#pragma unroll
      for (int s = 0; s < 4; ++s) ib[s] += W * (double)v[s];
      if (lam) lb += W * (double)lam[off];
    }
    const RayConsts& rc = rays[ray0 + r];
    const double w = rc.weight;
#pragma unroll
    for (int c = 0; c < 9; ++c)
      acc[c] += w * (rc.proj[c][0] * ib[0] + rc.proj[c][1] * ib[1] + rc.proj[c][2] * ib[2] +
                     rc.proj[c][3] * ib[3]);
    acc[9] += w * lb;
  }
#pragma unroll
  for (int c = 0; c < 10; ++c) jkq[c * N + p] += acc[c];
}

}  // namespace porta
