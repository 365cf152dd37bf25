// porta_adjoint.hpp -- reverse-mode derivative of the sweep of the upward rays
// for a loss on the Stokes vectors at the top plane.
//
// Forward recurrence for node p on plane k (one ray, one frequency):
//   I_M = sum_ab w_ab I_{k-1}[q_ab(p)]                       (bilinear at M)
//   b   = (e - psi'_M K'_M) I_M + omega_M S_M + omega_O S_O + omega_C c_M
//   (1 + psi'_O K'_O) I_O = b                                 (Eqs. fsbez, kappa)
// with S, K', c_M and tau built from the interpolated transfer coefficients.
// Going down from the top plane, the adjoint of I on plane k,
//   lambda_k(q) = sum_ab w_ab Lambda_{k+1}(q - shift_ab)       (transposed stencil),
// gives lambda_b = (1 + psi'_O K'_O)^-T lambda_k and
//   Lambda_k = (e - psi'_M K'_M)^T lambda_b,
// the adjoint of the interpolated upwind vector, which the next plane down
// gathers again.  The frequency loop accumulates the partials of the
// frequency-independent quantities (tau_MO at line centre, S_M, S_O, c_M, K'_M,
// K'_O); they are then propagated through the BESSER control point, the
// ratio of optical paths and the divisions by eta_I to the coefficients at O
// (written directly) and at M and P (gathered through transposed stencils).
#pragma once

#include <type_traits>

#include "porta_kernels.hpp"

namespace porta {

template <class T>
struct AdjArgs {
  const T* kappa;
  const T* prop;
  const T* emis;
  const RayConsts* rays;
  const T* phi;
  const T* iprev;      // forward state of plane kM, or nullptr for the boundary plane
  const T* lam_next;   // Lambda of plane kO + 1, or nullptr when kO is the top plane
  const T* seed;       // dL/dI on the top plane for this batch (used when lam_next is null)
  T* lam_cur;          // Lambda of plane kO, or nullptr when plane kM is the boundary
  T* g_o;              // [ray in batch][13][node]: coefficients at O
  T* g_m;              // [ray in batch][13][node]: coefficients interpolated at M
  T* g_p;              // [ray in batch][7][node]:  eta_I and eps interpolated at P
                       // (partials of one node and ray, formed in FP64, stored in the
                       // sweep precision; the gather sums them in FP64)
  size_t N;
  int nx, ny, np, nfreq;
  int kO, kM, kP;
  double dzM, dzP, dzN;   // dzN = |z_{kO+1} - z_kO| (plane above), 0 on the top plane
  double inv_dx, inv_dy;
  int ray0;
  int xcd_remap;       // tiles per XCD per round, see xcd_tile
  int parabolic;       // control point: 0 BESSER, 1 parabola through M, O, P
  T ibound;
};

// The bilinear form l^T K' x is linear in the six entries (e_Q, e_U, e_V, r_Q, r_U,
// r_V) of K' (kprime_apply's layout); q[c] is its partial in entry c, so that
// l^T K' x = sum_c entry_c q[c].
template <class T>
__device__ inline void kprime_forms(const T l[4], const T x[4], T q[6]) {
  q[0] = l[0] * x[1] + l[1] * x[0];
  q[1] = l[0] * x[2] + l[2] * x[0];
  q[2] = l[0] * x[3] + l[3] * x[0];
  q[3] = l[2] * x[3] - l[3] * x[2];
  q[4] = l[3] * x[1] - l[1] * x[3];
  q[5] = l[1] * x[2] - l[2] * x[1];
}

// Partials of b's K' I term: dL/d(e_Q, e_U, e_V, r_Q, r_U, r_V) of -psi lambda^T K' x.
template <class T>
__device__ inline void kprime_outer(T psi, const T l[4], const T x[4], T g[6]) {
  T q[6];
  kprime_forms(l, x, q);
#pragma unroll
  for (int c = 0; c < 6; ++c) g[c] -= psi * q[c];
}

// Where the 9-point stencil of a displacement (u, v) in cells sits, as make_stencil9
// places it: the centre is the node (fu, fv) away, the point at (tx, ty) from it.
struct Bez9Geom {
  int fu, fv;
  double tx, ty;
};

__device__ inline Bez9Geom bez9_geom(double u, double v, int nx, int ny) {
  u -= nx * floor(u / nx);
  v -= ny * floor(v / ny);
  Bez9Geom g;
  const double fu = floor(u + 0.5), fv = floor(v + 0.5);
  g.fu = (int)fu;
  g.fv = (int)fv;
  g.tx = u - fu;
  g.ty = v - fv;
  return g;
}

// Adjoint of the 9-point monotonic Bezier interpolation (x pass over three rows, then
// y), gathered at a node q: out += sum_p dB_p / df(q) adj(p) over the nine nodes p
// whose stencil holds q.  The stencil of p is centred (fu, fv) from p, so those p are
// q - (fu, fv) + (cc, rc), cc, rc in {-1, 0, 1}, with their centre at (cc, rc) from q.
// val(r, c, v) loads the K components of the interpolated field at q + (c, r), |c|,
// |r| <= 2; adj(rc, cc, g) loads the adjoint of the interpolated value at that p.  The
// partials follow the branches of the forward evaluation (bez_eval_grad); a node that
// the periodic wrap puts at several places of a stencil gets the sum of its partials,
// one per place.
template <class T, int K, class Val, class Adj>
__device__ inline void bez9_adjoint_gather(const BezW<T>& wx, const BezW<T>& wy, Val val,
                                           Adj adj, T out[K]) {
  T R[5][3][K];   // x pass of rows -2..2 (index + 2) about column centres -1, 0, 1
  T gx[3][K];     // d R[row 0][cc] / d f(q)
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    T v[5][K];
#pragma unroll
    for (int c = 0; c < 5; ++c) val(r - 2, c - 2, v[c]);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (r == 2) {
          T g[3];
          R[r][cc][k] = bez_eval_grad(wx, v[cc][k], v[cc + 1][k], v[cc + 2][k], g);
          gx[cc][k] = g[2 - cc];   // q is column 0: place 2 - cc of the triple
        } else {
          R[r][cc][k] = bez_eval(wx, v[cc][k], v[cc + 1][k], v[cc + 2][k]);
        }
      }
  }
#pragma unroll
  for (int rc = 0; rc < 3; ++rc)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      T ga[K];
      adj(rc - 1, cc - 1, ga);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        T g[3];
        bez_eval_grad(wy, R[rc][cc][k], R[rc + 1][cc][k], R[rc + 2][cc][k], g);
        out[k] += g[2 - rc] * gx[cc][k] * ga[k];   // q is row 0: place 2 - rc
      }
    }
}

// Adjoint of the Stokes vectors of plane kO in the 9-point mode: gathered from the
// adjoint of I_M at the nodes of plane kO + 1 (whose M points interpolate plane kO)
// through the transposed Bezier stencil, at every frequency.
template <class T>
struct TGatherArgs {
  const T* icur;       // forward state of plane kO ([ray][freq][node][4])
  const T* lam_next;   // adjoint of I_M at the nodes of plane kO + 1, same layout
  T* out;              // adjoint of I at the nodes of plane kO, same layout
  const RayConsts* rays;
  int nx, ny, np, nfreq;
  double dzN, inv_dx, inv_dy;   // dzN = |z_{kO+1} - z_kO|
  int ray0;
};

// A block takes a tile of TGX x TGY nodes q of one ray (blockIdx.z) and forms, per
// frequency, the pieces of bez9_adjoint_gather that neighbouring nodes share once in
// LDS: the x pass of every row triple (centre (x, y), rows of the tile +-2, columns +-1),
// its partials on the tile's rows, and the partials of the y pass of every centre
// (rows +-1).  Node q then sums, over the nine p whose stencil holds it, the product
// of the y partial of p's centre (qx + cc, qy + rc) at q's row, the x partial of the
// centre (qx + cc, qy) at q's column and the adjoint at p.  Positions, not nodes, are
// staged, so a small periodic plane that puts a node at several places works as in
// bez9_adjoint_gather.
template <class T>
struct TGTile {
  static constexpr int X = sizeof(T) == 4 ? 64 : 32, Y = 4;
};

template <class T>
__global__ void __launch_bounds__(256) k_bez9_tgather(const TGatherArgs<T> a) {
  constexpr int TX = TGTile<T>::X, TY = TGTile<T>::Y;
  constexpr int FX = TX + 4, FY = TY + 4;   // staged forward states: columns -2..TX+1
  constexpr int CX = TX + 2;                // centres: columns -1..TX
  __shared__ T sF[FY][FX][4];               // rows -2..TY+1
  __shared__ T sR[FY][CX][4];               // x pass at the centres, rows -2..TY+1
  __shared__ T sGx[TY][CX][3][4];           // its partials on the tile's rows
  __shared__ T sGy[TY + 2][CX][3][4];       // y-pass partials at centre rows -1..TY
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int rb = blockIdx.z;
  const int qx0 = blockIdx.x * TX, qy0 = blockIdx.y * TY;
  const RayConsts& rc = a.rays[a.ray0 + rb];
  const double dsN = a.dzN / fabs(rc.mu);
  const Bez9Geom gm = bez9_geom(-dsN * rc.sx * a.inv_dx, -dsN * rc.sy * a.inv_dy, a.nx, a.ny);
  const BezW<T> wx = bez_weights((T)gm.tx), wy = bez_weights((T)gm.ty);
  const int lx = tid % TX, ly = tid / TX;     // this thread's node of the tile
  const int qx = qx0 + lx, qy = qy0 + ly;
  const bool active = ly < TY && qx < a.nx && qy < a.ny;
  int prow[3], pcol[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    prow[d] = wrapi(qy - gm.fv + d - 1, a.ny) * a.nx;
    pcol[d] = wrapi(qx - gm.fu + d - 1, a.nx);
  }
  const size_t fstride = (size_t)a.np * 4;
  const size_t roff = (size_t)rb * a.nfreq * fstride;
  // The forward states of frequency f + 1 (this thread's share of the tile) and the
  // nine adjoints at p are loaded while frequency f is being worked on, and the states
  // go to LDS once the x passes of f have read it.
  constexpr int NF = (FY * FX + TX * TY - 1) / (TX * TY);   // tile entries per thread
  T fN[NF][4], lam[3][3][4], lamN[3][3][4];
  auto load_tile = [&](int f) __attribute__((always_inline)) {
    const T* ic = a.icur + roff + (size_t)f * fstride;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int e = tid + i * nthr;
      if (e < FY * FX) {
        const int r = e / FX, c = e % FX;
        const size_t n = (size_t)wrapi(qy0 + r - 2, a.ny) * a.nx + wrapi(qx0 + c - 2, a.nx);
        load4(ic + 4 * n, fN[i]);
      }
    }
  };
  auto store_tile = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int e = tid + i * nthr;
      if (e < FY * FX) {
        const int r = e / FX, c = e % FX;
#pragma unroll
        for (int k = 0; k < 4; ++k) sF[r][c][k] = fN[i][k];
      }
    }
  };
  auto load_lam = [&](int f, T (&dst)[3][3][4]) __attribute__((always_inline)) {
    const T* ln = a.lam_next + roff + (size_t)f * fstride;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) load4(ln + 4 * (size_t)(prow[r] + pcol[c]), dst[r][c]);
  };
  load_tile(0);
  load_lam(0, lam);
  store_tile();
  __syncthreads();
  for (int f = 0; f < a.nfreq; ++f) {
    const bool more = f + 1 < a.nfreq;
    if (more) {
      load_tile(f + 1);
      load_lam(f + 1, lamN);
    }
    for (int e = tid; e < FY * CX; e += nthr) {
      const int r = e / CX, c = e % CX;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (r >= 2 && r < TY + 2) {
          T g[3];
          sR[r][c][k] = bez_eval_grad(wx, sF[r][c][k], sF[r][c + 1][k], sF[r][c + 2][k], g);
          sGx[r - 2][c][0][k] = g[0];
          sGx[r - 2][c][1][k] = g[1];
          sGx[r - 2][c][2][k] = g[2];
        } else {
          sR[r][c][k] = bez_eval(wx, sF[r][c][k], sF[r][c + 1][k], sF[r][c + 2][k]);
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < (TY + 2) * CX; e += nthr) {
      const int r = e / CX, c = e % CX;   // centre row qy0 - 1 + r: R rows r .. r + 2
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        T g[3];
        bez_eval_grad(wy, sR[r][c][k], sR[r + 1][c][k], sR[r + 2][c][k], g);
        sGy[r][c][0][k] = g[0];
        sGy[r][c][1][k] = g[1];
        sGy[r][c][2][k] = g[2];
      }
    }
    if (more) store_tile();   // sF was last read before the barrier above
    __syncthreads();
    if (active) {
      T out[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int r = 0; r < 3; ++r)        // rc = r - 1
#pragma unroll
        for (int c = 0; c < 3; ++c)      // cc = c - 1
#pragma unroll
          for (int k = 0; k < 4; ++k)
            out[k] += sGy[ly + r][lx + c][2 - r][k] * sGx[ly][lx + c][2 - c][k] * lam[r][c][k];
      store4(a.out + roff + (size_t)f * fstride + 4 * ((size_t)qy * a.nx + qx), out);
    }
    if (more) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 4; ++k) lam[r][c][k] = lamN[r][c][k];
    }
    __syncthreads();   // sGx, sGy and sR are refilled for the next frequency
  }
}

// FP32: two waves per SIMD (256 VGPRs), which leaves room for the loads of the next
// frequency to be in flight during the current one's arithmetic, with no spill in
// the frequency loop; three waves without that prefetch were 13% slower, three with
// it spill inside the loop.
// MODE 1 (9-point Bezier): the set-up and I_M as the 9-point sweep forms them; the
// adjoint of the Stokes vectors at O comes gathered (k_bez9_tgather) in `seed`, with
// lam_next null.
template <class T, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1)))
k_adjoint_plane(const AdjArgs<T> a) {
  extern __shared__ double s_tab[];
  T* s_phi = reinterpret_cast<T*>(s_tab);
  for (int t = threadIdx.x; t < a.nfreq; t += blockDim.x) s_phi[t] = a.phi[t];
  __syncthreads();
  int bx, rb;
  xcd_tile(a.xcd_remap, bx, rb);
  const int p = bx * blockDim.x + threadIdx.x;
  if (p >= a.np) return;
  const RayConsts& rc = a.rays[a.ray0 + rb];
  PointSetup ps;
  Stencil9 sM9;
  setup_point<MODE>(a.kappa, a.prop, a.emis, a.N, a.nx, a.ny, a.np, a.kO, a.kM, a.kP, a.dzM,
                    a.dzP, a.inv_dx, a.inv_dy, rc, p, a.parabolic != 0, ps, sM9);
  const BezW<T> bwx = bez_weights(MODE == 1 ? (T)sM9.tx : T(0));
  const BezW<T> bwy = bez_weights(MODE == 1 ? (T)sM9.ty : T(0));
  const int i = p % a.nx, j = p / a.nx;
  const double inv_mu = 1.0 / fabs(rc.mu);
  // nodes of the plane above whose upwind stencil contains p
  Stencil tN{};
  if (a.lam_next) {
    const double dsN = a.dzN * inv_mu;
    tN = make_tstencil(i, j, a.nx, a.ny, -dsN * rc.sx * a.inv_dx, -dsN * rc.sy * a.inv_dy);
  }
  const T eMv[3] = {(T)(ps.etaM[0] * ps.ikM), (T)(ps.etaM[1] * ps.ikM), (T)(ps.etaM[2] * ps.ikM)};
  const T rMv[3] = {(T)(ps.etaM[3] * ps.ikM), (T)(ps.etaM[4] * ps.ikM), (T)(ps.etaM[5] * ps.ikM)};
  const T eOv[3] = {(T)(ps.etaO[0] * ps.ikO), (T)(ps.etaO[1] * ps.ikO), (T)(ps.etaO[2] * ps.ikO)};
  const T rOv[3] = {(T)(ps.etaO[3] * ps.ikO), (T)(ps.etaO[4] * ps.ikO), (T)(ps.etaO[5] * ps.ikO)};
  const StokesOp<T> KO = stokes_op(eOv, rOv);
  const T rMn[3] = {-rMv[0], -rMv[1], -rMv[2]};
  T SMt[4], SOt[4], cMt[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    SMt[s] = (T)ps.SM[s];
    SOt[s] = (T)ps.SO[s];
    cMt[s] = (T)ps.cM[s];
  }
  const T tau0 = (T)ps.tau0M;
  const T w00 = (T)ps.sM.w00, w10 = (T)ps.sM.w10, w01 = (T)ps.sM.w01, w11 = (T)ps.sM.w11;
  const T n00 = (T)tN.w00, n10 = (T)tN.w10, n01 = (T)tN.w01, n11 = (T)tN.w11;

  const size_t fstride = (size_t)a.np * 4;
  const size_t rstride = (size_t)a.nfreq * fstride;
  const T* ip = a.iprev ? a.iprev + rb * rstride : nullptr;
  const T* lp = a.lam_next ? a.lam_next + rb * rstride : nullptr;
  const T* sp = a.seed + rb * rstride + (size_t)p * 4;
  T* lo = a.lam_cur ? a.lam_cur + rb * rstride + (size_t)p * 4 : nullptr;

  // sums over frequency of the partials, in the sweep precision (FP32: each is a sum
  // of nfreq terms whose rounding stays at the level of the FP32 terms themselves)
  T aT = 0, aSM[4] = {0, 0, 0, 0}, aSO[4] = {0, 0, 0, 0}, aCM[4] = {0, 0, 0, 0};
  T aKM[6] = {0, 0, 0, 0, 0, 0}, aKO[6] = {0, 0, 0, 0, 0, 0};
  // The corner values of one frequency: the adjoint of the plane above (or the seed)
  // and the forward state of the plane below.  In FP32 they are loaded one frequency
  // ahead, so that a frequency's arithmetic covers the latency of the next one's
  // loads.  The loop is instantiated for the presence of the plane above (HL) and
  // below (HI), which is the same for every thread of a launch.
  struct Corners {
    T l[4][4], m[4][4];
  };
  auto run = [&](auto has_lp, auto has_ip) __attribute__((always_inline)) {
    constexpr bool HL = decltype(has_lp)::value, HI = decltype(has_ip)::value;
    auto issue = [&](int f, Corners& c) __attribute__((always_inline)) {
      const size_t fo = (size_t)f * fstride;
      if constexpr (HL) {
        load4(lp + fo + 4 * (size_t)tN.i00, c.l[0]);
        load4(lp + fo + 4 * (size_t)tN.i10, c.l[1]);
        load4(lp + fo + 4 * (size_t)tN.i01, c.l[2]);
        load4(lp + fo + 4 * (size_t)tN.i11, c.l[3]);
      } else {
        load4(sp + fo, c.l[0]);
      }
      if constexpr (HI && MODE == 0) {
        load4(ip + fo + 4 * (size_t)ps.sM.i00, c.m[0]);
        load4(ip + fo + 4 * (size_t)ps.sM.i10, c.m[1]);
        load4(ip + fo + 4 * (size_t)ps.sM.i01, c.m[2]);
        load4(ip + fo + 4 * (size_t)ps.sM.i11, c.m[3]);
      }
    };
    auto body = [&](int f, const Corners& c) __attribute__((always_inline)) {
      const size_t fo = (size_t)f * fstride;
      T lam[4];
      if constexpr (HL) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
          lam[s] = n00 * c.l[0][s] + n10 * c.l[1][s] + n01 * c.l[2][s] + n11 * c.l[3][s];
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) lam[s] = c.l[0][s];
      }
      T IM[4];
      if constexpr (HI && MODE == 1) {
        upwind_bez9(ip + fo, sM9, bwx, bwy, IM);
      } else if constexpr (HI) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
          IM[s] = w00 * c.m[0][s] + w10 * c.m[1][s] + w01 * c.m[2][s] + w11 * c.m[3][s];
      } else {
        IM[0] = a.ibound;
        IM[1] = IM[2] = IM[3] = T(0);
      }
      const T ph = s_phi[f];
      const T tau = tau0 * ph;
      const Coefs<T> cf = coefficients(tau);
      // the forward update at O again (Eq. fsbez), instead of reading the stored I_O
      T KIM[4], b[4], IO[4];
      kprime_apply(eMv, rMv, IM, KIM);
#pragma unroll
      for (int s = 0; s < 4; ++s)
        b[s] = cf.e * IM[s] - cf.psiM * KIM[s] + cf.omM * SMt[s] + cf.omO * SOt[s] +
               cf.omC * cMt[s];
      const StokesFreq<T> F = stokes_freq(KO, cf.psiO);
      stokes_solve<1>(KO, F, b, IO);
      // lambda_b = (1 + psi'_O K'_O)^-T lambda
      T lb[4];
      stokes_solve<-1>(KO, F, lam, lb);
      // lambda_b^T K'_O I_O is linear in the six entries of K'_O: its partials QO[c]
      // give both the psi'_O term and the K'_O partials
      T QO[6];
      kprime_forms(lb, IO, QO);
      T gPO = -(eOv[0] * QO[0] + eOv[1] * QO[1] + eOv[2] * QO[2] + rOv[0] * QO[3] +
                rOv[1] * QO[4] + rOv[2] * QO[5]);
#pragma unroll
      for (int c = 0; c < 6; ++c) aKO[c] -= cf.psiO * QO[c];
      T gE = 0, gPM = 0, gOM = 0, gOO = 0, gOC = 0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        gE += lb[s] * IM[s];
        gPM -= lb[s] * KIM[s];
        gOM += lb[s] * SMt[s];
        gOO += lb[s] * SOt[s];
        gOC += lb[s] * cMt[s];
        aSM[s] += cf.omM * lb[s];
        aSO[s] += cf.omO * lb[s];
        aCM[s] += cf.omC * lb[s];
      }
      aT += ph * coef_tau_grad(cf, gE, gPM, gPO, gOM, gOO, gOC);
      kprime_outer(cf.psiM, lb, IM, aKM);
      if (lo) {
        // Lambda = (e - psi'_M K'_M)^T lambda_b
        T KT[4];
        kprime_apply(eMv, rMn, lb, KT);
        T out[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) out[s] = cf.e * lb[s] - cf.psiM * KT[s];
        store4_nt(lo + fo, out);
      }
    };
    if constexpr (sizeof(T) == 4) {
      Corners cA, cB;
      issue(0, cA);
      for (int f = 0; f < a.nfreq; f += 2) {
        if (f + 1 < a.nfreq) issue(f + 1, cB);
        body(f, cA);
        if (f + 1 >= a.nfreq) break;
        if (f + 2 < a.nfreq) issue(f + 2, cA);
        body(f + 1, cB);
      }
    } else {
      // FP64: one buffer (a second one does not fit in the registers of one wave)
      for (int f = 0; f < a.nfreq; ++f) {
        Corners c;
        issue(f, c);
        body(f, c);
      }
    }
  };
  using yes = std::true_type;
  using no = std::false_type;
  if (lp) {
    if (ip) run(yes{}, yes{});
    else run(yes{}, no{});
  } else {
    if (ip) run(no{}, yes{});
    else run(no{}, no{});
  }

  double gT = aT, gSM[4], gSO[4], gCM[4], gKM[6], gKO[6];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    gSM[s] = aSM[s];
    gSO[s] = aSO[s];
    gCM[s] = aCM[s];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    gKM[c] = aKM[c];
    gKO[c] = aKO[c];
  }
  // control points (branch of the forward evaluation)
  double gSP[4] = {0, 0, 0, 0}, gR = 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (ps.hasP) {
      double d[4];
      if (a.parabolic)
        parabolic_cm_grad(ps.SM[s], ps.SO[s], ps.SP[s], ps.ratio, d);
      else
        besser_cm_grad(ps.SM[s], ps.SO[s], ps.SP[s], ps.ratio, d);
      gSM[s] += gCM[s] * d[0];
      gSO[s] += gCM[s] * d[1];
      gSP[s] += gCM[s] * d[2];
      gR += gCM[s] * d[3];
    } else {
      gSM[s] += 0.5 * gCM[s];
      gSO[s] += 0.5 * gCM[s];
    }
  }
  // ratio = tau0M / tau0P, tau0M = (kapM + kapO) dsM / 2, tau0P = (kapO + kapP) dsP / 2
  double gT0P = 0.0;
  if (ps.hasP) {
    gT += gR / ps.tau0P;
    gT0P = -gR * ps.ratio / ps.tau0P;
  }
  double gkM = 0.5 * ps.dsM * gT;
  double gkO = 0.5 * ps.dsM * gT + 0.5 * ps.dsP * gT0P;
  double gkP = 0.5 * ps.dsP * gT0P;
  // S_X = (emission table) eps_X / kap_X
  double geM[6], geO[6], geP[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double m = 0.0, o = 0.0, q = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      m += gSM[s] * rc.emis[s][c];
      o += gSO[s] * rc.emis[s][c];
      q += gSP[s] * rc.emis[s][c];
    }
    geM[c] = m * ps.ikM;
    geO[c] = o * ps.ikO;
    geP[c] = q * ps.ikP;
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    gkM -= gSM[s] * ps.SM[s] * ps.ikM;
    gkO -= gSO[s] * ps.SO[s] * ps.ikO;
    gkP -= gSP[s] * ps.SP[s] * ps.ikP;
  }
  // K'_X = eta_X / kap_X
  double ghM[6], ghO[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    ghM[c] = gKM[c] * ps.ikM;
    ghO[c] = gKO[c] * ps.ikO;
    gkM -= gKM[c] * ps.etaM[c] * ps.ikM * ps.ikM;
    gkO -= gKO[c] * ps.etaO[c] * ps.ikO * ps.ikO;
  }
  T* go = a.g_o + (size_t)rb * 13 * a.np + p;
  T* gm = a.g_m + (size_t)rb * 13 * a.np + p;
  const size_t np = (size_t)a.np;
  go[0] = (T)gkO;
  gm[0] = (T)gkM;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    go[(1 + c) * np] = (T)ghO[c];
    gm[(1 + c) * np] = (T)ghM[c];
    go[(7 + c) * np] = (T)geO[c];
    gm[(7 + c) * np] = (T)geM[c];
  }
  if (ps.hasP) {
    T* gp = a.g_p + (size_t)rb * 7 * a.np + p;
    gp[0] = (T)gkP;
#pragma unroll
    for (int c = 0; c < 6; ++c) gp[(1 + c) * np] = (T)geP[c];
  }
}

// Gather the per-(node, ray) partials of one plane onto the coefficient
// gradients of planes kM, kO and kP (fixed ray order per component, no atomics).
template <class T>
struct GatherArgs {
  const T* g_o;
  const T* g_m;
  const T* g_p;
  const RayConsts* rays;
  double* grad;       // [13][N]: kappa, propmat[6], emis[6]
  size_t N;
  int nx, ny, np;
  int kO, kM, kP;
  double dzM, dzP, inv_dx, inv_dy;
  int ray0, nrb;
  const T* kappa;     // the coefficients (MODE 1: the Bezier partials depend on them)
  const T* prop;
  const T* emis;
};

// blockIdx.y: component group (0: the 13 at O; 1, 2: the 13 at M in two halves; 3: the
// 7 at P), so that four threads share a node and each stencil is built once per group.
template <class T, int MODE>
__global__ void __launch_bounds__(256) k_adjoint_gather(const GatherArgs<T> a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int grp = blockIdx.y;
  if (q >= a.np || (grp == 3 && a.kP < 0)) return;
  const int i = q % a.nx, j = q / a.nx;
  const size_t np = (size_t)a.np;
  const int c0 = (grp == 2) ? 7 : 0;
  const int nc = (grp == 0) ? 13 : (grp == 1 ? 7 : (grp == 2 ? 6 : 7));
  double acc[13];
#pragma unroll
  for (int c = 0; c < 13; ++c) acc[c] = 0.0;
  if (grp == 0) {
    for (int rb = 0; rb < a.nrb; ++rb) {
      const T* go = a.g_o + (size_t)rb * 13 * np + q;
#pragma unroll
      for (int c = 0; c < 13; ++c) acc[c] += go[c * np];
    }
#pragma unroll
    for (int c = 0; c < 13; ++c) a.grad[c * a.N + (size_t)a.kO * np + q] += acc[c];
    return;
  }
  const bool atM = (grp < 3);
  for (int rb = 0; rb < a.nrb; ++rb) {
    const RayConsts& rc = a.rays[a.ray0 + rb];
    const double inv_mu = 1.0 / fabs(rc.mu);
    const double ds = (atM ? a.dzM : a.dzP) * inv_mu;
    const double sds = atM ? -ds : ds;   // M upwind, P downwind, as in the sweep
    const T* gb = atM ? a.g_m + ((size_t)rb * 13 + c0) * np : a.g_p + (size_t)rb * 7 * np;
    if constexpr (MODE == 0) {
      const Stencil t = make_tstencil(i, j, a.nx, a.ny, sds * rc.sx * a.inv_dx,
                                      sds * rc.sy * a.inv_dy);
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        if (c < nc) {
          const T* g = gb + c * np;
          acc[c] += t.w00 * g[t.i00] + t.w10 * g[t.i10] + t.w01 * g[t.i01] + t.w11 * g[t.i11];
        }
      }
    } else {
      // the transposed 9-point Bezier of each coefficient, whose clamps depend on the
      // coefficient's values around q
      const Bez9Geom gm = bez9_geom(sds * rc.sx * a.inv_dx, sds * rc.sy * a.inv_dy, a.nx, a.ny);
      const BezW<double> wx = bez_weights(gm.tx), wy = bez_weights(gm.ty);
      int rowb[5], coli[5], prow[3], pcol[3];
#pragma unroll
      for (int d = 0; d < 5; ++d) {
        rowb[d] = wrapi(j + d - 2, a.ny) * a.nx;
        coli[d] = wrapi(i + d - 2, a.nx);
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        prow[d] = wrapi(j - gm.fv + d - 1, a.ny) * a.nx;
        pcol[d] = wrapi(i - gm.fu + d - 1, a.nx);
      }
      const size_t kb = (size_t)(atM ? a.kM : a.kP) * np;
#pragma unroll 1
      for (int c = 0; c < nc; ++c) {
        // coefficient c of the group: M, first half kappa and propmat; M, second half
        // emis; P: kappa and emis
        const int cg = c0 + c;
        const T* fld = (!atM) ? (c == 0 ? a.kappa : a.emis + (size_t)(c - 1) * a.N)
                              : (cg == 0 ? a.kappa
                                         : (cg < 7 ? a.prop + (size_t)(cg - 1) * a.N
                                                   : a.emis + (size_t)(cg - 7) * a.N));
        const T* fb = fld + kb;
        const T* g = gb + c * np;
        double out[1] = {0.0};
        bez9_adjoint_gather<double, 1>(
            wx, wy,
            [&](int r, int cc, double v[1]) { v[0] = (double)fb[rowb[r + 2] + coli[cc + 2]]; },
            [&](int r, int cc, double w[1]) { w[0] = (double)g[prow[r + 1] + pcol[cc + 1]]; },
            out);
#pragma unroll
        for (int cc = 0; cc < 7; ++cc)   // (a register array takes no run-time index)
          if (cc == c) acc[cc] += out[0];
      }
    }
  }
  if (atM) {
#pragma unroll
    for (int c = 0; c < 7; ++c)
      if (c < nc) a.grad[(c0 + c) * a.N + (size_t)a.kM * np + q] += acc[c];
  } else {
    // eta_I and the six emissivities at P (gradient rows 0 and 7..12)
    a.grad[(size_t)a.kP * np + q] += acc[0];
#pragma unroll
    for (int c = 1; c < 7; ++c) a.grad[(6 + c) * a.N + (size_t)a.kP * np + q] += acc[c];
  }
}

// Add the FP64 gradient accumulator to the caller's arrays.
template <class T>
__global__ void __launch_bounds__(256) k_grad_out(const double* __restrict__ grad, size_t N,
                                                  T* __restrict__ gk, T* __restrict__ gp,
                                                  T* __restrict__ ge) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < N;
       p += (size_t)gridDim.x * blockDim.x) {
    gk[p] += (T)grad[p];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      gp[c * N + p] += (T)grad[(1 + c) * N + p];
      ge[c * N + p] += (T)grad[(7 + c) * N + p];
    }
  }
}

}  // namespace porta
