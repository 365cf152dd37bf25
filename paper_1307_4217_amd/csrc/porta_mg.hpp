// Kernels of the non-linear multigrid iteration (Sect. 5): the statistical-equilibrium
// operator L(rho) rho, restriction, prolongation and injection between a grid and the
// next coarser one, and the maximum relative change between two iterates.
//
// Grids: coarse node (i, j, k) is fine node (2i, 2j, 2k); x and y are periodic
// (n_x, n_y even, coarse n_x / 2), z is not (n_z odd, coarse (n_z + 1) / 2).  Fields
// are [c][N] with x fastest.
#pragma once

#include <hip/hip_runtime.h>

#include "porta_math.hpp"

namespace porta {

// Periodic index in [0, n).
__device__ inline int wrap_index(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// ---------------------------------------------------------------------------
// out = base + sign * L(rho) rho at every point, where (Sect. 2, Eq. nonlte, two-level
// atom, S^K_Q standing for rho):
//   K = 0:  S00 - (1-eps) J00
//   K = 2:  [1 + delta (1-eps)] S2_Q + i (1-eps) H sum_Q' <Q|b.J|Q'> S2_Q' - (1-eps) w2 conj(J2_Q)
// in the real rows (Q = 0, Re/Im Q = 1, Re/Im Q = 2) of the Jacobi update; base is
// an array [6][N] or, when absent, (eps_c B, 0, ...).
// ---------------------------------------------------------------------------
struct SeeOpArgs {
  const double* jkq;
  const double* s;
  const double* base;   // or nullptr
  double* out;
  const double* hanle;  // or nullptr
  const double* bhat;   // or nullptr
  size_t N;
  double sign, eps_c, delta2, w2, planck;
};

__global__ void __launch_bounds__(256) k_see_operator(const SeeOpArgs a) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.N) return;
  const size_t N = a.N;
  const double oe = 1.0 - a.eps_c;
  const double c = oe * a.w2;
  double s2[5], y[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) s2[q] = a.s[(q + 1) * N + p];
  const double ad = 1.0 + a.delta2 * oe;
  const double h = a.hanle ? oe * a.hanle[p] : 0.0;
  if (h != 0.0) {
    const double bx = a.bhat ? a.bhat[p] : 0.0;
    const double by = a.bhat ? a.bhat[N + p] : 0.0;
    const double bz = a.bhat ? a.bhat[2 * N + p] : 1.0;
    double A[5][5];
    hanle_system(ad, h, bx, by, bz, A);
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < 5; ++k) acc += A[r][k] * s2[k];
      y[r] = acc;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 5; ++q) y[q] = ad * s2[q];
  }
  y[0] -= c * a.jkq[4 * N + p];
  y[1] -= c * a.jkq[5 * N + p];
  y[2] += c * a.jkq[6 * N + p];
  y[3] -= c * a.jkq[7 * N + p];
  y[4] += c * a.jkq[8 * N + p];
  const double l0 = a.s[p] - oe * a.jkq[p];
  a.out[p] = (a.base ? a.base[p] : a.eps_c * a.planck) + a.sign * l0;
#pragma unroll
  for (int q = 0; q < 5; ++q)
    a.out[(q + 1) * N + p] = (a.base ? a.base[(q + 1) * N + p] : 0.0) + a.sign * y[q];
}

// ---------------------------------------------------------------------------
// Restriction (Sect. 5.2): thread = coarse node; the weighted mean of the 3^3 fine
// nodes around it with weights w(dx) w(dy) w(dz), w(0) = 1, w(+-1) = 1/2 (the adjoint
// of tri-linear prolongation), over the nodes that exist (2 x 3^2 at a z boundary),
// for ncomp components.  Optionally also emis = kappa_c * out in the sweep precision.
// ---------------------------------------------------------------------------
template <class T>
struct RestrictArgs {
  const double* f;
  double* out;
  const T* kappa_c;  // or nullptr
  T* emis_c;         // or nullptr
  int nx, ny, nz, ncomp;
};

template <class T>
__global__ void __launch_bounds__(256) k_restrict(const RestrictArgs<T> a) {
  const int nxc = a.nx / 2, nyc = a.ny / 2, nzc = (a.nz + 1) / 2;
  const size_t Nc = (size_t)nxc * nyc * nzc, Nf = (size_t)a.nx * a.ny * a.nz;
  const size_t pc = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pc >= Nc) return;
  const int ic = (int)(pc % nxc), jc = (int)((pc / nxc) % nyc), kc = (int)(pc / ((size_t)nxc * nyc));
  int col[3], row[3];
  const double w[3] = {0.5, 1.0, 0.5};
  for (int d = 0; d < 3; ++d) {
    col[d] = wrap_index(2 * ic + d - 1, a.nx);
    row[d] = wrap_index(2 * jc + d - 1, a.ny);
  }
  const int dz0 = (kc == 0) ? 1 : 0, dz1 = (kc == nzc - 1) ? 1 : 2;
  const double wz = (dz0 == 0 && dz1 == 2) ? 2.0 : 1.5;
  const double inv = 1.0 / (4.0 * wz);
  for (int c = 0; c < a.ncomp; ++c) {
    const double* fc = a.f + (size_t)c * Nf;
    double acc = 0.0;
    for (int dz = dz0; dz <= dz1; ++dz) {
      const double* plane = fc + (size_t)(2 * kc + dz - 1) * a.nx * a.ny;
      double ap = 0.0;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const double* r = plane + (size_t)row[dy] * a.nx;
        ap += w[dy] * (0.5 * r[col[0]] + r[col[1]] + 0.5 * r[col[2]]);
      }
      acc += w[dz] * ap;
    }
    const double v = acc * inv;
    a.out[(size_t)c * Nc + pc] = v;
    if (a.emis_c) a.emis_c[(size_t)c * Nc + pc] = (T)((double)a.kappa_c[pc] * v);
  }
}

// ---------------------------------------------------------------------------
// Prolongation of a coarse difference (Sect. 5.2): thread = fine node; fine += P(a - b)
// (b may be absent).  Along each axis a fine node on a coarse node takes its value;
// one between coarse nodes takes the linear mean of the two (order 1) or the cubic
// through four coarse nodes (order 3: centred, periodic in x and y; shifted inward next
// to the ends of z).  The tensor product gives tri-linear or tri-cubic-centred
// interpolation, bilinear / bicubic on coarse planes and linear / cubic on coarse
// lines.  Optionally emis = kappa * fine.
// ---------------------------------------------------------------------------
template <class T>
struct ProlongArgs {
  const double* ca;
  const double* cb;   // or nullptr
  double* fine;
  const T* kappa;     // or nullptr
  T* emis;            // or nullptr
  int nx, ny, nz, ncomp, order;
};

// Coarse indices and weights along one axis for fine index f (n coarse nodes).
__device__ inline int prolong_axis(int f, int n, bool periodic, int order, int idx[4],
                                   double w[4]) {
  const int c = f >> 1;
  if ((f & 1) == 0) {
    idx[0] = c;
    w[0] = 1.0;
    return 1;
  }
  if (order == 1) {
    idx[0] = c;
    idx[1] = (c + 1 == n) ? 0 : c + 1;   // only reached on a periodic axis at the seam
    w[0] = w[1] = 0.5;
    return 2;
  }
  int base = c - 1;
  if (!periodic) base = base < 0 ? 0 : (base > n - 4 ? n - 4 : base);
  const double x = c + 0.5;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double v = 1.0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (b != a) v *= (x - (base + b)) / (double)(a - b);
    w[a] = v;
    idx[a] = periodic ? wrap_index(base + a, n) : base + a;
  }
  return 4;
}

template <class T>
__global__ void __launch_bounds__(256) k_prolong(const ProlongArgs<T> a) {
  const int nxc = a.nx / 2, nyc = a.ny / 2, nzc = (a.nz + 1) / 2;
  const size_t Nc = (size_t)nxc * nyc * nzc, Nf = (size_t)a.nx * a.ny * a.nz;
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Nf) return;
  const int i = (int)(p % a.nx), j = (int)((p / a.nx) % a.ny), k = (int)(p / ((size_t)a.nx * a.ny));
  int xi[4], yi[4], zi[4];
  double xw[4], yw[4], zw[4];
  const int nxs = prolong_axis(i, nxc, true, a.order, xi, xw);
  const int nys = prolong_axis(j, nyc, true, a.order, yi, yw);
  const int nzs = prolong_axis(k, nzc, false, a.order, zi, zw);
  for (int c = 0; c < a.ncomp; ++c) {
    double acc = 0.0;
    for (int dz = 0; dz < nzs; ++dz)
      for (int dy = 0; dy < nys; ++dy) {
        const size_t row = (size_t)c * Nc + ((size_t)zi[dz] * nyc + yi[dy]) * nxc;
        const double wzy = zw[dz] * yw[dy];
        for (int dx = 0; dx < nxs; ++dx) {
          const size_t q = row + xi[dx];
          acc += wzy * xw[dx] * (a.cb ? a.ca[q] - a.cb[q] : a.ca[q]);
        }
      }
    const size_t o = (size_t)c * Nf + p;
    const double v = a.fine[o] + acc;
    a.fine[o] = v;
    if (a.emis) a.emis[o] = (T)((double)a.kappa[p] * v);
  }
}

// Values of a fine field at the coarse nodes, ncomp components of E.
template <class E>
__global__ void __launch_bounds__(256) k_inject(const E* __restrict__ f, E* __restrict__ out,
                                                int nx, int ny, int nz, int ncomp) {
  const int nxc = nx / 2, nyc = ny / 2, nzc = (nz + 1) / 2;
  const size_t Nc = (size_t)nxc * nyc * nzc, Nf = (size_t)nx * ny * nz;
  const size_t pc = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pc >= Nc) return;
  const int ic = (int)(pc % nxc), jc = (int)((pc / nxc) % nyc), kc = (int)(pc / ((size_t)nxc * nyc));
  const size_t pf = ((size_t)(2 * kc) * ny + 2 * jc) * nx + 2 * ic;
  for (int c = 0; c < ncomp; ++c) out[(size_t)c * Nc + pc] = f[(size_t)c * Nf + pf];
}

// emis = kappa * s for ncomp components (s FP64 [ncomp][N], kappa and emis in T).
template <class T>
__global__ void __launch_bounds__(256) k_emissivity(const T* __restrict__ kappa,
                                                    const double* __restrict__ s,
                                                    T* __restrict__ emis, size_t N, int ncomp) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const double k = (double)kappa[p];
  for (int c = 0; c < ncomp; ++c) emis[(size_t)c * N + p] = (T)(k * s[(size_t)c * N + p]);
}

// Per-block maximum of |a - b| / |a| over the first component (R_c between iterates).
__global__ void __launch_bounds__(256) k_rel_change(const double* __restrict__ a,
                                                    const double* __restrict__ b, size_t N,
                                                    double* __restrict__ blockmax) {
  __shared__ double red[256];
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  red[threadIdx.x] = (p < N) ? fabs(a[p] - b[p]) / fabs(a[p]) : 0.0;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) blockmax[blockIdx.x] = red[0];
}

}  // namespace porta
