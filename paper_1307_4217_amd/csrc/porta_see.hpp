// Statistical-equilibrium kernels of the two-level atom (Sect. 2, Eq. nonlte; the
// Jacobi update of Sect. 5) and the block maxima behind the convergence measure R_c.
#pragma once

#include <hip/hip_runtime.h>

#include "porta_math.hpp"

namespace porta {

// ---------------------------------------------------------------------------
// Statistical equilibrium (Jacobi for K = 0, Lambda iteration with Hanle
// rotation for K = 2) and the per-block maximum of |dS00| / |S00|.
// ---------------------------------------------------------------------------
template <class T>
struct SeeArgs {
  const double* jkq;
  const double* rhs;     // [6][N] replacing (eps_c B, 0, ...), or nullptr
  const double* s_old;
  double* s_new;
  const double* hanle;   // or nullptr
  const double* bhat;    // or nullptr
  const T* kappa;        // or nullptr
  T* emis_out;           // or nullptr
  double* blockmax;      // [gridDim.x] or nullptr
  size_t N;
  double eps_c, delta2, w2, planck;
};

template <class T>
__global__ void __launch_bounds__(256) k_see(const SeeArgs<T> a) {
  __shared__ double red[256];
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double rel = 0.0;
  if (p < a.N) {
    const size_t N = a.N;
    const double oe = 1.0 - a.eps_c;
    const double J00 = a.jkq[p], Lb = a.jkq[9 * N + p];
    const double so = a.s_old[p];
    const double f0 = a.rhs ? a.rhs[p] : a.eps_c * a.planck;
    const double s00 = (oe * (J00 - Lb * so) + f0) / (1.0 - oe * Lb);
    const double c = oe * a.w2;
    // rows: Re, Re, Im, Re, Im of the K = 2 equations for Q = 0, 1, 1, 2, 2
    double x[5] = {c * a.jkq[4 * N + p], c * a.jkq[5 * N + p], -c * a.jkq[6 * N + p],
                   c * a.jkq[7 * N + p], -c * a.jkq[8 * N + p]};
    if (a.rhs) {
#pragma unroll
      for (int q = 0; q < 5; ++q) x[q] += a.rhs[(q + 1) * N + p];
    }
    const double ad = 1.0 + a.delta2 * oe;
    const double h = a.hanle ? oe * a.hanle[p] : 0.0;
    if (h != 0.0) {
      const double bx = a.bhat ? a.bhat[p] : 0.0;
      const double by = a.bhat ? a.bhat[N + p] : 0.0;
      const double bz = a.bhat ? a.bhat[2 * N + p] : 1.0;
      double A[5][5];
      hanle_system(ad, h, bx, by, bz, A);
      solve_pivot<5>(A, x);
    } else {
#pragma unroll
      for (int q = 0; q < 5; ++q) x[q] /= ad;
    }
    a.s_new[p] = s00;
#pragma unroll
    for (int q = 0; q < 5; ++q) a.s_new[(q + 1) * N + p] = x[q];
    if (a.emis_out) {
      const double k = (double)a.kappa[p];
      a.emis_out[p] = (T)(k * s00);
#pragma unroll
      for (int q = 0; q < 5; ++q) a.emis_out[(q + 1) * N + p] = (T)(k * x[q]);
    }
    rel = fabs(s00 - so) / fabs(s00);
  }
  if (!a.blockmax) return;
  red[threadIdx.x] = rel;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) a.blockmax[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_max_final(const double* __restrict__ v, int n,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace porta
