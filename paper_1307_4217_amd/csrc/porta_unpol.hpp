// Sweep kernel of the unpolarized problem (Stokes I only): the scalar form of
// Eqs. fsint / fsbez with K' = 0 and the emission eps^0_0, which PORTA also solves
// (the non-LTE problem of unpolarized radiation, Sect. 1).  Same plane walk, thread
// mapping, control points and fused J reduction as k_sweep_plane; the plane state
// holds one value per node and frequency ([ray][frequency][node]).
#pragma once

#include "porta_kernels.hpp"

namespace porta {

template <class T>
__global__ void __launch_bounds__(256) k_sweep_plane_i(const PlaneArgs<T> a) {
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
  if (p >= a.np) return;   // no barrier follows
  if (rb == 0 && a.jkq)
    jreduce_point(a.jkq, a.jpart_prev, a.rays, a.ray0, gridDim.y, a.np, a.N, a.prev_off, p,
                  a.jpart_prev == nullptr, (double)a.ibound);
  const RayConsts& rc = a.rays[a.ray0 + rb];

  // M on the upwind plane, O, and P on the downwind plane (bilinear in the plane)
  const int i = p % a.nx, j = p / a.nx;
  const double inv_mu = 1.0 / fabs(rc.mu);
  const double dsM = a.dzM * inv_mu;
  const Stencil sM = make_stencil(i, j, a.nx, a.ny, -dsM * rc.sx * a.inv_dx,
                                  -dsM * rc.sy * a.inv_dy);
  const size_t bM = (size_t)a.kM * a.np, bO = (size_t)a.kO * a.np + p;
  const double kapM = bil(a.kappa + bM, sM), kapO = (double)a.kappa[bO];
  const double SM = bil(a.emis + bM, sM) / kapM, SO = (double)a.emis[bO] / kapO;
  const double tau0M = 0.5 * (kapM + kapO) * dsM;
  double cM = 0.5 * (SM + SO), lamfac = 0.5;   // no downwind plane: linear control point
  if (a.kP >= 0) {
    const double dsP = a.dzP * inv_mu;
    const Stencil sP = make_stencil(i, j, a.nx, a.ny, dsP * rc.sx * a.inv_dx,
                                    dsP * rc.sy * a.inv_dy);
    const size_t bP = (size_t)a.kP * a.np;
    const double kapP = bil(a.kappa + bP, sP);
    const double SP = bil(a.emis + bP, sP) / kapP;
    const double ratio = tau0M / (0.5 * (kapO + kapP) * dsP);
    cM = control_cm(SM, SO, SP, ratio, a.parabolic != 0);
    lamfac = control_cm(0.0, 1.0, 0.0, ratio, a.parabolic != 0);   // unit source at O
  }
  const T SMt = (T)SM, SOt = (T)SO, cMt = (T)cM, tau0 = (T)tau0M, lf = (T)lamfac;
  const T w00 = (T)sM.w00, w10 = (T)sM.w10, w01 = (T)sM.w01, w11 = (T)sM.w11;

  const size_t fstride = (size_t)a.np;
  const T* ip = a.iprev ? a.iprev + (size_t)rb * a.nfreq * fstride : nullptr;
  T* op = a.inext + (size_t)rb * a.nfreq * fstride + p;
  double jacc = 0.0, lacc = 0.0;
  // one update (the scalar Eq. fsbez) at frequency f from the upwind intensity IM
  auto update = [&](int f, T IM) __attribute__((always_inline)) {
    const Coefs<T> cf = coefficients(tau0 * s_phi[f]);
    const T x = cf.e * IM + cf.omM * SMt + cf.omO * SOt + cf.omC * cMt;
    __builtin_nontemporal_store(x, op + (size_t)f * fstride);   // as store4_nt
    const double W = s_wn[f];
    jacc += W * (double)x;
    lacc += W * (double)(cf.omO + lf * cf.omC);
  };
  if (!ip) {
    // the upwind plane is the boundary
    for (int f = 0; f < a.nfreq; ++f) update(f, a.ibound);
  } else {
    // the four corners of frequency f + 1 are loaded during the arithmetic of frequency f
    auto load = [&](int f, T v[4]) __attribute__((always_inline)) {
      const T* q = ip + (size_t)f * fstride;
      v[0] = q[sM.i00];
      v[1] = q[sM.i10];
      v[2] = q[sM.i01];
      v[3] = q[sM.i11];
    };
    T vA[4], vB[4];
    load(0, vA);
    for (int f = 0; f < a.nfreq; f += 2) {
      if (f + 1 < a.nfreq) load(f + 1, vB);
      update(f, w00 * vA[0] + w10 * vA[1] + w01 * vA[2] + w11 * vA[3]);
      if (f + 1 >= a.nfreq) break;
      if (f + 2 < a.nfreq) load(f + 2, vA);
      update(f + 1, w00 * vB[0] + w10 * vB[1] + w01 * vB[2] + w11 * vB[3]);
    }
  }
  if (a.jpart) {
    // the per-ray partial sums of J in the layout of the polarized sweep (Q, U, V zero)
    double* jp = a.jpart + (size_t)rb * 5 * a.np + p;
    jp[0] = jacc;
    jp[(size_t)a.np] = 0.0;
    jp[2 * (size_t)a.np] = 0.0;
    jp[3 * (size_t)a.np] = 0.0;
    jp[4 * (size_t)a.np] = lacc;
  }
}

}  // namespace porta
