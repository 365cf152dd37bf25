// porta_faces.hpp -- the plane step of the sweep with M and P on the first face of
// the grid that the short characteristic crosses (Sect. 3.1: M and P may lie on a
// vertical plane of the grid instead of a horizontal one).
//
// With uniform spacing in x and y the first face is of the same kind for every node
// of a plane, for a given ray: the horizontal plane next to it (within one cell),
// a vertical plane x = const through the neighbouring column, or y = const through
// the neighbouring row.  On a vertical face the point is interpolated bilinearly in
// (y, z) or (x, z) from two nodes of plane k itself and two of the upwind plane, so
// the nodes of plane k depend on each other along the ray's horizontal direction and,
// x and y being periodic, around the box.  The plane is then the fixed point of its
// node equations.  A block holds one ray and a few frequencies of a whole plane and
// marches across it row by row: each step solves one row of nodes (the lanes, at
// consecutive addresses) from the previous row (kept in LDS, in FP64 in either
// precision) and the upwind plane.  A
// ray that reaches an x = const face before a y = const one is solved on a transposed
// copy of the transfer coefficients (its own plane states transposed too), so that its
// in-plane dependencies also run from row to row.  The march starts m rows early: the
// part of I_M taken from plane k carries the weight 1 - t_z per
// step (t_z the fraction of the layer the ray descends while crossing a cell), and the
// rest of the update is a contraction, so after m >= ln(tol)/ln(1 - t_z) steps the
// starting guess no longer shows at the working precision and the remaining rows are
// the fixed point.  The frequency-independent work (interpolation of the transfer
// coefficients on the faces, S, K', control points, in FP64) is done once per node and
// ray by a parallel kernel before the march, which reads its results in the sweep
// precision as rows of a plane-sized table.
#pragma once

#include "porta_kernels.hpp"

namespace porta {

// The working frame of a ray: the grid as stored, or with x and y exchanged for a ray
// that meets a vertical face x = const before one y = const, so that in the working
// frame the first vertical face is always y = const (ties also go to y).
struct Frame {
  bool tr;                 // x and y exchanged
  int nx, ny;              // sizes in the working frame
  double inv_dx, inv_dy;
  double sx, sy;           // horizontal direction of the ray in the working frame
};

__device__ inline Frame ray_frame(const RayConsts& rc, int nx, int ny, double inv_dx,
                                  double inv_dy) {
  Frame f;
  f.tr = fabs(rc.sx) * inv_dx > fabs(rc.sy) * inv_dy;
  f.nx = f.tr ? ny : nx;
  f.ny = f.tr ? nx : ny;
  f.inv_dx = f.tr ? inv_dy : inv_dx;
  f.inv_dy = f.tr ? inv_dx : inv_dy;
  f.sx = f.tr ? rc.sy : rc.sx;
  f.sy = f.tr ? rc.sx : rc.sy;
  return f;
}

// First face crossed from a node, going upwind (dir = -1, point M) or downwind
// (dir = +1, point P), in the working frame: the plane next to it (kind 0) or the
// vertical plane y = const of the neighbouring row (kind 2), with the offsets and
// fractions of the bilinear interpolation on that face.  The path to the plane and the
// shift on it are formed as in setup_point, so that a horizontal face gives the
// plane-hop kernel's stencil.
struct FaceGeom {
  int kind;       // 0: horizontal plane kz; 2: y = const (row j + off)
  int off;        // +-1: the neighbouring row (kind 2)
  double ds;      // path length from O to the face
  double u, v;    // offsets of the point in cells (kind 0: both; kind 2: u)
  double tz;      // kind 2: fraction of the way from plane k to plane kz
};

__device__ inline FaceGeom face_geom(double mu, const Frame& fr, int dir, double dz) {
  const double inv_mu = 1.0 / fabs(mu);
  const double sz = dz * inv_mu;
  const double uy = dir * fr.sy;
  const double syf = uy != 0.0 ? 1.0 / (fabs(uy) * fr.inv_dy) : INFINITY;
  FaceGeom g;
  if (sz <= syf) {   // the frame puts the x face no nearer than the y face
    g.kind = 0;
    g.off = 0;
    g.ds = sz;
    g.u = dir * (sz * fr.sx * fr.inv_dx);
    g.v = dir * (sz * fr.sy * fr.inv_dy);
    g.tz = 1.0;
  } else {
    g.kind = 2;
    g.off = uy > 0.0 ? 1 : -1;
    g.ds = syf;
    g.u = syf * (dir * fr.sx) * fr.inv_dx;
    g.v = 0.0;
    g.tz = syf / sz;
  }
  return g;
}

// The four nodes and weights of a face point of node (i, j) of the working frame: on a
// horizontal face the bilinear stencil on plane kz; on a y face nodes 0, 1 on plane k
// (row j + off) and 2, 3 the same columns on plane kz.  Indices within a plane.
struct FaceStencil {
  int n[4];
  double w[4];
  double a, b;    // the same as two linear steps: a between nodes 0, 1 (and 2, 3), b from
                  // the pair 0, 1 to the pair 2, 3
  bool inplane;   // nodes 0 and 1 lie on plane k itself
};

__device__ inline FaceStencil face_stencil(const FaceGeom& g, int i, int j, int nx, int ny) {
  FaceStencil s;
  if (g.kind == 0) {
    const Stencil b = make_stencil(i, j, nx, ny, g.u, g.v);
    s.n[0] = b.i00; s.n[1] = b.i10; s.n[2] = b.i01; s.n[3] = b.i11;
    s.w[0] = b.w00; s.w[1] = b.w10; s.w[2] = b.w01; s.w[3] = b.w11;
    // the fractions of the cell, reduced as make_stencil reduces them
    const double u = g.u - nx * floor(g.u / nx), v = g.v - ny * floor(g.v / ny);
    s.a = u - floor(u);
    s.b = v - floor(v);
    s.inplane = false;
    return s;
  }
  s.inplane = true;
  const double fu = floor(g.u), f = g.u - fu;
  const int jc = wrapi(j + g.off, ny);
  const int i0 = wrapi(i + (int)fu, nx);
  // |u| <= 1, and at |u| = 1 (f = 0) the second corner has weight 0: take the first
  // again, so the corners of row j are always columns i - 1, i or i + 1
  const int i1 = f == 0.0 ? i0 : ((i0 + 1 == nx) ? 0 : i0 + 1);
  s.n[0] = jc * nx + i0; s.n[1] = jc * nx + i1;
  s.n[2] = s.n[0];       s.n[3] = s.n[1];
  s.w[0] = (1.0 - f) * (1.0 - g.tz);
  s.w[1] = f * (1.0 - g.tz);
  s.w[2] = (1.0 - f) * g.tz;
  s.w[3] = f * g.tz;
  s.a = f;
  s.b = g.tz;
  return s;
}

// A field at a face point: planes k (offset bk) and kz (offset bz).
template <class T>
__device__ inline double face_val(const T* __restrict__ f, const FaceStencil& s, size_t bk,
                                  size_t bz) {
  const size_t b01 = s.inplane ? bk : bz;
  return s.w[0] * (double)f[b01 + s.n[0]] + s.w[1] * (double)f[b01 + s.n[1]] +
         s.w[2] * (double)f[bz + s.n[2]] + s.w[3] * (double)f[bz + s.n[3]];
}

template <class T>
struct FacesArgs {
  const T* kappa;    // transfer coefficients as stored
  const T* prop;
  const T* emis;
  const T* kappa_t;  // the same with x and y exchanged in every plane, or nullptr if no ray
  const T* prop_t;   // of the call needs them
  const T* emis_t;
  const RayConsts* rays;
  const T* phi;
  const double* wn;
  const T* iprev;    // upwind plane states ([ray][freq][node][4], node in the ray's
                     // working frame), or nullptr: the boundary
  T* inext;          // states of plane k, same layout
  int top;           // inext is I_top: nodes in the stored frame
  double* jchunk;    // [ray][chunk][5][node] (working frame): per frequency chunk,
                     // sum_j W_j I_i and sum_j W_j Lambda*
  T* cache;          // [ray][kFacesCache][node] (working frame): the set-up of each node
  size_t N;
  int nx, ny, np, nfreq, fchunk, nchunk;
  int kO, kM, kP;    // plane of O, upwind plane, downwind plane (-1: none)
  double dzM, dzP;
  double inv_dx, inv_dy;
  int ray0;
  int parabolic;
  double tol;        // the march's starting guess is damped below tol (the unit roundoff)
  T ibound;
  int nrb;           // rays of the launch
};

// Workgroups of a launch go to the 8 XCDs in turn (workgroup w to XCD w % 8).  The march
// takes a one-dimensional grid of 8 * ceil(nrb / 8) * nchunk workgroups and gives XCD x
// the rays x, x + 8, x + 16, ... (every inclination alike on each XCD), each ray's
// chunks one after another: they start together and walk the same rows, so the rows
// of the set-up table that every chunk of the ray reads come from that XCD's L2.
constexpr int kFacesXcds = 8;
inline int faces_grid(int nrb, int nchunk) {
  return kFacesXcds * ((nrb + kFacesXcds - 1) / kFacesXcds) * nchunk;
}

// Values of the set-up of a node and ray that the march reads, in the sweep precision:
// K'_M / eta_I entries (eta 3, rho 3), K'_O (3, 3), S_M (4), S_O (4), c_M (4), the
// optical depth tau_MO at line centre and the Lambda* factor of omega_C.
enum FacesCacheSlot {
  kCeM = 0, kCrM = 3, kCeO = 6, kCrO = 9, kCSM = 12, kCSO = 16, kCcM = 20, kCtau = 24,
  kClf = 25, kFacesCache = 26
};

// frequencies per block, at most (LDS may set fewer).  Small chunks give more blocks
// (the launch is nchunk x rays of them, of unequal lengths: the most inclined rays
// march 4x the rows of the steep ones) and more blocks per CU, and shorten the longest
// block; the set-up table is read once per chunk (from L2 for all but the first chunk
// of a ray, with the order of faces_grid).  At 256x256x128, 80 rays and 101
// frequencies, a sweep took 6.51, 6.49 and 6.37 s with FP64 chunks of 5, 6 and 7; in
// FP32, with the previous row held in FP64 (36 KB of LDS per block at chunks of 4, four
// blocks per CU), 2.53 and 2.59 s with chunks of 4 and 5.
template <class T>
__host__ __device__ constexpr int faces_chunk() {
  return sizeof(T) == 4 ? 4 : 7;
}
constexpr int kFacesMaxLanes = 512;  // columns of a plane held by one block
constexpr int kFacesMaxWarm = 65536; // warm-up rows of a march, at most
constexpr size_t kFacesLds = 65536;  // LDS of one block, at most

// LDS of the kernel: W_j and phi_j of every frequency; then (16-byte aligned) the row of
// Stokes vectors of each lane, [f][lane][4]; then the first and last lane's vectors of
// every wave, twice (rows of even and odd parity), [parity][f][wave][2][4].
template <class T>
__host__ __device__ inline size_t faces_col_offset(int nfreq) {
  return ((size_t)nfreq * (sizeof(double) + sizeof(T)) + 15) & ~(size_t)15;
}
// The previous row's Stokes vectors are kept in FP64 in either precision (see
// k_sweep_plane_faces).
template <class T>
__host__ __device__ inline size_t faces_lds_bytes(int nfreq, int fchunk, int lanes) {
  const size_t waves = (size_t)(lanes + 63) / 64;
  return faces_col_offset<T>(nfreq) + (size_t)fchunk * (lanes + 4 * waves) * 4 * sizeof(double);
}

// Frequency-independent part of the update of node p (working frame): the PointSetup of
// the plane-hop kernel with the coefficients at M and P taken on their faces.
template <class T>
__device__ inline void setup_point_faces(const T* __restrict__ kappa, const T* __restrict__ prop,
                                         const T* __restrict__ emis, const FacesArgs<T>& a,
                                         const RayConsts& rc, const FaceGeom& gM,
                                         const FaceStencil& sM, const FaceGeom& gP,
                                         const FaceStencil& sP, bool hasP, int p,
                                         PointSetup& ps) {
  const size_t N = a.N, bk = (size_t)a.kO * a.np, bM = (size_t)a.kM * a.np;
  ps.dsM = gM.ds;
  ps.kapM = face_val(kappa, sM, bk, bM);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    ps.epsM[c] = face_val(emis + c * N, sM, bk, bM);
    ps.etaM[c] = face_val(prop + c * N, sM, bk, bM);
  }
  const size_t bO = bk + p;
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
  ps.tau0M = 0.5 * (ps.kapM + ps.kapO) * ps.dsM;
  ps.hasP = hasP;
  if (hasP) {
    const size_t bP = (size_t)a.kP * a.np;
    ps.dsP = gP.ds;
    ps.kapP = face_val(kappa, sP, bk, bP);
#pragma unroll
    for (int c = 0; c < 6; ++c) ps.epsP[c] = face_val(emis + c * N, sP, bk, bP);
    ps.ikP = 1.0 / ps.kapP;
    ps.tau0P = 0.5 * (ps.kapO + ps.kapP) * ps.dsP;
    ps.ratio = ps.tau0M / ps.tau0P;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double ep = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) ep += rc.emis[s][c] * ps.epsP[c];
      ps.SP[s] = ep * ps.ikP;
      ps.cM[s] = control_cm(ps.SM[s], ps.SO[s], ps.SP[s], ps.ratio, a.parabolic != 0);
    }
  } else {
    ps.dsP = ps.kapP = ps.ikP = ps.tau0P = ps.ratio = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      ps.SP[s] = 0.0;
      ps.cM[s] = 0.5 * (ps.SM[s] + ps.SO[s]);
    }
  }
}

// The frequency-independent set-up of every node of plane kO (working frame) for every
// ray of the batch (blockIdx.y), in FP64, stored in the sweep precision.
template <class T>
__global__ void __launch_bounds__(256) k_faces_setup(const FacesArgs<T> a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x, rb = blockIdx.y;
  if (p >= a.np) return;
  const RayConsts& rc = a.rays[a.ray0 + rb];
  const Frame fr = ray_frame(rc, a.nx, a.ny, a.inv_dx, a.inv_dy);
  const T* kappa = fr.tr ? a.kappa_t : a.kappa;
  const T* prop = fr.tr ? a.prop_t : a.prop;
  const T* emis = fr.tr ? a.emis_t : a.emis;
  const FaceGeom gM = face_geom(rc.mu, fr, -1, a.dzM);
  const bool hasP = a.kP >= 0;
  const FaceGeom gP = hasP ? face_geom(rc.mu, fr, +1, a.dzP) : gM;
  const int i = p % fr.nx, j = p / fr.nx;
  const FaceStencil sM = face_stencil(gM, i, j, fr.nx, fr.ny);
  const FaceStencil sP = hasP ? face_stencil(gP, i, j, fr.nx, fr.ny) : sM;
  PointSetup ps;
  setup_point_faces(kappa, prop, emis, a, rc, gM, sM, gP, sP, hasP, p, ps);
  const double lamfac = hasP ? control_cm(0.0, 1.0, 0.0, ps.ratio, a.parabolic != 0) : 0.5;
  const size_t np = (size_t)a.np;
  T* c = a.cache + (size_t)rb * kFacesCache * np + p;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c[(kCeM + k) * np] = (T)(ps.etaM[k] * ps.ikM);
    c[(kCrM + k) * np] = (T)(ps.etaM[3 + k] * ps.ikM);
    c[(kCeO + k) * np] = (T)(ps.etaO[k] * ps.ikO);
    c[(kCrO + k) * np] = (T)(ps.etaO[3 + k] * ps.ikO);
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    c[(kCSM + s) * np] = (T)ps.SM[s];
    c[(kCSO + s) * np] = (T)ps.SO[s];
    c[(kCcM + s) * np] = (T)ps.cM[s];
  }
  c[kCtau * np] = (T)ps.tau0M;
  c[kClf * np] = (T)lamfac;
}

// One plane for one ray and one chunk of frequencies (order: faces_grid).  Lanes
// are the columns of the working frame; the block walks its rows.  Each lane keeps its
// own column's Stokes vectors of the previous row in LDS (FP64) and reads the neighbouring
// column's there too when that lane is in its wave (the lanes of a wave read before
// they write); a neighbour in another wave is read from the copy of the first and last
// lanes of every wave, which is kept for rows of either parity, so one barrier per row
// orders the exchange.  A ray whose first face is the plane itself has no in-plane
// dependency and takes no barrier.
template <class T>
__global__ void __launch_bounds__(kFacesMaxLanes) k_sweep_plane_faces(const FacesArgs<T> a) {
  // this workgroup's ray and chunk (faces_grid); the few past the last ray leave at once
  const int wx = blockIdx.x % kFacesXcds, wk = blockIdx.x / kFacesXcds;
  const int rb = wx + kFacesXcds * (wk / a.nchunk), chunk = wk % a.nchunk;
  if (rb >= a.nrb) return;
  extern __shared__ double s_tab[];
  double* s_wn = s_tab;
  T* s_phi = reinterpret_cast<T*>(s_tab + a.nfreq);
  // the in-plane chain in FP64 (D): on the thin cell steps of an inclined ray in the line
  // wings the change of I per step falls below half a unit in the last place of an FP32
  // I, so an FP32 chain would drop it at every step; the FP32 arithmetic forms that
  // change and the chain adds it in FP64 (the plane states stored are FP32)
  using D = double;
  D* s_row = reinterpret_cast<D*>(reinterpret_cast<char*>(s_tab) + faces_col_offset<T>(a.nfreq));
  const int lanes = blockDim.x, nwaves = (lanes + 63) >> 6;
  D* s_bnd = s_row + (size_t)a.fchunk * lanes * 4;
  const size_t bpar = (size_t)a.fchunk * nwaves * 8;   // one parity of s_bnd
  for (int t = threadIdx.x; t < a.nfreq; t += blockDim.x) {
    s_wn[t] = a.wn[t];
    s_phi[t] = a.phi[t];
  }
  const int f0 = chunk * a.fchunk;
  const int nf = min(a.fchunk, a.nfreq - f0);
  const RayConsts& rc = a.rays[a.ray0 + rb];
  const Frame fr = ray_frame(rc, a.nx, a.ny, a.inv_dx, a.inv_dy);
  const FaceGeom gM = face_geom(rc.mu, fr, -1, a.dzM);
  const bool chain = gM.kind != 0;   // same for the whole block
  const size_t np = (size_t)a.np;
  const T* cache = a.cache + (size_t)rb * kFacesCache * np;
  const int lane = threadIdx.x, wave = lane >> 6;
  const bool active = lane < fr.nx;
  const int nstep = fr.ny;
  // march direction: away from the row M lies on (kind 0: any order)
  const int mdir = chain ? -gM.off : 1;
  int warm = 0;
  if (chain) {
    // (1 - t_z)^warm <= tol (37 / t_z rows in FP64, 17 / t_z in FP32), however many
    // times around the box that takes; at most kFacesMaxWarm rows (t_z >= 5.6e-4 in
    // FP64), clamped before the cast
    const double q = log1p(-fmin(gM.tz, 1.0));
    const double w = q < 0.0 ? ceil(log(a.tol) / q) : 0.0;
    warm = (int)fmin(fmax(w, 0.0), (double)kFacesMaxWarm);
  }
  const size_t fstride = (size_t)a.np * 4;
  const size_t rstride = (size_t)a.nfreq * fstride;
  const T* ip = a.iprev ? a.iprev + rb * rstride : nullptr;
  T* op = a.inext + rb * rstride;
  // this lane's slots: its own column, and its copy for the other waves if it is the
  // first or last active lane of its wave
  const int side = lane == (wave << 6) ? 0 : (lane == min((wave << 6) + 63, fr.nx - 1) ? 1 : -1);
  const bool last_too = side == 0 && lane == min((wave << 6) + 63, fr.nx - 1);
  // where the two in-plane corners of the previous row are read (y face): the column's
  // own slot if its lane is in this wave, else the other wave's copy, whose offset
  // moves by bpar with the row's parity (corner = column i - 1, i or i + 1)
  int c_off[2] = {0, 0}, c_str[2] = {4 * lanes, 4 * lanes};
  bool c_bnd[2] = {false, false};
  if (chain && active) {
    const FaceStencil s0 = face_stencil(gM, lane, 0, fr.nx, fr.ny);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int l = s0.n[c] % fr.nx, w = l >> 6;
      if (w == wave) {
        c_off[c] = 4 * l;
      } else {
        c_bnd[c] = true;
        c_str[c] = 8 * nwaves;
        c_off[c] = 8 * w + 4 * (l == (w << 6) ? 0 : 1);
      }
    }
  }
  // the row before the first step: the upwind plane's values there (the guess)
  const int c_first = wrapi((mdir > 0 ? 0 : nstep - 1) - mdir * warm, nstep);
  if (chain) {
    const int cprev = wrapi(c_first - mdir, nstep);
    for (int f = 0; f < nf && active; ++f) {
      T v[4] = {a.ibound, T(0), T(0), T(0)};
      if (ip) load4(ip + (size_t)(f0 + f) * fstride + 4 * (size_t)(cprev * fr.nx + lane), v);
      const D vd[4] = {(D)v[0], (D)v[1], (D)v[2], (D)v[3]};
      store4(s_row + ((size_t)f * lanes + lane) * 4, vd);
      // the parity read at step 0 is that of step -1
      D* b = s_bnd + bpar + ((size_t)f * nwaves + wave) * 8;
      if (side >= 0) store4(b + 4 * side, vd);
      if (last_too) store4(b + 4, vd);
    }
    __syncthreads();
  }
  const T ib = a.ibound;
  double* jc = a.jchunk ? a.jchunk + ((size_t)rb * a.nchunk + chunk) * 5 * a.np : nullptr;
  for (int t = 0; t < warm + nstep; ++t) {
    const int j = wrapi(c_first + mdir * t, nstep), i = lane;
    const bool store = t >= warm;
    const size_t rd = (t & 1) ? 0 : bpar, wr = (t & 1) ? bpar : 0;   // s_bnd parities
    if (active) {
      const int p = j * fr.nx + i;                         // working frame
      const int po = fr.tr ? i * a.nx + j : p;            // stored frame
      const FaceStencil sM = face_stencil(gM, i, j, fr.nx, fr.ny);
      const T* cp = cache + p;
      const T eMv[3] = {cp[(kCeM + 0) * np], cp[(kCeM + 1) * np], cp[(kCeM + 2) * np]};
      const T rMv[3] = {cp[(kCrM + 0) * np], cp[(kCrM + 1) * np], cp[(kCrM + 2) * np]};
      const T eOv[3] = {cp[(kCeO + 0) * np], cp[(kCeO + 1) * np], cp[(kCeO + 2) * np]};
      const T rOv[3] = {cp[(kCrO + 0) * np], cp[(kCrO + 1) * np], cp[(kCrO + 2) * np]};
      const StokesOp<T> KO = stokes_op(eOv, rOv);
      T SMt[4], SOt[4], cMt[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        SMt[s] = cp[(kCSM + s) * np];
        SOt[s] = cp[(kCSO + s) * np];
        cMt[s] = cp[(kCcM + s) * np];
      }
      const T tau0 = cp[kCtau * np], lf = cp[kClf * np];
      // I_M as two linear steps (x, then z or y): a field constant over the stencil is
      // returned exactly, so the rounding of the four weights, the same for every node
      // of a ray, adds no bias that the many cell steps of an inclined ray would pile up
      const D fa = sM.a, fb = sM.b;
      const D* r0 = (c_bnd[0] ? s_bnd + rd : s_row) + c_off[0];
      const D* r1 = (c_bnd[1] ? s_bnd + rd : s_row) + c_off[1];
      D* own = s_row + 4 * (size_t)lane;
      D* bown = s_bnd + wr + 8 * (size_t)wave;
      const size_t ostore = a.top ? (size_t)po : (size_t)p;
      double jacc[4] = {0, 0, 0, 0}, lacc = 0.0;
      for (int f = 0; f < nf; ++f) {
        const int fg = f0 + f;
        D IM[4];
        T up[2][4];   // the corners on the upwind plane (or the boundary)
        if (ip) {
          const T* q = ip + (size_t)fg * fstride;
          load4(q + 4 * (size_t)sM.n[2], up[0]);
          load4(q + 4 * (size_t)sM.n[3], up[1]);
        } else {
          up[0][0] = up[1][0] = ib;
          up[0][1] = up[0][2] = up[0][3] = up[1][1] = up[1][2] = up[1][3] = T(0);
        }
        if (sM.inplane) {
          D c0[4], c1[4];
          load4(r0 + (size_t)f * c_str[0], c0);
          load4(r1 + (size_t)f * c_str[1], c1);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const D A = c0[s] + fa * (c1[s] - c0[s]);
            const D u0 = up[0][s], u1 = up[1][s];
            const D B = u0 + fa * (u1 - u0);
            IM[s] = A + fb * (B - A);
          }
        } else {
          T v0[4], v1[4];
          if (ip) {
            const T* q = ip + (size_t)fg * fstride;
            load4(q + 4 * (size_t)sM.n[0], v0);
            load4(q + 4 * (size_t)sM.n[1], v1);
          } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) v0[s] = v1[s] = up[0][s];
          }
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const D w0 = v0[s], w1 = v1[s], u0 = up[0][s], u1 = up[1][s];
            const D A = w0 + fa * (w1 - w0);
            const D B = u0 + fa * (u1 - u0);
            IM[s] = A + fb * (B - A);
          }
        }
        const T tau = tau0 * s_phi[fg];
        const Coefs<T> cf = coefficients<true>(tau);
        const T IMt[4] = {(T)IM[0], (T)IM[1], (T)IM[2], (T)IM[3]};
        T KI[4], dv[4];
        kprime_apply(eMv, rMv, IMt, KI);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          // e I_M as I_M - (1 - e) I_M (see Coefs::em1), and the change of a step summed
          // before it is added to I_M: on thin steps each term alone can fall below half
          // a unit in the last place of I_M, and dropping the source terms while keeping
          // the attenuation would bias a long chain of steps
          dv[s] = -cf.em1 * IMt[s] - cf.psiM * KI[s] + cf.omM * SMt[s] + cf.omO * SOt[s] +
                  cf.omC * cMt[s];
        }
        const StokesFreq<T> F = stokes_freq(KO, cf.psiO);
        D res[4];
        if constexpr (sizeof(T) == 4) {
          // (1 + psi'_O K'_O) I_O = I_M + d, so I_O = I_M + x with
          // (1 + psi'_O K'_O) x = d - psi'_O K'_O I_M: x in FP32, I_M + x in FP64
          T KOI[4], rhs[4], x[4];
          kprime_apply(eOv, rOv, IMt, KOI);
#pragma unroll
          for (int s = 0; s < 4; ++s) rhs[s] = dv[s] - cf.psiO * KOI[s];
          stokes_solve<1>(KO, F, rhs, x);
#pragma unroll
          for (int s = 0; s < 4; ++s) res[s] = IM[s] + (D)x[s];
        } else {
          T b[4];
#pragma unroll
          for (int s = 0; s < 4; ++s) b[s] = IM[s] + dv[s];
          stokes_solve<1>(KO, F, b, res);
        }
        const T rest[4] = {(T)res[0], (T)res[1], (T)res[2], (T)res[3]};
        if (chain) {
          store4(own + (size_t)f * lanes * 4, res);
          D* b2 = bown + (size_t)f * nwaves * 8;
          if (side >= 0) store4(b2 + 4 * side, res);
          if (last_too) store4(b2 + 4, res);
        }
        if (store) {
          // I_top of a ray in the exchanged frame goes to the grid's own indices, across
          // rows: there the plain store, whose lines the cache merges, is the faster
          if (a.top) store4(op + (size_t)fg * fstride + 4 * ostore, rest);
          else store4_nt(op + (size_t)fg * fstride + 4 * ostore, rest);
          const double W = s_wn[fg];
#pragma unroll
          for (int s = 0; s < 4; ++s) jacc[s] += W * res[s];
          lacc += W * (double)(cf.omO + lf * cf.omC);
        }
      }
      if (store && jc) {
#pragma unroll
        for (int s = 0; s < 4; ++s) __builtin_nontemporal_store(jacc[s], jc + (size_t)s * a.np + p);
        __builtin_nontemporal_store(lacc, jc + 4 * (size_t)a.np + p);
      }
    }
    // the row is complete (and its copies for the other waves) before the next reads it
    if (chain) __syncthreads();
  }
}

// Transpose every plane of nfield fields ([field][k][ny][nx] -> [field][k][nx][ny]).
template <class T>
__global__ void __launch_bounds__(256)
    k_transpose_planes(const T* __restrict__ src, T* __restrict__ dst, int nx, int ny,
                       size_t nplanes) {
  const size_t np = (size_t)nx * ny;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * nplanes) return;
  const size_t q = e / np, r = e % np;
  const int j = (int)(r % ny), i = (int)(r / ny);   // dst index r = i * ny + j
  dst[e] = src[q * np + (size_t)j * nx + i];
}

// Sum the frequency-chunk partials of every ray into the per-ray layout of the J
// reduction, from the ray's working frame to the grid's own: jpart[ray][5][node] =
// sum_chunk jchunk[ray][chunk][5][working node].  A block takes a 32 x 32 tile of the
// working frame (blockIdx.x, blockIdx.y over a square of the larger side) for one ray
// (blockIdx.z) and writes it through LDS, so that both the reads and, for a ray
// solved with x and y exchanged, the transposed writes are coalesced.
constexpr int kSumTile = 32;

__global__ void __launch_bounds__(256)
    k_sum_chunks(double* __restrict__ jpart, const double* __restrict__ jchunk,
                 const RayConsts* __restrict__ rays, int ray0, int nchunk, int nx, int ny,
                 double inv_dx, double inv_dy) {
  __shared__ double tile[kSumTile][kSumTile + 1];
  const int rb = blockIdx.z;
  const Frame fr = ray_frame(rays[ray0 + rb], nx, ny, inv_dx, inv_dy);
  const int x0 = blockIdx.x * kSumTile, y0 = blockIdx.y * kSumTile;
  if (x0 >= fr.nx || y0 >= fr.ny) return;   // the same for the whole block
  const size_t np = (size_t)nx * ny;
  const int tx = threadIdx.x % kSumTile, ty = threadIdx.x / kSumTile;   // 32 x 8
  for (int c = 0; c < 5; ++c) {
    for (int r = ty; r < kSumTile; r += 8) {
      const int xw = x0 + tx, yw = y0 + r;
      double sum = 0.0;
      if (xw < fr.nx && yw < fr.ny) {
        const size_t pw = (size_t)yw * fr.nx + xw;
        const double* src = jchunk + ((size_t)rb * nchunk * 5 + c) * np + pw;
        const size_t kst = 5 * np;   // from one chunk to the next
        int k = 0;
        // eight loads in flight, then added in chunk order (the sum of one loop)
        for (; k + 8 <= nchunk; k += 8) {
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = src[(size_t)(k + u) * kst];
#pragma unroll
          for (int u = 0; u < 8; ++u) sum += v[u];
        }
        for (; k < nchunk; ++k) sum += src[(size_t)k * kst];
      }
      tile[r][tx] = sum;
    }
    __syncthreads();
    double* out = jpart + ((size_t)rb * 5 + c) * np;
    for (int r = ty; r < kSumTile; r += 8) {
      if (!fr.tr) {
        const int xw = x0 + tx, yw = y0 + r;
        if (xw < fr.nx && yw < fr.ny) out[(size_t)yw * nx + xw] = tile[r][tx];
      } else {
        // stored (x, y) = working (y, x): consecutive lanes take consecutive stored x
        const int yw = y0 + tx, xw = x0 + r;
        if (xw < fr.nx && yw < fr.ny) out[(size_t)xw * nx + yw] = tile[tx][r];
      }
    }
    __syncthreads();
  }
}

}  // namespace porta
