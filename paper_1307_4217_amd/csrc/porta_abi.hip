// porta_abi.hip -- host side of the C ABI declared in include/porta.h:
// argument validation, workspace layout and the launch sequence of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/porta.h"
#include "porta_adjoint.hpp"
#include "porta_faces.hpp"
#include "porta_host.hpp"
#include "porta_kernels.hpp"
#include "porta_unpol.hpp"

// Workspace of porta_fs_sweep_noalloc, one copy on every device the library runs on,
// held until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace porta {
namespace host {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PORTA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return PORTA_OK;
}

int validate_prec(int prec) {
  if (prec != PORTA_F64 && prec != PORTA_F32) return fail(PORTA_EINVAL, "unknown precision %d", prec);
  return PORTA_OK;
}

}  // namespace host
}  // namespace porta

namespace {

using namespace porta;
using namespace porta::host;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
int validate_grid(const porta_grid* g) {
  if (!g) return fail(PORTA_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 2)
    return fail(PORTA_EINVAL, "grid sizes must be nx >= 1, ny >= 1, nz >= 2 (got %d %d %d)",
                g->nx, g->ny, g->nz);
  const double n = (double)g->nx * g->ny * g->nz;
  if (n * 10.0 >= 9.0e18 || (double)g->nx * g->ny >= 2147483647.0)
    return fail(PORTA_EINVAL, "grid too large");
  if (!(g->lx > 0.0) || !(g->ly > 0.0) || !std::isfinite(g->lx) || !std::isfinite(g->ly))
    return fail(PORTA_EINVAL, "horizontal periods must be positive and finite");
  if (!g->z) return fail(PORTA_EINVAL, "grid z is NULL");
  for (int k = 0; k < g->nz; ++k)
    if (!std::isfinite(g->z[k])) return fail(PORTA_EINVAL, "z[%d] is not finite", k);
  for (int k = 1; k < g->nz; ++k)
    if (!(g->z[k] > g->z[k - 1])) return fail(PORTA_EINVAL, "z must increase strictly (z[%d])", k);
  return PORTA_OK;
}

int validate_quad(const porta_quad* q) {
  if (!q) return fail(PORTA_EINVAL, "quadrature is NULL");
  if (q->nmu < 1 || q->nmu > kMaxMu) return fail(PORTA_EINVAL, "nmu must be in 1..%d", kMaxMu);
  if (q->nchi < 1 || q->nchi > 4096) return fail(PORTA_EINVAL, "nchi must be in 1..4096");
  if (q->nfreq < 1 || q->nfreq > kMaxFreq)
    return fail(PORTA_EINVAL, "nfreq must be in 1..%d", kMaxFreq);
  if (!q->mu || !q->wmu || !q->phi || !q->wfreq)
    return fail(PORTA_EINVAL, "quadrature arrays must not be NULL");
  double sw = 0.0;
  for (int a = 0; a < q->nmu; ++a) {
    if (!(q->mu[a] > 0.0 && q->mu[a] <= 1.0))
      return fail(PORTA_EINVAL, "mu[%d] = %g is not in (0, 1]", a, q->mu[a]);
    if (!(q->wmu[a] >= 0.0) || !std::isfinite(q->wmu[a]))
      return fail(PORTA_EINVAL, "wmu[%d] must be finite and >= 0", a);
    sw += q->wmu[a];
  }
  if (std::fabs(sw - 1.0) > 1e-12) return fail(PORTA_EINVAL, "wmu must sum to 1 (sum = %.17g)", sw);
  double sf = 0.0;
  for (int j = 0; j < q->nfreq; ++j) {
    if (!(q->phi[j] > 0.0) || !std::isfinite(q->phi[j]))
      return fail(PORTA_EINVAL, "phi[%d] must be finite and > 0", j);
    if (!(q->wfreq[j] >= 0.0) || !std::isfinite(q->wfreq[j]))
      return fail(PORTA_EINVAL, "wfreq[%d] must be finite and >= 0", j);
    sf += q->wfreq[j] * q->phi[j];
  }
  if (!(sf > 0.0)) return fail(PORTA_EINVAL, "sum of wfreq * phi must be > 0");
  return PORTA_OK;
}

int validate_interp(int interp) {
  if (interp != PORTA_INTERP_BILINEAR && interp != PORTA_INTERP_BEZIER2D)
    return fail(PORTA_EINVAL, "unknown interpolation mode %d", interp);
  return PORTA_OK;
}

size_t elem(int prec) { return prec == PORTA_F32 ? sizeof(float) : sizeof(double); }

// Tiles per XCD per round of the plane kernels (measured best on MI355X: 8).
int xcd_chunk(const porta_options* o) { return (o && o->xcd_remap >= 0) ? o->xcd_remap : 8; }
int parabolic_of(const porta_options* o) { return (o && o->control == PORTA_CONTROL_PARABOLIC) ? 1 : 0; }
// Stokes parameters carried by the sweep: 4, or 1 for the unpolarized problem.
int nstokes(const porta_options* o) { return (o && o->stokes == 1) ? 1 : 4; }

int validate_options(const porta_options* o) {
  if (!o) return PORTA_OK;
  if (o->ray_batch < 0 || o->block < 0 || o->xcd_remap < -1)
    return fail(PORTA_EINVAL, "ray_batch and block must be >= 0, xcd_remap >= -1");
  if (o->control != PORTA_CONTROL_BESSER && o->control != PORTA_CONTROL_PARABOLIC)
    return fail(PORTA_EINVAL, "unknown control point rule %d", o->control);
  if (o->stokes != 0 && o->stokes != 1 && o->stokes != 4)
    return fail(PORTA_EINVAL, "stokes must be 0 or 4 (Stokes vector) or 1 (intensity only)");
  if (o->ray_count < 0 || o->ray_first < 0)
    return fail(PORTA_EINVAL, "ray_first and ray_count must be >= 0");
  if (o->check_inputs != 0 && o->check_inputs != 1)
    return fail(PORTA_EINVAL, "check_inputs must be 0 or 1");
  if (o->faces != 0 && o->faces != 1) return fail(PORTA_EINVAL, "faces must be 0 or 1");
  if (o->faces_chunk < 0) return fail(PORTA_EINVAL, "faces_chunk must be >= 0");
  return PORTA_OK;
}

bool faces_of(const porta_options* o) { return o && o->faces == 1; }

// Lanes of a block of the first-face kernel (the columns of a plane in either frame)
// and the frequencies it holds: the options' faces_chunk if it fits, else as many as
// its LDS (kFacesLds) has room for, at most faces_chunk<T>(), spread evenly over the
// chunks; 0 if they do not fit.
void faces_shape(const porta_grid* g, const porta_quad* q, int prec, const porta_options* o,
                 int& lanes, int& fchunk) {
  const int n = std::max(g->nx, g->ny);
  lanes = (n + 63) / 64 * 64;
  const bool f32 = prec == PORTA_F32;
  const size_t base = f32 ? faces_lds_bytes<float>(q->nfreq, 0, lanes)
                          : faces_lds_bytes<double>(q->nfreq, 0, lanes);
  const size_t per = (f32 ? faces_lds_bytes<float>(q->nfreq, 1, lanes)
                          : faces_lds_bytes<double>(q->nfreq, 1, lanes)) - base;
  const size_t cap = f32 ? faces_chunk<float>() : faces_chunk<double>();
  const size_t fit = kFacesLds > base ? (kFacesLds - base) / per : 0;
  if (o && o->faces_chunk > 0) {
    const int want = std::min(o->faces_chunk, q->nfreq);
    fchunk = (size_t)want <= fit ? want : 0;
    return;
  }
  fchunk = (int)std::min<size_t>({cap, fit, (size_t)q->nfreq});
  if (fchunk > 0) {
    const int nchunk = (q->nfreq + fchunk - 1) / fchunk;
    fchunk = (q->nfreq + nchunk - 1) / nchunk;
  }
}

int validate_rays(const porta_quad* q, const porta_options* o) {
  if (o && o->ray_count > 0 && (int64_t)o->ray_first + o->ray_count > 2LL * q->nmu * q->nchi)
    return fail(PORTA_EINVAL, "ray range %d + %d beyond the %d rays", o->ray_first, o->ray_count,
                2 * q->nmu * q->nchi);
  return PORTA_OK;
}

// Rays of the call: [first, first + count) of the enumeration (upward rays first), all
// rays when count is 0; the part of it in one hemisphere as [lo, hi) of 0..nh-1.
void hemi_range(const porta_quad* q, const porta_options* o, int hemi, int& lo, int& hi) {
  const int nh = q->nmu * q->nchi;
  const int first = (o && o->ray_count > 0) ? o->ray_first : 0;
  const int last = (o && o->ray_count > 0) ? o->ray_first + o->ray_count : 2 * nh;
  lo = std::max(first, hemi * nh) - hemi * nh;
  hi = std::min(last, (hemi + 1) * nh) - hemi * nh;
  if (hi < lo) hi = lo;
}

// Rays swept together: the options' batch, at most the call's rays in one hemisphere.
int ray_batch(const porta_quad* q, const porta_options* o) {
  const int nh = q->nmu * q->nchi;
  int rb = (o && o->ray_batch > 0) ? o->ray_batch : nh, cap = 1;
  for (int hemi = 0; hemi < 2; ++hemi) {
    int lo, hi;
    hemi_range(q, o, hemi, lo, hi);
    cap = std::max(cap, hi - lo);
  }
  return std::min(rb, cap);
}

// ---------------------------------------------------------------------------
// Workspace layout (every region 256-byte aligned)
// ---------------------------------------------------------------------------
struct Layout {
  size_t stage;     // doubles: mu[kMaxMu], wmu[kMaxMu], phi[nfreq], wfreq[nfreq]
  size_t rays;      // RayConsts[nrays]
  size_t phiT;      // T[nfreq]
  size_t wn;        // double[nfreq]
  size_t flag;      // int: result of the optional input check
  size_t end_tables;
  size_t stateA, stateB;   // sweep plane states
  size_t jpart;
  // adjoint: checkpoints, recompute slots, Lambda ping-pong, per-ray partials, gradient
  size_t ck, slots, lamA, lamB, go, gm, gp, grad;
  size_t tf;               // first-face sweep: transposed transfer coefficients
  size_t fcache;           // first-face sweep: set-up of the nodes of a plane
  size_t plane;            // bytes of one plane state of a ray batch
  int nck, nslot;
  size_t total;
};

Layout tables_layout(const porta_quad* q, int prec) {
  Layout L{};
  size_t off = 0;
  L.stage = off;
  off = align_up(off + sizeof(double) * (2 * kMaxMu + 2 * (size_t)q->nfreq));
  L.rays = off;
  off = align_up(off + sizeof(RayConsts) * 2 * (size_t)q->nmu * q->nchi);
  L.phiT = off;
  off = align_up(off + elem(prec) * q->nfreq);
  L.wn = off;
  off = align_up(off + sizeof(double) * q->nfreq);
  L.flag = off;
  off = align_up(off + sizeof(int));
  L.end_tables = off;
  L.total = off;
  return L;
}

Layout sweep_layout(const porta_grid* g, const porta_quad* q, int prec, const porta_options* o) {
  Layout L = tables_layout(q, prec);
  const size_t np = (size_t)g->nx * g->ny;
  const size_t nrb = (size_t)ray_batch(q, o);
  const size_t state = nrb * q->nfreq * np * nstokes(o) * elem(prec);
  size_t off = L.end_tables;
  L.stateA = off;
  off = align_up(off + state);
  L.stateB = off;
  off = align_up(off + state);
  L.jpart = off;
  off = align_up(off + 2 * nrb * 5 * np * sizeof(double));   // double-buffered partial sums
  if (faces_of(o)) {
    // per-chunk partial sums of the first-face kernel
    int lanes, fchunk;
    faces_shape(g, q, prec, o, lanes, fchunk);
    const size_t nchunk = fchunk > 0 ? (q->nfreq + fchunk - 1) / fchunk : 1;
    L.ck = off;
    off = align_up(off + nrb * nchunk * 5 * np * sizeof(double));
    // the transfer coefficients with x and y exchanged in every plane
    L.tf = off;
    off = align_up(off + 13 * np * g->nz * elem(prec));
    // the set-up of every node and ray of one plane
    L.fcache = off;
    off = align_up(off + nrb * kFacesCache * np * elem(prec));
  }
  L.total = off;
  return L;
}

// Checkpoint planes are k = C, 2C, ... <= nz - 2 (the top plane is recomputed).
int checkpoint_count(int nz, int C) { return nz >= 3 ? (nz - 2) / C : 0; }
bool is_checkpoint(int k, int nz, int C) { return k >= 1 && k % C == 0 && k <= nz - 2; }

// Adjoint: checkpoint planes (unless the caller brings them), C slots for the
// planes recomputed between two checkpoints, two planes of Lambda, the
// per-(node, ray) partials of one plane and the FP64 gradient accumulator.
Layout adjoint_layout(const porta_grid* g, const porta_quad* q, int prec, int stride,
                      const porta_options* o, bool own_checkpoints) {
  Layout L = tables_layout(q, prec);
  const size_t np = (size_t)g->nx * g->ny, N = np * g->nz;
  const size_t nrb = (size_t)ray_batch(q, o);
  L.plane = nrb * q->nfreq * np * 4 * elem(prec);
  L.nck = own_checkpoints ? checkpoint_count(g->nz, stride) : 0;
  L.nslot = stride;
  size_t off = L.end_tables;
  L.ck = off;
  off = align_up(off + (size_t)L.nck * L.plane);
  L.slots = off;
  off = align_up(off + (size_t)L.nslot * L.plane);
  L.lamA = off;
  off = align_up(off + L.plane);
  L.lamB = off;
  off = align_up(off + L.plane);
  // per-(node, ray) partials in the sweep precision
  L.go = off;
  off = align_up(off + nrb * 13 * np * elem(prec));
  L.gm = off;
  off = align_up(off + nrb * 13 * np * elem(prec));
  L.gp = off;
  off = align_up(off + nrb * 7 * np * elem(prec));
  L.grad = off;
  off = align_up(off + 13 * N * sizeof(double));
  L.total = off;
  return L;
}

// Checkpoints hold the upward rays of the call's ray range:
// [(nz-2)/C][upward rays of the range][nfreq][ny][nx][4].
size_t checkpoint_bytes(const porta_grid* g, const porta_quad* q, int prec, int stride,
                        const porta_options* o) {
  int lo, hi;
  hemi_range(q, o, 0, lo, hi);
  return (size_t)checkpoint_count(g->nz, stride) * (hi - lo) * q->nfreq *
         ((size_t)g->nx * g->ny) * 4 * elem(prec);
}

// Upload host doubles through kernel arguments (ordered on the stream).
int upload(double* dst, const double* src, size_t n, hipStream_t st) {
  for (size_t o = 0; o < n; o += kUploadChunk) {
    UploadChunk c;
    c.n = (int)std::min<size_t>(kUploadChunk, n - o);
    std::memcpy(c.v, src + o, sizeof(double) * c.n);
    c.dst = dst + o;
    hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, st, c);
  }
  return check_launch("upload");
}

template <class T>
int prepare_tables(char* ws, const Layout& L, const porta_quad* q, double w2, hipStream_t st) {
  double* stage = reinterpret_cast<double*>(ws + L.stage);
  int rc;
  if ((rc = upload(stage, q->mu, q->nmu, st))) return rc;
  if ((rc = upload(stage + kMaxMu, q->wmu, q->nmu, st))) return rc;
  if ((rc = upload(stage + 2 * kMaxMu, q->phi, q->nfreq, st))) return rc;
  if ((rc = upload(stage + 2 * kMaxMu + q->nfreq, q->wfreq, q->nfreq, st))) return rc;
  hipLaunchKernelGGL(k_prepare<T>, dim3(1), dim3(256), 0, st, stage, stage + kMaxMu, q->nmu,
                     q->nchi, w2, stage + 2 * kMaxMu, stage + 2 * kMaxMu + q->nfreq, q->nfreq,
                     reinterpret_cast<RayConsts*>(ws + L.rays), reinterpret_cast<T*>(ws + L.phiT),
                     reinterpret_cast<double*>(ws + L.wn));
  return check_launch("prepare");
}

int fill(double* p, size_t n, double v, hipStream_t st) {
  if (n == 0) return PORTA_OK;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return check_launch("fill");
}

// The opt-in input check: one pass over the fields, then a wait on the stream for
// its verdict.
template <class T>
int check_inputs(const porta_grid* g, const porta_fields* f, char* ws, const Layout& L,
                 hipStream_t st) {
  const size_t N = (size_t)g->nx * g->ny * g->nz;
  int* flag = reinterpret_cast<int*>(ws + L.flag);
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(64), 0, st, flag);
  int rc;
  if ((rc = check_launch("zero_flag"))) return rc;
  const size_t blocks = std::min<size_t>((N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_check_fields<T>, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<const T*>(f->kappa), static_cast<const T*>(f->propmat),
                     static_cast<const T*>(f->emis), N, flag);
  if ((rc = check_launch("check_fields"))) return rc;
  int h = 0;
  if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(PORTA_EDEVICE, "reading the input check failed");
  if (h) return fail(PORTA_ENONFINITE, "a transfer coefficient is not finite, or eta_I <= 0");
  return PORTA_OK;
}

// ---------------------------------------------------------------------------
// Forward sweep with M and P on the first face crossed (options.faces = 1)
// ---------------------------------------------------------------------------
template <class T>
int sweep_faces_impl(const porta_grid* g, const porta_quad* q, const porta_fields* f,
                     const porta_options* o, double* jkq, T* itop, char* ws, const Layout& L,
                     const RayConsts* rays, const T* phiT, const double* wn, T* state[2],
                     hipStream_t st) {
  int rc;
  const int nx = g->nx, ny = g->ny, nz = g->nz, np = nx * ny;
  const size_t N = (size_t)np * nz;
  const int nh = q->nmu * q->nchi;
  const int nrb_max = ray_batch(q, o);
  int lanes, fchunk;
  faces_shape(g, q, sizeof(T) == 4 ? PORTA_F32 : PORTA_F64, o, lanes, fchunk);
  const int nchunk = (q->nfreq + fchunk - 1) / fchunk;
  double* jpart = reinterpret_cast<double*>(ws + L.jpart);
  double* jchunk = reinterpret_cast<double*>(ws + L.ck);
  const size_t lds = faces_lds_bytes<T>(q->nfreq, fchunk, lanes);
  const dim3 rblk(256), rgrid((np + 255) / 256);
  // rays that meet an x face first read the fields with x and y exchanged
  T* tf = reinterpret_cast<T*>(ws + L.tf);
  {
    const T* src[3] = {static_cast<const T*>(f->kappa), static_cast<const T*>(f->propmat),
                       static_cast<const T*>(f->emis)};
    const size_t nfield[3] = {1, 6, 6}, dst[3] = {0, N, 7 * N};
    for (int c = 0; c < 3; ++c) {
      const size_t n = nfield[c] * N;
      hipLaunchKernelGGL(k_transpose_planes<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                         st, src[c], tf + dst[c], nx, ny, nfield[c] * nz);
      if ((rc = check_launch("transpose_planes"))) return rc;
    }
  }
  for (int hemi = 0; hemi < 2; ++hemi) {
    const bool up = (hemi == 0);
    const int kb = up ? 0 : nz - 1, s = up ? 1 : -1;
    const T ibound = up ? (T)f->i_bottom : T(0);
    int lo, hi;
    hemi_range(q, o, hemi, lo, hi);
    for (int r0 = lo; r0 < hi; r0 += nrb_max) {
      const int nrb = std::min(nrb_max, hi - r0);
      const int ray0 = hemi * nh + r0;
      if (jkq) {
        // the boundary plane
        hipLaunchKernelGGL(k_jreduce, rgrid, rblk, 0, st, jkq, (const double*)nullptr, rays,
                           ray0, nrb, np, N, (size_t)kb * np, 1, (double)ibound);
        if ((rc = check_launch("jreduce (boundary)"))) return rc;
      }
      const T* prev = nullptr;
      for (int step = 1; step < nz; ++step) {
        const int k = kb + s * step;
        const bool last = (step == nz - 1);
        FacesArgs<T> a;
        a.kappa = static_cast<const T*>(f->kappa);
        a.prop = static_cast<const T*>(f->propmat);
        a.emis = static_cast<const T*>(f->emis);
        a.kappa_t = tf;
        a.prop_t = tf + N;
        a.emis_t = tf + 7 * N;
        a.rays = rays;
        a.phi = phiT;
        a.wn = wn;
        a.iprev = prev;
        a.top = last && up && itop;
        a.inext = a.top ? itop + (size_t)r0 * q->nfreq * np * 4 : state[step & 1];
        a.jchunk = jkq ? jchunk : nullptr;
        a.N = N;
        a.nx = nx;
        a.ny = ny;
        a.np = np;
        a.nfreq = q->nfreq;
        a.fchunk = fchunk;
        a.nchunk = nchunk;
        a.kO = k;
        a.kM = k - s;
        a.kP = last ? -1 : k + s;
        a.dzM = std::fabs(g->z[k] - g->z[k - s]);
        a.dzP = last ? 0.0 : std::fabs(g->z[k + s] - g->z[k]);
        a.inv_dx = nx / g->lx;
        a.inv_dy = ny / g->ly;
        a.ray0 = ray0;
        a.parabolic = parabolic_of(o);
        a.tol = sizeof(T) == 4 ? 0x1p-24 : 0x1p-53;   // the unit roundoff of the sweep precision
        a.ibound = ibound;
        a.cache = reinterpret_cast<T*>(ws + L.fcache);
        a.nrb = nrb;
        hipLaunchKernelGGL(k_faces_setup<T>, dim3((np + 255) / 256, nrb), dim3(256), 0, st, a);
        if ((rc = check_launch("faces_setup"))) return rc;
        hipLaunchKernelGGL(k_sweep_plane_faces<T>, dim3(faces_grid(nrb, nchunk)), dim3(lanes),
                           lds, st, a);
        if ((rc = check_launch("sweep_plane_faces"))) return rc;
        if (jkq) {
          const unsigned tiles = (unsigned)((std::max(nx, ny) + kSumTile - 1) / kSumTile);
          hipLaunchKernelGGL(k_sum_chunks, dim3(tiles, tiles, nrb), dim3(256), 0, st, jpart,
                             (const double*)jchunk, rays, ray0, nchunk, nx, ny, nx / g->lx,
                             ny / g->ly);
          if ((rc = check_launch("sum_chunks"))) return rc;
          hipLaunchKernelGGL(k_jreduce, rgrid, rblk, 0, st, jkq, (const double*)jpart, rays,
                             ray0, nrb, np, N, (size_t)k * np, 0, 0.0);
          if ((rc = check_launch("jreduce"))) return rc;
        }
        prev = a.inext;
      }
    }
  }
  return PORTA_OK;
}

// ---------------------------------------------------------------------------
// Forward sweep
// ---------------------------------------------------------------------------
template <class T>
int sweep_impl(const porta_grid* g, const porta_quad* q, const porta_fields* f, int interp,
               const porta_options* o, double* jkq, int accumulate, T* itop, T* ckpt, int C,
               char* ws, const Layout& L, hipStream_t st) {
  int rc;
  if ((rc = prepare_tables<T>(ws, L, q, f->w2, st))) return rc;
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  const int np = nx * ny;
  const size_t N = (size_t)np * nz;
  if (jkq && !accumulate)
    if ((rc = fill(jkq, 10 * N, 0.0, st))) return rc;
  const int nh = q->nmu * q->nchi;
  const int nrb_max = ray_batch(q, o);
  const int ns = nstokes(o);
  const int block = (o && o->block > 0) ? o->block : 256;
  if (block % 64 != 0 || block > 256) return fail(PORTA_EINVAL, "block must be 64, 128, 192 or 256");
  const RayConsts* rays = reinterpret_cast<const RayConsts*>(ws + L.rays);
  const T* phiT = reinterpret_cast<const T*>(ws + L.phiT);
  const double* wn = reinterpret_cast<const double*>(ws + L.wn);
  T* state[2] = {reinterpret_cast<T*>(ws + L.stateA), reinterpret_cast<T*>(ws + L.stateB)};
  if (faces_of(o))
    return sweep_faces_impl<T>(g, q, f, o, jkq, itop, ws, L, rays, phiT, wn, state, st);
  double* jpart[2] = {nullptr, nullptr};
  if (jkq) {
    jpart[0] = reinterpret_cast<double*>(ws + L.jpart);
    jpart[1] = jpart[0] + (size_t)nrb_max * 5 * np;
  }
  const dim3 rblk(256), rgrid((np + 255) / 256);

  for (int hemi = 0; hemi < 2; ++hemi) {
    const bool up = (hemi == 0);
    const int kb = up ? 0 : nz - 1, s = up ? 1 : -1;
    const T ibound = up ? (T)f->i_bottom : T(0);
    int lo, hi, up_lo, up_hi;
    hemi_range(q, o, hemi, lo, hi);
    hemi_range(q, o, 0, up_lo, up_hi);
    for (int r0 = lo; r0 < hi; r0 += nrb_max) {
      const int nrb = std::min(nrb_max, hi - r0);
      const int ray0 = hemi * nh + r0;
      const T* prev = nullptr;
      for (int step = 1; step < nz; ++step) {
        const int k = kb + s * step;
        PlaneArgs<T> a;
        a.kappa = static_cast<const T*>(f->kappa);
        a.prop = static_cast<const T*>(f->propmat);
        a.emis = static_cast<const T*>(f->emis);
        a.rays = rays;
        a.phi = phiT;
        a.wn = wn;
        a.iprev = prev;
        const bool last = (step == nz - 1);
        const size_t batch_off = (size_t)r0 * q->nfreq * np * ns;
        if (last && up && itop)
          a.inext = itop + batch_off;
        else if (up && ckpt && is_checkpoint(k, nz, C))   // kept for the adjoint
          a.inext = ckpt + ((size_t)(k / C - 1) * (up_hi - up_lo) + (r0 - up_lo)) *
                               q->nfreq * np * 4;
        else
          a.inext = state[step & 1];
        // plane k writes partial sums into jpart[step & 1] while the first ray row of
        // blocks adds those of plane k - s (or the boundary plane) to J
        a.jpart = jpart[step & 1];
        a.jkq = jkq;
        a.jpart_prev = (step == 1) ? nullptr : jpart[(step - 1) & 1];
        a.prev_off = (size_t)(k - s) * np;
        a.N = N;
        a.nx = nx;
        a.ny = ny;
        a.np = np;
        a.nfreq = q->nfreq;
        a.kO = k;
        a.kM = k - s;
        a.kP = last ? -1 : k + s;
        a.dzM = std::fabs(g->z[k] - g->z[k - s]);
        a.dzP = last ? 0.0 : std::fabs(g->z[k + s] - g->z[k]);
        a.inv_dx = nx / g->lx;
        a.inv_dy = ny / g->ly;
        a.ray0 = ray0;
        a.xcd_remap = xcd_chunk(o);
        a.parabolic = parabolic_of(o);
        a.ibound = ibound;
        const size_t lds = (size_t)q->nfreq * (sizeof(double) + sizeof(T));
        const dim3 grid((np + block - 1) / block, nrb);
        if (ns == 1)
          hipLaunchKernelGGL(k_sweep_plane_i<T>, grid, dim3(block), lds, st, a);
        else if (interp == PORTA_INTERP_BEZIER2D)
          hipLaunchKernelGGL((k_sweep_plane<T, 1>), grid, dim3(block), lds, st, a);
        else
          hipLaunchKernelGGL((k_sweep_plane<T, 0>), grid, dim3(block), lds, st, a);
        if ((rc = check_launch("sweep_plane"))) return rc;
        prev = a.inext;
      }
      if (jkq) {
        // the last plane of the batch
        const int klast = kb + s * (nz - 1);
        hipLaunchKernelGGL(k_jreduce, rgrid, rblk, 0, st, jkq, (const double*)jpart[(nz - 1) & 1],
                           rays, ray0, nrb, np, N, (size_t)klast * np, 0, 0.0);
        if ((rc = check_launch("jreduce"))) return rc;
      }
    }
  }
  return PORTA_OK;
}

// ---------------------------------------------------------------------------
// Adjoint of the sweep of the upward rays
// ---------------------------------------------------------------------------
template <class T>
int forward_plane(const porta_grid* g, const porta_quad* q, const porta_fields* f,
                  const porta_options* o, int interp, char* ws, const Layout& L, int k,
                  const T* prev, T* next, int ray0, int nrb, int block, hipStream_t st) {
  const int nx = g->nx, ny = g->ny, nz = g->nz, np = nx * ny;
  PlaneArgs<T> a;
  a.kappa = static_cast<const T*>(f->kappa);
  a.prop = static_cast<const T*>(f->propmat);
  a.emis = static_cast<const T*>(f->emis);
  a.rays = reinterpret_cast<const RayConsts*>(ws + L.rays);
  a.phi = reinterpret_cast<const T*>(ws + L.phiT);
  a.wn = reinterpret_cast<const double*>(ws + L.wn);
  a.iprev = prev;
  a.inext = next;
  a.jpart = nullptr;
  a.jkq = nullptr;
  a.jpart_prev = nullptr;
  a.prev_off = 0;
  a.N = (size_t)np * nz;
  a.nx = nx;
  a.ny = ny;
  a.np = np;
  a.nfreq = q->nfreq;
  a.kO = k;
  a.kM = k - 1;
  a.kP = (k == nz - 1) ? -1 : k + 1;
  a.dzM = std::fabs(g->z[k] - g->z[k - 1]);
  a.dzP = (k == nz - 1) ? 0.0 : std::fabs(g->z[k + 1] - g->z[k]);
  a.inv_dx = nx / g->lx;
  a.inv_dy = ny / g->ly;
  a.ray0 = ray0;
  a.xcd_remap = xcd_chunk(o);
  a.parabolic = parabolic_of(o);
  a.ibound = (T)f->i_bottom;
  const size_t lds = (size_t)q->nfreq * (sizeof(double) + sizeof(T));
  if (interp == PORTA_INTERP_BEZIER2D)
    hipLaunchKernelGGL((k_sweep_plane<T, 1>), dim3((np + block - 1) / block, nrb), dim3(block),
                       lds, st, a);
  else
    hipLaunchKernelGGL((k_sweep_plane<T, 0>), dim3((np + block - 1) / block, nrb), dim3(block),
                       lds, st, a);
  return check_launch("sweep_plane (adjoint recompute)");
}

template <class T>
int adjoint_impl(const porta_grid* g, const porta_quad* q, const porta_fields* f,
                 const porta_options* o, int interp, const T* seed, const T* ext_ck, int C, T* gk,
                 T* gpm, T* ge, char* ws, const Layout& L, hipStream_t st) {
  int rc;
  if ((rc = prepare_tables<T>(ws, L, q, f->w2, st))) return rc;
  const int nx = g->nx, ny = g->ny, nz = g->nz, np = nx * ny;
  const size_t N = (size_t)np * nz;
  double* grad = reinterpret_cast<double*>(ws + L.grad);
  if ((rc = fill(grad, 13 * N, 0.0, st))) return rc;
  const int nrb_max = ray_batch(q, o);
  const int block = (o && o->block > 0) ? o->block : 256;
  if (block % 64 != 0 || block > 256) return fail(PORTA_EINVAL, "block must be 64, 128, 192 or 256");
  const size_t pe = L.plane / sizeof(T);   // elements of one plane state
  T* ck = reinterpret_cast<T*>(ws + L.ck);
  T* slots = reinterpret_cast<T*>(ws + L.slots);
  T* lam[2] = {reinterpret_cast<T*>(ws + L.lamA), reinterpret_cast<T*>(ws + L.lamB)};
  // forward state of plane k of the current batch: the boundary (nullptr), a
  // checkpoint (own or the caller's, rays contiguous in both), or a recompute slot
  int r0 = 0, up_lo, up_hi;
  hemi_range(q, o, 0, up_lo, up_hi);
  auto plane = [&](int k) -> T* {
    if (k == 0) return nullptr;
    if (is_checkpoint(k, nz, C)) {
      if (ext_ck)
        return const_cast<T*>(ext_ck) +
               ((size_t)(k / C - 1) * (up_hi - up_lo) + (r0 - up_lo)) * q->nfreq * np * 4;
      return ck + (size_t)(k / C - 1) * pe;
    }
    return slots + (size_t)((k - 1) % C) * pe;
  };
  const size_t lds_adj = (size_t)q->nfreq * sizeof(T);
  for (r0 = up_lo; r0 < up_hi; r0 += nrb_max) {
    const int nrb = std::min(nrb_max, up_hi - r0);
    // forward pass up to the last checkpoint plane, keeping every C-th plane (unless
    // the sweep already kept them); the planes above it are recomputed with the top
    // segment
    if (!ext_ck)
      for (int k = 1; k <= C * checkpoint_count(nz, C); ++k)
        if ((rc = forward_plane<T>(g, q, f, o, interp, ws, L, k, plane(k - 1), plane(k), r0,
                                   nrb, block, st)))
          return rc;
    // reverse pass, one segment between checkpoints at a time
    const T* lam_next = nullptr;
    int cur = 0;
    for (int khi = nz - 1; khi >= 1;) {
      const int s0 = C * ((khi - 1) / C);
      // the adjoint of plane k reads the forward state of plane k-1 only, so the top
      // plane of a segment needs no state
      for (int k = s0 + 1; k < khi; ++k)
        if (!is_checkpoint(k, nz, C))
          if ((rc = forward_plane<T>(g, q, f, o, interp, ws, L, k, plane(k - 1), plane(k), r0,
                                     nrb, block, st)))
            return rc;
      for (int k = khi; k > s0; --k) {
        AdjArgs<T> a;
        a.kappa = static_cast<const T*>(f->kappa);
        a.prop = static_cast<const T*>(f->propmat);
        a.emis = static_cast<const T*>(f->emis);
        a.rays = reinterpret_cast<const RayConsts*>(ws + L.rays);
        a.phi = reinterpret_cast<const T*>(ws + L.phiT);
        a.iprev = plane(k - 1);
        a.lam_next = lam_next;
        a.seed = seed + (size_t)r0 * q->nfreq * np * 4;
        a.lam_cur = (k - 1 >= 1) ? lam[cur] : nullptr;
        a.g_o = reinterpret_cast<T*>(ws + L.go);
        a.g_m = reinterpret_cast<T*>(ws + L.gm);
        a.g_p = reinterpret_cast<T*>(ws + L.gp);
        a.N = N;
        a.nx = nx;
        a.ny = ny;
        a.np = np;
        a.nfreq = q->nfreq;
        a.kO = k;
        a.kM = k - 1;
        a.kP = (k == nz - 1) ? -1 : k + 1;
        a.dzM = std::fabs(g->z[k] - g->z[k - 1]);
        a.dzP = (k == nz - 1) ? 0.0 : std::fabs(g->z[k + 1] - g->z[k]);
        a.dzN = a.dzP;
        a.inv_dx = nx / g->lx;
        a.inv_dy = ny / g->ly;
        a.ray0 = r0;
        a.xcd_remap = xcd_chunk(o);
        a.parabolic = parabolic_of(o);
        a.ibound = (T)f->i_bottom;
        const bool bez = interp == PORTA_INTERP_BEZIER2D;
        if (bez && lam_next) {
          // the adjoint of the Stokes vectors of plane k, gathered through the transposed
          // 9-point stencils of plane k + 1, into the buffer the adjoint of plane k then
          // reads as its seed and overwrites, node by node, with its own output
          TGatherArgs<T> t;
          t.icur = plane(k);
          t.lam_next = lam_next;
          t.out = lam[cur];
          t.rays = a.rays;
          t.nx = nx;
          t.ny = ny;
          t.np = np;
          t.nfreq = q->nfreq;
          t.dzN = a.dzN;
          t.inv_dx = a.inv_dx;
          t.inv_dy = a.inv_dy;
          t.ray0 = r0;
          constexpr int TX = TGTile<T>::X, TY = TGTile<T>::Y;
          hipLaunchKernelGGL(k_bez9_tgather<T>,
                             dim3((nx + TX - 1) / TX, (ny + TY - 1) / TY, nrb), dim3(TX * TY),
                             0, st, t);
          if ((rc = check_launch("bez9_tgather"))) return rc;
          a.lam_next = nullptr;
          a.seed = lam[cur];
          a.lam_cur = (k - 1 >= 1) ? lam[cur] : nullptr;
        }
        if (bez)
          hipLaunchKernelGGL((k_adjoint_plane<T, 1>), dim3((np + block - 1) / block, nrb),
                             dim3(block), lds_adj, st, a);
        else
          hipLaunchKernelGGL((k_adjoint_plane<T, 0>), dim3((np + block - 1) / block, nrb),
                             dim3(block), lds_adj, st, a);
        if ((rc = check_launch("adjoint_plane"))) return rc;
        GatherArgs<T> b;
        b.g_o = a.g_o;
        b.g_m = a.g_m;
        b.g_p = a.g_p;
        b.kappa = a.kappa;
        b.prop = a.prop;
        b.emis = a.emis;
        b.rays = a.rays;
        b.grad = grad;
        b.N = N;
        b.nx = nx;
        b.ny = ny;
        b.np = np;
        b.kO = a.kO;
        b.kM = a.kM;
        b.kP = a.kP;
        b.dzM = a.dzM;
        b.dzP = a.dzP;
        b.inv_dx = a.inv_dx;
        b.inv_dy = a.inv_dy;
        b.ray0 = r0;
        b.nrb = nrb;
        if (bez)
          hipLaunchKernelGGL((k_adjoint_gather<T, 1>), dim3((np + 255) / 256, 4), dim3(256), 0, st,
                             b);
        else
          hipLaunchKernelGGL((k_adjoint_gather<T, 0>), dim3((np + 255) / 256, 4), dim3(256), 0, st,
                             b);
        if ((rc = check_launch("adjoint_gather"))) return rc;
        lam_next = a.lam_cur;
        cur ^= 1;
      }
      khi = s0;
    }
  }
  const size_t blocks = std::min<size_t>((N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_grad_out<T>, dim3((unsigned)blocks), dim3(256), 0, st, grad, N, gk, gpm, ge);
  return check_launch("grad_out");
}


// ---------------------------------------------------------------------------
// Static scratch of porta_fs_sweep_noalloc: one array per device, the workspace of
// that entry point.  Host code never uses the symbol itself as an address: the
// device address is looked up once per device (with that device current) and kept.
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0)
    return fail(PORTA_EDEVICE, "no current HIP device");
  if (dev >= kMaxDevices) return fail(PORTA_EUNSUPPORTED, "device index %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PORTA_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PORTA_OK;
}

// Validation and launch of a forward sweep.  With use_scratch the workspace is this
// device's static scratch array instead of the caller's buffer.
int sweep_entry(const porta_grid* grid, const porta_quad* quad, const porta_fields* fields,
                int prec, int interp, const porta_options* opts, double* jkq, int accumulate,
                void* i_top, void* checkpoints, size_t ck_bytes, int checkpoint_stride,
                void* workspace, size_t ws_bytes, bool use_scratch, void* stream) {
  int rc;
  if ((rc = validate_grid(grid)) || (rc = validate_quad(quad)) || (rc = validate_prec(prec)) ||
      (rc = validate_interp(interp)))
    return rc;
  if (!fields || !fields->kappa || !fields->propmat || !fields->emis)
    return fail(PORTA_EINVAL, "fields and their arrays must not be NULL");
  if (!std::isfinite(fields->i_bottom) || !std::isfinite(fields->w2))
    return fail(PORTA_EINVAL, "i_bottom and w2 must be finite");
  if ((rc = validate_options(opts)) || (rc = validate_rays(quad, opts))) return rc;
  if (nstokes(opts) == 1 && interp != PORTA_INTERP_BILINEAR)
    return fail(PORTA_EUNSUPPORTED, "the intensity-only sweep interpolates bilinearly only");
  if (nstokes(opts) == 1 && checkpoints)
    return fail(PORTA_EUNSUPPORTED, "checkpoints are for the Stokes-vector sweep");
  if (faces_of(opts)) {
    if (nstokes(opts) == 1 || interp != PORTA_INTERP_BILINEAR || checkpoints)
      return fail(PORTA_EUNSUPPORTED,
                  "faces = 1 is for the bilinear Stokes-vector sweep without checkpoints");
    if (std::max(grid->nx, grid->ny) > kFacesMaxLanes)
      return fail(PORTA_EUNSUPPORTED, "faces = 1 needs nx, ny <= %d", kFacesMaxLanes);
    int lanes, fchunk;
    faces_shape(grid, quad, prec, opts, lanes, fchunk);
    if (fchunk < 1)
      return fail(PORTA_EUNSUPPORTED, "faces = 1: the LDS of a block has no room for %s",
                  opts->faces_chunk > 0 ? "faces_chunk frequencies" : "one frequency");
  }
  if (checkpoints && (checkpoint_stride < 1 || checkpoint_stride > grid->nz - 1))
    return fail(PORTA_EINVAL, "checkpoint_stride must be in 1..nz-1");
  if (checkpoints) {
    const size_t need = checkpoint_bytes(grid, quad, prec, checkpoint_stride, opts);
    if (ck_bytes < need)
      return fail(PORTA_ENOMEM, "checkpoint buffer of %zu bytes is smaller than the %zu required",
                  ck_bytes, need);
  }
  if (!use_scratch && !workspace) return fail(PORTA_EINVAL, "workspace is NULL");
  const Layout L = sweep_layout(grid, quad, prec, opts);
  if (use_scratch) {
    if (L.total > kScratchBytes)
      return fail(PORTA_ENOMEM,
                  "this sweep needs %zu bytes of workspace; the static scratch holds %zu "
                  "(use a smaller opts->ray_batch, or porta_fs_sweep)",
                  L.total, kScratchBytes);
    if ((rc = scratch_address(&workspace))) return rc;
    ws_bytes = kScratchBytes;
  }
  if (ws_bytes < L.total)
    return fail(PORTA_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                L.total);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  if (opts && opts->check_inputs &&
      (rc = (prec == PORTA_F64) ? check_inputs<double>(grid, fields, ws, L, st)
                                : check_inputs<float>(grid, fields, ws, L, st)))
    return rc;
  if (prec == PORTA_F64)
    return sweep_impl<double>(grid, quad, fields, interp, opts, jkq, accumulate,
                              static_cast<double*>(i_top), static_cast<double*>(checkpoints),
                              checkpoint_stride, ws, L, st);
  return sweep_impl<float>(grid, quad, fields, interp, opts, jkq, accumulate,
                           static_cast<float*>(i_top),
                           static_cast<float*>(checkpoints), checkpoint_stride, ws, L, st);
}

}  // namespace

extern "C" {

const char* porta_version(void) { return "porta-mi355x 0.1.0 (gfx950)"; }

const char* porta_last_error(void) { return g_last_error.c_str(); }

const char* porta_strerror(int status) {
  switch (status) {
    case PORTA_OK: return "success";
    case PORTA_EINVAL: return "invalid argument";
    case PORTA_EUNSUPPORTED: return "unsupported combination of arguments";
    case PORTA_ENOMEM: return "workspace too small";
    case PORTA_EDEVICE: return "HIP device error";
    case PORTA_ENONFINITE: return "non-finite transfer coefficient or eta_I <= 0";
    default: return "unknown status";
  }
}

size_t porta_workspace_size(const porta_grid* grid, const porta_quad* quad, int prec, int kind,
                            int checkpoint_stride, const porta_options* opts) {
  if (validate_prec(prec)) return 0;
  switch (kind) {
    case PORTA_WS_SWEEP:
      if (validate_grid(grid) || validate_quad(quad)) return 0;
      return sweep_layout(grid, quad, prec, opts).total;
    case PORTA_WS_ADJOINT:
    case PORTA_WS_ADJOINT_CKPT:
      if (validate_grid(grid) || validate_quad(quad) || checkpoint_stride < 1 ||
          checkpoint_stride > grid->nz - 1)
        return 0;
      return adjoint_layout(grid, quad, prec, checkpoint_stride, opts, kind == PORTA_WS_ADJOINT)
          .total;
    case PORTA_WS_JKQ:
      if (validate_quad(quad)) return 0;
      return tables_layout(quad, prec).total;
    case PORTA_WS_SEE: {
      if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return 0;
      const size_t n = (size_t)grid->nx * grid->ny * grid->nz;
      return align_up(sizeof(double) * ((n + 255) / 256));
    }
    default:
      fail(PORTA_EINVAL, "unknown workspace kind %d", kind);
      return 0;
  }
}

size_t porta_checkpoint_size(const porta_grid* grid, const porta_quad* quad, int prec,
                             int checkpoint_stride, const porta_options* opts) {
  if (validate_prec(prec) || validate_grid(grid) || validate_quad(quad) ||
      validate_options(opts) || validate_rays(quad, opts))
    return 0;
  if (checkpoint_stride < 1 || checkpoint_stride > grid->nz - 1) {
    fail(PORTA_EINVAL, "checkpoint_stride must be in 1..nz-1");
    return 0;
  }
  return checkpoint_bytes(grid, quad, prec, checkpoint_stride, opts);
}

int porta_fs_sweep(const porta_grid* grid, const porta_quad* quad, const porta_fields* fields,
                   int prec, int interp, const porta_options* opts, double* jkq, int accumulate,
                   void* i_top, void* checkpoints, size_t ck_bytes, int checkpoint_stride,
                   void* workspace, size_t ws_bytes, void* stream) {
  return sweep_entry(grid, quad, fields, prec, interp, opts, jkq, accumulate, i_top, checkpoints,
                     ck_bytes, checkpoint_stride, workspace, ws_bytes, false, stream);
}

int porta_fs_sweep_noalloc(const porta_grid* grid, const porta_quad* quad,
                           const porta_fields* fields, int prec, int interp,
                           const porta_options* opts, double* jkq, int accumulate, void* i_top,
                           void* stream) {
  return sweep_entry(grid, quad, fields, prec, interp, opts, jkq, accumulate, i_top, nullptr, 0,
                     0, nullptr, 0, true, stream);
}

int porta_jkq_accumulate(const porta_grid* grid, const porta_quad* quad, int ray0, int nray,
                         int f0, int nf, const void* stokes, const void* lambda_star, int prec,
                         double* jkq, void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = validate_grid(grid)) || (rc = validate_quad(quad)) || (rc = validate_prec(prec)))
    return rc;
  const int nrays = 2 * quad->nmu * quad->nchi;
  if (ray0 < 0 || nray < 0 || ray0 + nray > nrays)
    return fail(PORTA_EINVAL, "ray range [%d, %d) outside [0, %d)", ray0, ray0 + nray, nrays);
  if (f0 < 0 || nf < 0 || f0 + nf > quad->nfreq)
    return fail(PORTA_EINVAL, "frequency range [%d, %d) outside [0, %d)", f0, f0 + nf,
                quad->nfreq);
  if (!stokes || !jkq) return fail(PORTA_EINVAL, "stokes and jkq must not be NULL");
  if (!workspace) return fail(PORTA_EINVAL, "workspace is NULL");
  const Layout L = tables_layout(quad, prec);
  if (ws_bytes < L.total)
    return fail(PORTA_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                L.total);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  const size_t N = (size_t)grid->nx * grid->ny * grid->nz;
  if (nray == 0 || nf == 0) return PORTA_OK;
  const dim3 grd((unsigned)((N + 255) / 256)), blk(256);
  if (prec == PORTA_F64) {
    if ((rc = prepare_tables<double>(ws, L, quad, 1.0, st))) return rc;
    hipLaunchKernelGGL(k_jkq_accumulate<double>, grd, blk, 0, st, jkq,
                       static_cast<const double*>(stokes), static_cast<const double*>(lambda_star),
                       reinterpret_cast<const RayConsts*>(ws + L.rays),
                       reinterpret_cast<const double*>(ws + L.wn), ray0, nray, f0, nf, N);
  } else {
    if ((rc = prepare_tables<float>(ws, L, quad, 1.0, st))) return rc;
    hipLaunchKernelGGL(k_jkq_accumulate<float>, grd, blk, 0, st, jkq,
                       static_cast<const float*>(stokes), static_cast<const float*>(lambda_star),
                       reinterpret_cast<const RayConsts*>(ws + L.rays),
                       reinterpret_cast<const double*>(ws + L.wn), ray0, nray, f0, nf, N);
  }
  return check_launch("jkq_accumulate");
}

int porta_fs_adjoint(const porta_grid* grid, const porta_quad* quad, const porta_fields* fields,
                     int prec, int interp, const porta_options* opts, const void* dl_ditop,
                     const void* checkpoints, size_t ck_bytes, int checkpoint_stride,
                     void* g_kappa, void* g_propmat, void* g_emis, void* workspace,
                     size_t ws_bytes, void* stream) {
  int rc;
  if ((rc = validate_grid(grid)) || (rc = validate_quad(quad)) || (rc = validate_prec(prec)) ||
      (rc = validate_interp(interp)))
    return rc;
  if (!fields || !fields->kappa || !fields->propmat || !fields->emis)
    return fail(PORTA_EINVAL, "fields and their arrays must not be NULL");
  if (!dl_ditop || !g_kappa || !g_propmat || !g_emis)
    return fail(PORTA_EINVAL, "seed and gradient arrays must not be NULL");
  if (checkpoint_stride < 1 || checkpoint_stride > grid->nz - 1)
    return fail(PORTA_EINVAL, "checkpoint_stride must be in 1..nz-1");
  if ((rc = validate_options(opts)) || (rc = validate_rays(quad, opts))) return rc;
  if (nstokes(opts) == 1)
    return fail(PORTA_EUNSUPPORTED, "the adjoint is for the Stokes-vector sweep");
  if (faces_of(opts))
    return fail(PORTA_EUNSUPPORTED, "the adjoint differentiates the plane-hop sweep (faces = 0)");
  if (checkpoints) {
    const size_t need = checkpoint_bytes(grid, quad, prec, checkpoint_stride, opts);
    if (ck_bytes < need)
      return fail(PORTA_ENOMEM, "checkpoint buffer of %zu bytes is smaller than the %zu required",
                  ck_bytes, need);
  }
  if (!workspace) return fail(PORTA_EINVAL, "workspace is NULL");
  const Layout L = adjoint_layout(grid, quad, prec, checkpoint_stride, opts, !checkpoints);
  if (ws_bytes < L.total)
    return fail(PORTA_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                L.total);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  if (opts && opts->check_inputs &&
      (rc = (prec == PORTA_F64) ? check_inputs<double>(grid, fields, ws, L, st)
                                : check_inputs<float>(grid, fields, ws, L, st)))
    return rc;
  if (prec == PORTA_F64)
    return adjoint_impl<double>(grid, quad, fields, opts, interp,
                                static_cast<const double*>(dl_ditop),
                                static_cast<const double*>(checkpoints), checkpoint_stride,
                                static_cast<double*>(g_kappa), static_cast<double*>(g_propmat),
                                static_cast<double*>(g_emis), ws, L, st);
  return adjoint_impl<float>(grid, quad, fields, opts, interp,
                             static_cast<const float*>(dl_ditop),
                             static_cast<const float*>(checkpoints), checkpoint_stride,
                             static_cast<float*>(g_kappa), static_cast<float*>(g_propmat),
                             static_cast<float*>(g_emis), ws, L, st);
}

}  // extern "C"
