/*
 * porta.h -- C ABI of the MI355X (gfx950) implementation of the PORTA hot
 * path: the short-characteristics BESSER formal solver of the Stokes-vector
 * transfer equation on a horizontally periodic 3-D grid, the angle and
 * frequency integration of the radiation-field tensors J^K_Q, the Jacobi
 * update of the two-level (J_l = 0 -> J_u = 1) statistical equilibrium with
 * Hanle rotation, and the reverse-mode adjoint of the sweep.
 *
 * Reference: J. Stepan and J. Trujillo Bueno, "PORTA: A three-dimensional
 * multilevel radiative transfer code for modeling the intensity and
 * polarization of spectral lines with massively parallel computers",
 * A&A (2013), arXiv:1307.4217.  Sections, equations and tables cited below
 * are those of that paper.
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Points are stored x fastest: p = (k * ny + j) * nx + i, N = nx*ny*nz.
 *    x and y are periodic with spacing lx/nx and ly/ny; z is given per plane.
 *  - Rays: r in [0, nmu*nchi) propagate upward (mu > 0), r in
 *    [nmu*nchi, 2*nmu*nchi) downward; inside a hemisphere the inclination
 *    index a is slow and the azimuth index m fast.  The ray direction is
 *    (sin t cos chi, sin t sin chi, +-mu[a]) with chi = (m + 1/2) 2 pi / nchi
 *    (trapezoid rule, Appendix A) and weight wmu[a] / (2 nchi); the weights
 *    of all rays sum to one.
 *  - Frequencies: every absorption and emission coefficient is its
 *    line-centre value times phi[j] (complete redistribution, one line
 *    profile).  The frequency weights of Eq. 1 are renormalized (Sect. 4.2) on the
 *    discrete grid: W_j = wfreq[j] phi[j] / sum_j' wfreq[j'] phi[j'].
 *  - Multipole components are stored in the order
 *    (X00, X20, Re X21, Im X21, Re X22, Im X22); the Q < 0 components follow
 *    from X^K_-Q = (-1)^Q conj(X^K_Q).
 *  - J output [10][N] (FP64): J00, J10, Re J11, Im J11, J20, Re J21, Im J21,
 *    Re J22, Im J22, and the Lambda* average
 *    Lbar = sum_rays w sum_j W_j Lambda*_{ray,j} (Sect. 3.3, Eq. 14).
 *  - Pointers named "host" are read during the call only.  Every other data
 *    pointer is device memory owned by the caller; the library never keeps
 *    or frees it.  Work is enqueued on `stream` (a hipStream_t, NULL for the
 *    default stream) and returns before it completes; the caller
 *    synchronizes before reading results.  The library keeps no state
 *    between calls; calls on different streams must not share a workspace.
 *  - Inputs are validated on the host before anything is enqueued; a
 *    failure returns a negative porta_status, enqueues nothing and records a
 *    message for porta_last_error() (thread-local).  HIP launch failures
 *    return PORTA_EDEVICE.
 *  - Physical preconditions that are not checked: kappa > 0 everywhere and
 *    all inputs finite.  Violations give undefined numbers, never a fault.
 */
#ifndef PORTA_H
#define PORTA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PORTA_OK = 0,
  PORTA_EINVAL = -1,       /* invalid argument (shape, pointer, range) */
  PORTA_EUNSUPPORTED = -2, /* valid but not implemented combination */
  PORTA_ENOMEM = -3,       /* workspace smaller than porta_workspace_size() */
  PORTA_EDEVICE = -4,      /* a HIP call failed */
  PORTA_ENONFINITE = -5    /* opts->check_inputs: a transfer coefficient is not finite,
                              or eta_I <= 0 somewhere */
} porta_status;

typedef enum { PORTA_F64 = 0, PORTA_F32 = 1 } porta_prec;   /* sweep precision */

typedef enum {
  PORTA_INTERP_BILINEAR = 0, /* 4-point bilinear at M and P (Sect. 3.1) */
  PORTA_INTERP_BEZIER2D = 1  /* 9-point stencil around the nearest node; monotonic
                                quadratic Bezier (BESSER control points, Sect. 3.2)
                                along x for each row, then along y.  Forward sweep
                                only: porta_fs_adjoint returns PORTA_EUNSUPPORTED */
} porta_interp;

typedef enum {
  PORTA_WS_SWEEP = 0,   /* porta_fs_sweep */
  PORTA_WS_ADJOINT = 1, /* porta_fs_adjoint */
  PORTA_WS_JKQ = 2,     /* porta_jkq_accumulate */
  PORTA_WS_SEE = 3,     /* porta_see_update */
  PORTA_WS_ADJOINT_CKPT = 4 /* porta_fs_adjoint given checkpoints from porta_fs_sweep */
} porta_ws_kind;

/* Spatial grid (Sect. 3.1, Appendix A). */
typedef struct {
  int32_t nx, ny, nz; /* nx, ny >= 1; nz >= 2 */
  double lx, ly;      /* horizontal periods, > 0 */
  const double* z;    /* host, nz plane heights, strictly increasing */
} porta_grid;

/* Angle and frequency quadrature (Eq. 1, Appendix A). */
typedef struct {
  int32_t nmu;         /* inclinations per hemisphere, 1..64 */
  int32_t nchi;        /* azimuths over 2 pi, >= 1 */
  int32_t nfreq;       /* frequencies, 1..4096 */
  const double* mu;    /* host [nmu], each in (0, 1] */
  const double* wmu;   /* host [nmu], >= 0, summing to 1 within 1e-12 */
  const double* phi;   /* host [nfreq], profile relative to line centre, > 0 */
  const double* wfreq; /* host [nfreq], >= 0, with sum wfreq*phi > 0 */
} porta_quad;

/* Transfer coefficients at line centre (Sect. 3, Eq. rte). Element type is
 * double for PORTA_F64 and float for PORTA_F32. */
typedef struct {
  const void* kappa;   /* device [N]: eta_I (> 0) */
  const void* propmat; /* device [6][N]: eta_Q, eta_U, eta_V, rho_Q, rho_U, rho_V;
                          K = [[eI,eQ,eU,eV],[eQ,eI,rV,-rU],[eU,-rV,eI,rQ],[eV,rU,-rQ,eI]] */
  const void* emis;    /* device [6][N]: eps^K_Q multipoles (component order above);
                          eps_i(Omega) = sum_KQ w^K T^K_Q(i, Omega) eps^K_Q, w^0 = 1 */
  double i_bottom;     /* Stokes I entering at z[0] for upward rays (Q=U=V=0);
                          downward rays enter at z[nz-1] with I = 0 */
  double w2;           /* w^(2) of the line (1 for J_l = 0 -> J_u = 1) */
} porta_fields;

/* Two-level atom for the statistical equilibrium (Sect. 2, Eq. nonlte). */
typedef struct {
  double eps_c;        /* collisional destruction probability, in [0, 1] */
  double delta2;       /* depolarizing collision rate delta^(2) (>= 0) */
  double w2;           /* w^(2) of the line */
  double planck;       /* Planck function B */
  const double* hanle; /* device [N] Hanle parameter H_u >= 0, or NULL for no field */
  const double* bhat;  /* device [3][N] unit field direction; NULL for b = z */
} porta_atom;

/* Optional tuning; pass NULL for defaults. */
typedef struct {
  int32_t ray_batch;        /* rays swept together (0: all of the call's rays in a hemisphere) */
  int32_t block;            /* threads per block of the sweep kernel (0: 256) */
  int32_t xcd_remap;        /* R > 0: each XCD takes R consecutive tiles per round;
                               0: hardware order; -1: default (8) */
  int32_t control;          /* control point of the source function along a ray:
                               PORTA_CONTROL_BESSER (Sect. 3.2, default) or
                               PORTA_CONTROL_PARABOLIC (parabola through M, O, P: steps
                               1, 3, 4 only, the DELOPAR choice of Sect. 3) */
  int32_t stokes;           /* 0 or 4: the Stokes vector (default); 1: intensity only,
                               the unpolarized problem (K' = 0, emission eps^0_0; the
                               propagation matrix and the K = 2 emissivities are not
                               read).  With 1, i_top holds one value per node
                               ([nmu*nchi][nfreq][ny][nx]), J^K_Q comes from Stokes I
                               alone, and checkpoints, PORTA_INTERP_BEZIER2D and
                               porta_fs_adjoint return PORTA_EUNSUPPORTED */
  int32_t ray_first;        /* rays of the call: [ray_first, ray_first + ray_count) of the */
  int32_t ray_count;        /* ray enumeration (0 = every ray).  porta_fs_sweep sweeps only
                               them (J with accumulate = 1 then sums the calls),
                               porta_fs_adjoint takes only their upward part; i_top and
                               dl_ditop keep the layout of all upward rays; checkpoints
                               hold only the upward rays of the range */
  int32_t check_inputs;     /* 1: porta_fs_sweep and porta_fs_adjoint first check that every
                               kappa is finite and > 0 and every propmat and emis entry is
                               finite, returning PORTA_ENONFINITE before any other launch
                               if not.  The check reads the fields once and waits on the
                               stream for its result (so it cannot be captured in a HIP
                               graph); 0 (default): no check, no wait */
  int32_t faces;            /* where the points M and P of a short characteristic lie
                               (Sect. 3.1): 0 (default) on the neighbouring horizontal
                               planes, however far the ray travels sideways in between;
                               1 on the first face of the grid the ray crosses, horizontal
                               or vertical, interpolated bilinearly on that face.  A
                               vertical face makes the nodes of a plane depend on each
                               other around the periodic box; each plane is then solved to
                               its fixed point (to the rounding of the sweep precision).
                               With 1: Stokes vector, PORTA_INTERP_BILINEAR, no
                               checkpoints, nx and ny <= 512; porta_fs_adjoint returns
                               PORTA_EUNSUPPORTED */
  int32_t faces_chunk;      /* with faces = 1: frequencies one block of the first-face
                               kernel carries through a plane (0: 4 in FP32, 7 in FP64,
                               fewer where 64 KiB of LDS holds fewer rows of that width,
                               evened out over the chunks); PORTA_EUNSUPPORTED if more
                               than fit */
} porta_options;

typedef enum { PORTA_CONTROL_BESSER = 0, PORTA_CONTROL_PARABOLIC = 1 } porta_control;

/* Bytes of device workspace needed by one call of the given kind (0 on invalid
 * arguments).  `prec` selects the sweep precision; `checkpoint_stride` is
 * used by the two adjoint kinds only. */
size_t porta_workspace_size(const porta_grid* grid, const porta_quad* quad, int prec,
                            int kind, int checkpoint_stride, const porta_options* opts);

/* Bytes of the checkpoint buffer that porta_fs_sweep fills for porta_fs_adjoint:
 * the states of the upward rays of the options' ray range (all by default) on planes
 * C, 2C, ... below the top plane, layout [(nz-2)/C][those rays][nfreq][ny][nx][4] in
 * the sweep precision.  opts may be NULL. */
size_t porta_checkpoint_size(const porta_grid* grid, const porta_quad* quad, int prec,
                             int checkpoint_stride, const porta_options* opts);

/*
 * Formal solution for every ray and frequency (Sect. 3; Eqs. fsint, fsbez,
 * kappa; BESSER control points of Sect. 3.2; Table 1 for small tau_MO),
 * sweeping the planes of each ray in upwind order, fused with the angle and
 * frequency integration of Eq. 1 and of Lambda* (Eq. 14).
 *   prec, interp  : porta_prec, porta_interp
 *   jkq           : device [10][N] FP64, or NULL; overwritten (accumulate = 0)
 *                   or added to (accumulate = 1)
 *   i_top         : device [nmu*nchi][nfreq][ny][nx][4] (sweep precision),
 *                   Stokes vectors of the upward rays at z[nz-1], or NULL
 *                   ([..][nx] without the Stokes axis when opts->stokes == 1)
 *   checkpoints   : device, porta_checkpoint_size() bytes, or NULL; filled with
 *                   the upward rays' states every checkpoint_stride planes for a
 *                   later porta_fs_adjoint of the same fields (no extra traffic:
 *                   those planes are written there instead of the workspace),
 *                   with the same interp (the states of a 9-point sweep are not
 *                   those of a bilinear one: the adjoint cannot tell which mode wrote
 *                   them, so matching them is the caller's to ensure)
 *   checkpoint_bytes : size of that buffer; below porta_checkpoint_size() the
 *                   call returns PORTA_ENOMEM before any launch
 *   workspace     : device, >= porta_workspace_size(..., PORTA_WS_SWEEP, ...)
 */
int porta_fs_sweep(const porta_grid* grid, const porta_quad* quad, const porta_fields* fields,
                   int prec, int interp, const porta_options* opts, double* jkq, int accumulate,
                   void* i_top, void* checkpoints, size_t checkpoint_bytes,
                   int checkpoint_stride, void* workspace, size_t ws_bytes, void* stream);

/*
 * porta_fs_sweep without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  The call allocates nothing: its workspace is a static array of
 * 64 MiB (64 << 20 bytes) in the library's device code, one per device, held until
 * the process ends; its device address is looked up once per device on the first
 * call with that device current.  Arguments are those of porta_fs_sweep with the
 * same meaning, minus the checkpoints and the workspace; the work goes to the
 * current device, to which `stream` must belong.  A problem whose sweep workspace
 * (porta_workspace_size(..., PORTA_WS_SWEEP, ...) with the same options) exceeds
 * 64 MiB returns PORTA_ENOMEM before anything is enqueued; a smaller
 * opts->ray_batch shrinks it.  Nothing in the array needs to start at zero.  Every
 * call on one device shares that device's array: calls whose work overlaps in time
 * on one device (different streams, or different host threads) race and give wrong
 * results; calls ordered on one stream do not.
 */
int porta_fs_sweep_noalloc(const porta_grid* grid, const porta_quad* quad,
                           const porta_fields* fields, int prec, int interp,
                           const porta_options* opts, double* jkq, int accumulate, void* i_top,
                           void* stream);

/*
 * Eq. 1 (and the Lambda* average) from a stored block of Stokes vectors:
 *   stokes      : device [nray][nf][N][4] (sweep precision) for rays
 *                 ray0..ray0+nray-1 and frequencies f0..f0+nf-1
 *   lambda_star : device [nray][nf][N] (sweep precision) or NULL
 *   jkq         : device [10][N] FP64, added to
 */
int porta_jkq_accumulate(const porta_grid* grid, const porta_quad* quad, int ray0, int nray,
                         int f0, int nf, const void* stokes, const void* lambda_star, int prec,
                         double* jkq, void* workspace, size_t ws_bytes, void* stream);

/*
 * One Jacobi update of the two-level statistical equilibrium at every point
 * (Sect. 2 Eq. nonlte; Jacobi iteration of Sect. 5), for L(rho) rho = f with the
 * right-hand side f = rhs, or f = (eps_c B, 0, 0, 0, 0, 0) when rhs is NULL:
 *   S00 <- [(1-eps)(J00 - Lbar S00_old) + f_0] / [1 - (1-eps) Lbar]
 *   [1 + delta (1-eps)] S2_Q + i (1-eps) H_u sum_Q' <Q|b.J|Q'> S2_Q'
 *        = (1-eps) w2 conj(J2_Q) + f2_Q                   (Q = -2..2)
 *   rhs          : device [6][N] FP64 (S00, S20, Re S21, Im S21, Re S22, Im S22 rows
 *                  of f; Q < 0 follows from f_-Q = (-1)^Q conj(f_Q)) or NULL
 *   s_old, s_new : device [6][N] FP64 source-function multipoles S^K_Q
 *   kappa        : device [N] (sweep precision), used for emis_out only
 *   emis_out     : device [6][N] (sweep precision) = kappa * S_new, or NULL
 *   rc_out       : device FP64 scalar, max_p |S00_new - S00_old| / |S00_new|,
 *                  or NULL (the convergence measure R_c of Sect. 5.3)
 *   workspace    : device, >= porta_workspace_size(..., PORTA_WS_SEE, ...) when
 *                  rc_out is given
 */
int porta_see_update(int64_t npoints, const double* jkq, const porta_atom* atom,
                     const double* rhs, const double* s_old, double* s_new, const void* kappa,
                     void* emis_out, int prec, double* rc_out, void* workspace, size_t ws_bytes,
                     void* stream);

/*
 * The statistical-equilibrium operator of the two-level atom applied to its own
 * unknowns, L(rho) rho of Sect. 2 Eq. nonlte (left-hand sides above, with J from
 * the formal solution of these s), combined as
 *   out = base + sign * L(rho) rho,   base = [6][N] FP64 or, if NULL, (eps_c B, 0, ...).
 * sign = -1 gives the residual r = f - L(rho) rho of Sect. 5.1 Eq. resid; sign = +1
 * with base = R(r) gives the coarse-grid right-hand side of Eq. mgcsfy.
 *   jkq : device [10][N] FP64 (Lbar unused); s, out : device [6][N] FP64.
 * out may not alias s or jkq; it may alias base.
 */
int porta_see_operator(int64_t npoints, const double* jkq, const porta_atom* atom,
                       const double* s, const double* base, double sign, double* out,
                       void* stream);

/*
 * Grid transfer of the multigrid iteration (Sect. 5.1-5.2).  The coarser grid keeps
 * every second node along each axis: coarse node (i, j, k) is fine node (2i, 2j, 2k).
 * The fine grid (nx, ny, nz) needs even nx, ny >= 2 (periodic; coarse nx/2, ny/2)
 * and odd nz >= 3 (coarse (nz+1)/2); otherwise PORTA_EINVAL.  Fields are
 * [ncomp][points] with x fastest, 1 <= ncomp <= 64.
 *
 * porta_mg_restrict: coarse = R(fine), at each coarse node the mean of the 3^3 fine
 *   nodes around it weighted w(dx) w(dy) w(dz), w(0) = 1, w(+-1) = 1/2 (the adjoint
 *   of tri-linear prolongation), over the nodes that exist (2 x 3^2 on a z boundary),
 *   divided by the sum of those weights.  FP64.  If kappa_coarse (device [Nc], sweep
 *   precision prec) is given, emis_coarse = kappa_coarse * coarse is written too
 *   ([ncomp][Nc], sweep precision); both or neither.
 */
int porta_mg_restrict(int nx, int ny, int nz, int ncomp, const double* fine, double* coarse,
                      const void* kappa_coarse, void* emis_coarse, int prec, void* stream);

/*
 * porta_mg_prolong: fine += P(coarse_a - coarse_b) (coarse_b may be NULL), P the
 *   prolongation of Sect. 5.2 of the given order.  order 1, tri-linear: a fine node on
 *   a coarse node takes its value, one on a coarse line or plane the linear or
 *   bilinear mean, the others the tri-linear mean of 8 coarse nodes.  order 3,
 *   tri-cubic-centred: the same with cubics through 4 coarse nodes per axis (centred,
 *   periodic in x and y; next to the ends of z the four nearest nodes inside), up to
 *   4^3 nodes; needs (nz + 1)/2 >= 4.  FP64.  With kappa (device [Nf], precision
 *   prec), emis = kappa * fine is written too ([ncomp][Nf]); both or neither.
 */
int porta_mg_prolong(int nx, int ny, int nz, int ncomp, int order, const double* coarse_a,
                     const double* coarse_b, double* fine, const void* kappa, void* emis,
                     int prec, void* stream);

/*
 * porta_mg_inject: coarse = fine sampled at the coarse nodes, for model fields
 *   (opacities, propagation matrix, magnetic field) of a coarser grid; elements of
 *   elem_bytes = 4 or 8 bytes.
 */
int porta_mg_inject(int nx, int ny, int nz, int ncomp, int elem_bytes, const void* fine,
                    void* coarse, void* stream);

/*
 * Emissivities from source-function multipoles, eps^K_Q = kappa S^K_Q (Sect. 2):
 *   kappa : device [N] (precision prec); s : device [ncomp][N] FP64;
 *   emis  : device [ncomp][N] (precision prec), overwritten.  1 <= ncomp <= 64.
 */
int porta_emissivity(int64_t npoints, int ncomp, const void* kappa, const double* s,
                     void* emis, int prec, void* stream);

/*
 * R_c between two iterates: rc_out (device FP64 scalar) = max_p |a_p - b_p| / |a_p|
 * over the first npoints entries (S00 rows of two [6][N] arrays).  workspace as for
 * porta_see_update.
 */
int porta_rel_change(int64_t npoints, const double* s_new, const double* s_old, double* rc_out,
                     void* workspace, size_t ws_bytes, void* stream);

/*
 * Reverse-mode derivative of a scalar loss L(i_top) through the sweep of the
 * upward rays, i.e. of the formal solution of Sect. 3.3 (Eqs. fsbez and kappa, the
 * BESSER or parabolic control point of Sect. 3.2, Table 1 for small tau_MO, the
 * interpolation at M and P of Sect. 3.1 that interp names): given dL/d i_top (same
 * layout and precision
 * as i_top), adds
 * dL/dkappa, dL/dpropmat and dL/demis (each in the layout of its field, in
 * the sweep precision) to g_kappa [N], g_propmat [6][N], g_emis [6][N].
 * The intensity field is recomputed from plane checkpoints every
 * `checkpoint_stride` planes (1..nz-1) instead of being stored.  With
 * `checkpoints` NULL the call first sweeps the upward rays to make them
 * (workspace kind PORTA_WS_ADJOINT); otherwise they are the ones porta_fs_sweep
 * wrote for these fields with the same stride and the same options' ray range
 * (kind PORTA_WS_ADJOINT_CKPT); checkpoint_bytes is the buffer's size, and below
 * porta_checkpoint_size() the call returns PORTA_ENOMEM before any launch (that
 * the contents come from such a sweep is the caller's to ensure).  With a ray
 * range in the options only its upward rays are differentiated, and the
 * gradients add up over calls.  Stride 1 keeps every plane, so nothing is
 * recomputed.  The per-frequency partials of each (node, ray) are summed over the
 * frequencies in the sweep precision, taken through the node's set-up (interpolation,
 * S = eps/eta_I, K', control point) in FP64, stored between launches in the sweep
 * precision and gathered onto the coefficients in FP64.
 * With PORTA_INTERP_BEZIER2D the derivatives of the 9-point monotonic Bezier follow
 * the branches of its clamps at the interpolated values (they depend on the values
 * around each point, so the adjoint of the Stokes vectors of a plane is gathered from
 * the plane above through the transposed stencils in a launch of its own, reading the
 * forward states of that plane; the coefficients likewise).
 */
int porta_fs_adjoint(const porta_grid* grid, const porta_quad* quad, const porta_fields* fields,
                     int prec, int interp, const porta_options* opts, const void* dl_ditop,
                     const void* checkpoints, size_t checkpoint_bytes, int checkpoint_stride,
                     void* g_kappa, void* g_propmat, void* g_emis, void* workspace,
                     size_t ws_bytes, void* stream);

/* Text of a porta_status. */
const char* porta_strerror(int status);

/* Message of the last failed call on this thread ("" if none). */
const char* porta_last_error(void);

/* Library version string. */
const char* porta_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PORTA_H */
