// porta_see_mg.hip -- host side of the statistical-equilibrium and multigrid calls of
// the C ABI declared in include/porta.h: argument checks and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/porta.h"
#include "porta_host.hpp"
#include "porta_mg.hpp"
#include "porta_see.hpp"

namespace {

using namespace porta;
using namespace porta::host;

int validate_atom(const porta_atom* atom) {
  if (!(atom->eps_c >= 0.0 && atom->eps_c <= 1.0))
    return fail(PORTA_EINVAL, "eps_c must be in [0, 1]");
  if (!(atom->delta2 >= 0.0) || !std::isfinite(atom->delta2) || !std::isfinite(atom->w2) ||
      !std::isfinite(atom->planck))
    return fail(PORTA_EINVAL, "atom parameters must be finite (delta2 >= 0)");
  return PORTA_OK;
}

int validate_coarsening(int nx, int ny, int nz, int ncomp) {
  if (nx < 2 || ny < 2 || nz < 3 || nx % 2 || ny % 2 || nz % 2 == 0)
    return fail(PORTA_EINVAL, "coarsening needs even nx, ny >= 2 and odd nz >= 3 (got %d %d %d)",
                nx, ny, nz);
  if ((double)nx * ny * nz * 10.0 >= 9.0e18 || (double)nx * ny >= 2147483647.0)
    return fail(PORTA_EINVAL, "grid too large");
  if (ncomp < 1 || ncomp > 64) return fail(PORTA_EINVAL, "ncomp must be in 1..64");
  return PORTA_OK;
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

int porta_see_update(int64_t npoints, const double* jkq, const porta_atom* atom,
                     const double* rhs, const double* s_old, double* s_new, const void* kappa,
                     void* emis_out, int prec, double* rc_out, void* workspace, size_t ws_bytes,
                     void* stream) {
  int rc;
  if ((rc = validate_prec(prec))) return rc;
  if (npoints < 1 || npoints > (int64_t)1 << 40) return fail(PORTA_EINVAL, "npoints out of range");
  if (!jkq || !atom || !s_old || !s_new) return fail(PORTA_EINVAL, "NULL argument");
  if (emis_out && !kappa) return fail(PORTA_EINVAL, "emis_out needs kappa");
  if ((rc = validate_atom(atom))) return rc;
  const size_t N = (size_t)npoints;
  const unsigned nb = (unsigned)((N + 255) / 256);
  double* blockmax = nullptr;
  if (rc_out) {
    if (!workspace) return fail(PORTA_EINVAL, "workspace is NULL");
    if (ws_bytes < sizeof(double) * nb)
      return fail(PORTA_ENOMEM, "workspace of %zu bytes is smaller than the %zu required",
                  ws_bytes, sizeof(double) * nb);
    blockmax = static_cast<double*>(workspace);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == PORTA_F64) {
    SeeArgs<double> a{jkq, rhs, s_old, s_new, atom->hanle, atom->bhat,
                      static_cast<const double*>(kappa), static_cast<double*>(emis_out),
                      blockmax, N, atom->eps_c, atom->delta2, atom->w2, atom->planck};
    hipLaunchKernelGGL(k_see<double>, dim3(nb), dim3(256), 0, st, a);
  } else {
    SeeArgs<float> a{jkq, rhs, s_old, s_new, atom->hanle, atom->bhat,
                     static_cast<const float*>(kappa), static_cast<float*>(emis_out),
                     blockmax, N, atom->eps_c, atom->delta2, atom->w2, atom->planck};
    hipLaunchKernelGGL(k_see<float>, dim3(nb), dim3(256), 0, st, a);
  }
  if ((rc = check_launch("see"))) return rc;
  if (rc_out) {
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, st, blockmax, (int)nb, rc_out);
    if ((rc = check_launch("see_rc"))) return rc;
  }
  return PORTA_OK;
}

int porta_see_operator(int64_t npoints, const double* jkq, const porta_atom* atom,
                       const double* s, const double* base, double sign, double* out,
                       void* stream) {
  int rc;
  if (npoints < 1 || npoints > (int64_t)1 << 40) return fail(PORTA_EINVAL, "npoints out of range");
  if (!jkq || !atom || !s || !out) return fail(PORTA_EINVAL, "NULL argument");
  if ((rc = validate_atom(atom))) return rc;
  if (!std::isfinite(sign)) return fail(PORTA_EINVAL, "sign must be finite");
  const size_t N = (size_t)npoints;
  SeeOpArgs a{jkq, s, base, out, atom->hanle, atom->bhat, N, sign,
              atom->eps_c, atom->delta2, atom->w2, atom->planck};
  hipLaunchKernelGGL(k_see_operator, dim3(blocks_for(N)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), a);
  return check_launch("see_operator");
}

int porta_mg_restrict(int nx, int ny, int nz, int ncomp, const double* fine, double* coarse,
                      const void* kappa_coarse, void* emis_coarse, int prec, void* stream) {
  int rc;
  if ((rc = validate_coarsening(nx, ny, nz, ncomp)) || (rc = validate_prec(prec))) return rc;
  if (!fine || !coarse) return fail(PORTA_EINVAL, "NULL argument");
  if ((emis_coarse == nullptr) != (kappa_coarse == nullptr))
    return fail(PORTA_EINVAL, "kappa_coarse and emis_coarse go together");
  const size_t Nc = (size_t)(nx / 2) * (ny / 2) * ((nz + 1) / 2);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == PORTA_F64) {
    RestrictArgs<double> a{fine, coarse, static_cast<const double*>(kappa_coarse),
                           static_cast<double*>(emis_coarse), nx, ny, nz, ncomp};
    hipLaunchKernelGGL(k_restrict<double>, dim3(blocks_for(Nc)), dim3(256), 0, st, a);
  } else {
    RestrictArgs<float> a{fine, coarse, static_cast<const float*>(kappa_coarse),
                          static_cast<float*>(emis_coarse), nx, ny, nz, ncomp};
    hipLaunchKernelGGL(k_restrict<float>, dim3(blocks_for(Nc)), dim3(256), 0, st, a);
  }
  return check_launch("mg_restrict");
}

int porta_mg_prolong(int nx, int ny, int nz, int ncomp, int order, const double* coarse_a,
                     const double* coarse_b, double* fine, const void* kappa, void* emis,
                     int prec, void* stream) {
  int rc;
  if ((rc = validate_coarsening(nx, ny, nz, ncomp)) || (rc = validate_prec(prec))) return rc;
  if (order != 1 && order != 3) return fail(PORTA_EINVAL, "order must be 1 or 3");
  if (order == 3 && (nz + 1) / 2 < 4)
    return fail(PORTA_EINVAL, "cubic prolongation needs at least 4 coarse planes (nz >= 7)");
  if (!coarse_a || !fine) return fail(PORTA_EINVAL, "NULL argument");
  if ((emis == nullptr) != (kappa == nullptr))
    return fail(PORTA_EINVAL, "kappa and emis go together");
  const size_t Nf = (size_t)nx * ny * nz;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == PORTA_F64) {
    ProlongArgs<double> a{coarse_a, coarse_b, fine, static_cast<const double*>(kappa),
                          static_cast<double*>(emis), nx, ny, nz, ncomp, order};
    hipLaunchKernelGGL(k_prolong<double>, dim3(blocks_for(Nf)), dim3(256), 0, st, a);
  } else {
    ProlongArgs<float> a{coarse_a, coarse_b, fine, static_cast<const float*>(kappa),
                         static_cast<float*>(emis), nx, ny, nz, ncomp, order};
    hipLaunchKernelGGL(k_prolong<float>, dim3(blocks_for(Nf)), dim3(256), 0, st, a);
  }
  return check_launch("mg_prolong");
}

int porta_mg_inject(int nx, int ny, int nz, int ncomp, int elem_bytes, const void* fine,
                    void* coarse, void* stream) {
  int rc;
  if ((rc = validate_coarsening(nx, ny, nz, ncomp))) return rc;
  if (!fine || !coarse) return fail(PORTA_EINVAL, "NULL argument");
  const size_t Nc = (size_t)(nx / 2) * (ny / 2) * ((nz + 1) / 2);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_inject<double>, dim3(blocks_for(Nc)), dim3(256), 0, st,
                       static_cast<const double*>(fine), static_cast<double*>(coarse), nx, ny,
                       nz, ncomp);
  else if (elem_bytes == 4)
    hipLaunchKernelGGL(k_inject<float>, dim3(blocks_for(Nc)), dim3(256), 0, st,
                       static_cast<const float*>(fine), static_cast<float*>(coarse), nx, ny, nz,
                       ncomp);
  else
    return fail(PORTA_EINVAL, "elem_bytes must be 4 or 8");
  return check_launch("mg_inject");
}

int porta_rel_change(int64_t npoints, const double* s_new, const double* s_old, double* rc_out,
                     void* workspace, size_t ws_bytes, void* stream) {
  int rc;
  if (npoints < 1 || npoints > (int64_t)1 << 40) return fail(PORTA_EINVAL, "npoints out of range");
  if (!s_new || !s_old || !rc_out || !workspace) return fail(PORTA_EINVAL, "NULL argument");
  const size_t N = (size_t)npoints;
  const unsigned nb = blocks_for(N);
  if (ws_bytes < sizeof(double) * nb)
    return fail(PORTA_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                sizeof(double) * nb);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double* blockmax = static_cast<double*>(workspace);
  hipLaunchKernelGGL(k_rel_change, dim3(nb), dim3(256), 0, st, s_new, s_old, N, blockmax);
  if ((rc = check_launch("rel_change"))) return rc;
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, st, blockmax, (int)nb, rc_out);
  return check_launch("rel_change_final");
}

int porta_emissivity(int64_t npoints, int ncomp, const void* kappa, const double* s,
                     void* emis, int prec, void* stream) {
  int rc;
  if ((rc = validate_prec(prec))) return rc;
  if (npoints < 1 || npoints > (int64_t)1 << 40) return fail(PORTA_EINVAL, "npoints out of range");
  if (ncomp < 1 || ncomp > 64) return fail(PORTA_EINVAL, "ncomp must be in 1..64");
  if (!kappa || !s || !emis) return fail(PORTA_EINVAL, "NULL argument");
  const size_t N = (size_t)npoints;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (prec == PORTA_F64)
    hipLaunchKernelGGL(k_emissivity<double>, dim3(blocks_for(N)), dim3(256), 0, st,
                       static_cast<const double*>(kappa), s, static_cast<double*>(emis), N, ncomp);
  else
    hipLaunchKernelGGL(k_emissivity<float>, dim3(blocks_for(N)), dim3(256), 0, st,
                       static_cast<const float*>(kappa), s, static_cast<float*>(emis), N, ncomp);
  return check_launch("emissivity");
}

}  // extern "C"
