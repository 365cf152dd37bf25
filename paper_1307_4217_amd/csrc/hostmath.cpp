// hostmath.cpp -- host build of porta_math.hpp, exported for CPU unit tests of
// the per-update arithmetic used by the GPU kernels.
#include "porta_math.hpp"

extern "C" {

void hm_coefficients_f32(float tau, float* out6) {
  const porta::Coefs<float> c = porta::coefficients(tau);
  out6[0] = c.e; out6[1] = c.psiM; out6[2] = c.psiO;
  out6[3] = c.omM; out6[4] = c.omO; out6[5] = c.omC;
}

void hm_coefficients_f64(double tau, double* out6) {
  const porta::Coefs<double> c = porta::coefficients(tau);
  out6[0] = c.e; out6[1] = c.psiM; out6[2] = c.psiO;
  out6[3] = c.omM; out6[4] = c.omO; out6[5] = c.omC;
}

double hm_besser_cm(double yM, double yO, double yP, double ratio) {
  return porta::besser_cm(yM, yO, yP, ratio);
}

double hm_parabolic_cm(double yM, double yO, double yP, double ratio) {
  return porta::parabolic_cm(yM, yO, yP, ratio);
}

double hm_parabolic_cm_grad(double yM, double yO, double yP, double ratio, double* d4) {
  return porta::parabolic_cm_grad(yM, yO, yP, ratio, d4);
}

double hm_bezier3_f64(double ym, double y0, double yp, double t) {
  return porta::bezier3(ym, y0, yp, t);
}

float hm_bezier3_f32(float ym, float y0, float yp, float t) {
  return porta::bezier3(ym, y0, yp, t);
}

double hm_bezier3_grad_f64(double ym, double y0, double yp, double t, double* g3) {
  return porta::bez_eval_grad(porta::bez_weights(t), ym, y0, yp, g3);
}

void hm_solve_stokes_f64(const double* e3, const double* r3, const double* b4, double* x4) {
  porta::solve_stokes(e3, r3, b4, x4);
}

void hm_solve_stokes_f32(const float* e3, const float* r3, const float* b4, float* x4) {
  porta::solve_stokes(e3, r3, b4, x4);
}

// (1 + p K')^-1 b (sgn = 1) or its transpose (sgn = -1), through the per-node
// operator and per-frequency scalars the kernels use.
void hm_stokes_solve_scaled_f64(const double* e3, const double* r3, double p, const double* b4,
                                int sgn, double* x4) {
  const porta::StokesOp<double> k = porta::stokes_op(e3, r3);
  const porta::StokesFreq<double> F = porta::stokes_freq(k, p);
  if (sgn > 0)
    porta::stokes_solve<1>(k, F, b4, x4);
  else
    porta::stokes_solve<-1>(k, F, b4, x4);
}

void hm_stokes_solve_scaled_f32(const float* e3, const float* r3, float p, const float* b4,
                                int sgn, float* x4) {
  const porta::StokesOp<float> k = porta::stokes_op(e3, r3);
  const porta::StokesFreq<float> F = porta::stokes_freq(k, p);
  if (sgn > 0)
    porta::stokes_solve<1>(k, F, b4, x4);
  else
    porta::stokes_solve<-1>(k, F, b4, x4);
}

void hm_kprime_apply(const double* e3, const double* r3, const double* x4, double* y4) {
  porta::kprime_apply(e3, r3, x4, y4);
}

// emis[4][6] then proj[9][4] then (mu, sx, sy, weight)
void hm_ray_consts(double mu, double chi, double weight, double w2, double* out) {
  porta::RayConsts rc;
  porta::ray_consts(mu, chi, weight, w2, rc);
  int k = 0;
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 6; ++c) out[k++] = rc.emis[i][c];
  for (int c = 0; c < 9; ++c)
    for (int i = 0; i < 4; ++i) out[k++] = rc.proj[c][i];
  out[k++] = rc.mu;
  out[k++] = rc.sx;
  out[k++] = rc.sy;
  out[k++] = rc.weight;
}

// Solve the K = 2 Hanle system; rhs5 in, x5 out.
void hm_hanle_solve(double a, double h, double bx, double by, double bz, const double* rhs5,
                    double* x5) {
  double A[5][5], b[5];
  porta::hanle_system(a, h, bx, by, bz, A);
  for (int i = 0; i < 5; ++i) b[i] = rhs5[i];
  porta::solve_pivot<5>(A, b);
  for (int i = 0; i < 5; ++i) x5[i] = b[i];
}

// The pivoted 5x5 elimination of the SEE on a general system: A row-major, b in, x out.
void hm_solve_pivot5(const double* A25, const double* b5, double* x5) {
  double A[5][5], b[5];
  for (int i = 0; i < 5; ++i) {
    for (int k = 0; k < 5; ++k) A[i][k] = A25[5 * i + k];
    b[i] = b5[i];
  }
  porta::solve_pivot<5>(A, b);
  for (int i = 0; i < 5; ++i) x5[i] = b[i];
}

double hm_besser_cm_grad(double yM, double yO, double yP, double ratio, double* d4) {
  return porta::besser_cm_grad(yM, yO, yP, ratio, d4);
}

double hm_coef_tau_grad_f64(double tau, const double* g6) {
  const porta::Coefs<double> c = porta::coefficients(tau);
  return porta::coef_tau_grad(c, g6[0], g6[1], g6[2], g6[3], g6[4], g6[5]);
}

float hm_coef_tau_grad_f32(float tau, const float* g6) {
  const porta::Coefs<float> c = porta::coefficients(tau);
  return porta::coef_tau_grad(c, g6[0], g6[1], g6[2], g6[3], g6[4], g6[5]);
}

}  // extern "C"
