// adjoint.h -- argument blocks and launch wrappers of the adjoint kernels (adjoint.hip),
// shared with the C ABI (api.hip).
#pragma once

#include "gmhc_internal.h"

namespace gmhc {

// ---- adjoint of the step and of initialization (adjoint.hip; quadratic shape, FP64) --

enum AdjMode { ADJ_BOUND = 0, ADJ_SCATTER = 1, ADJ_FINAL = 2, ADJ_PREP = 3 };
// scattered field arrays in dimension d: grad phi (d), A^n (3), A^{n+1} (3)
constexpr int adj_nvals(int d) { return d + 6; }
// Per-particle values of the step that do not depend on the adjoint current: the columns
// dv_out/dvbar_j, j < d (3 d), the part of the inner right side from the output
// cotangents (d), and the gather cotangents (grad-phi-bar (d), D (3 d), A^- (3), A^+ (3))
// of the reverse sweeps for the unit cotangents of v_out along x, y, z and for the
// cotangent of P^{n+1} (4 sets).
constexpr int adj_ngath(int d) { return 4 * d + 6; }
constexpr int adj_ncache(int d) { return 4 * d + 4 * adj_ngath(d); }

// Per-particle reverse sweep at the converged step.  ADJ_PREP (k_adj_particle): the values
// above into cache; ADJ_BOUND (k_adj_iter): per-block sums of a bound on the values to be
// scattered (for the fixed-point scale); ADJ_SCATTER (k_adj_iter): the cotangents of the
// trial fields into acc; ADJ_FINAL (k_adj_particle): the cotangents of x, P and q.
struct AdjArgs {
  Mesh M;
  int64_t np;
  double dt, kappa;
  int ngl;
  double glx[kMaxGL], glw[kMaxGL];
  // particle state in the library's internal order, component stride ps
  int64_t ps;
  const double* x;
  const double* P;
  const double* q;
  const int32_t* id;     // internal index -> load order
  // load order, component stride np
  const double* vbar;    // [3] converged orbit velocity of the step
  const double* lx;      // [dim] cotangent of x^{n+1}
  const double* lP;      // [3] cotangent of P^{n+1}
  // trial fields of the converged current (real, stride Ng)
  const double* gphi;    // [dim]
  const double* An;      // [3]
  const double* Anp1;    // [3]
  const double* mu;      // [3] adjoint current (already projected); null = zero
  int mode;
  double* partials;      // ADJ_BOUND: per-block sums of the scatter bound
  unsigned long long* acc;  // ADJ_SCATTER: [dim + 6][Ng] fixed-point pairs
  const double* fx;      // ADJ_SCATTER: the fixed-point scale (up, hi, lo) in device memory
  double* cache;         // [adj_ncache(dim)][ps]: written by ADJ_PREP, read by ADJ_BOUND, ADJ_SCATTER, ADJ_FINAL
  double* gx;            // ADJ_FINAL outputs, load order
  double* gP;
  double* gq;
};

hipError_t launch_adj_particle(const AdjArgs& a, hipStream_t s);  // ADJ_PREP, ADJ_FINAL
hipError_t launch_adj_iter(const AdjArgs& a, hipStream_t s);      // ADJ_BOUND, ADJ_SCATTER
int64_t adj_particle_blocks(int64_t np);

struct AdjFieldArgs {
  Mesh M;
  double dt, kappa2, sigma1, sigma2;
  int project;
  const double2* Lf;    // [9][Ng] spectra of the output-state cotangents: phi psi rho A(3) U(3)
  const double2* Pb;    // [d+6][Ng] spectra of the trial-field cotangents: grad phi (d), A^n (3), A^{n+1} (3); null = 0
  double2* Ls;          // out [9][Ng]: input-state cotangents
  double2* Lj;          // out [3][Ng]: current cotangent
};

hipError_t launch_adj_field(const AdjFieldArgs& a, hipStream_t s);
// Spectra [9][Ng] of the cotangent of the field energy with respect to the state S.
hipError_t launch_energy_grad(const Mesh& M, double sigma1, double sigma2, const double2* S, double2* out,
                              hipStream_t s);
// Spectrum of the total charge cotangent at initialization from the state cotangent spectra L.
hipError_t launch_adj_init_field(const Mesh& M, double sigma1, int project, const double2* L, double2* out,
                                 hipStream_t s);
struct AdjInitArgs {
  Mesh M;
  int64_t np, ps;
  double kappa;
  const double* x;
  const double* P;
  const double* q;
  const int32_t* id;
  const double* A0;   // [3][Ng] real A^0
  const double* rb;   // [Ng] real rho-bar_total
  const double* lx;   // load order
  const double* lP;
  double* gx;
  double* gu;
  double* gq;
};

hipError_t launch_adj_init_particle(const AdjInitArgs& a, hipStream_t s);
// mu <- mu + beta (mnew - mu) over n values; out[0] = max |mnew - mu|, out[1] = max |mnew|.
hipError_t launch_adj_update(double* mu, const double* mnew, int64_t n, double beta, double* out, hipStream_t s);
// out[0] = fixed-order sum of p[0..n).
hipError_t launch_adj_sum(const double* p, int64_t n, double* out, hipStream_t s);
// The fixed-point scale (up, hi, lo) of sums bounded by bound[0] (fix_scale, on the device),
// and the conversion of fixed-point pairs to doubles with a scale in device memory.
hipError_t launch_adj_scale(const double* bound, double* fx, hipStream_t s);
hipError_t launch_adj_fix_to_double(const unsigned long long* acc, double* out, int64_t n, const double* fx,
                                    hipStream_t s);

}  // namespace gmhc
