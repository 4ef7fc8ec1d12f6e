// orc_config.h -- run parameters of the CPU oracle (test infrastructure only; shared by
// the oracle's own translation units, never by the GPU library).
#pragma once

#include <stdint.h>

extern "C" {

// Run parameters (Table 1 and the common settings of the numerical-results section).
struct orc_config {
  int32_t dim;          // resolved spatial dimensions d in {1,2,3}; momenta are always 3V
  int32_t n[3];         // nodes per axis (1 for unresolved axes)
  double lo[3];         // lower domain corner
  double len[3];        // periodic lengths
  double kappa;         // nondimensional speed of light
  double sigma1;        // source coefficient of the phi equation
  double sigma2;        // source coefficient of the A equation
  double dt;            // time step
  int32_t gl_order;     // Gauss-Legendre points per knot segment (paper: 8)
  int32_t project;      // 1: apply the Nyquist projector
  double tol_outer_abs, tol_outer_rel;
  double tol_inner_abs, tol_inner_rel;
  int32_t max_outer, max_inner;
  double beta;          // damping of the outer current iteration (Picard step beta r)
  int32_t threads;      // OpenMP threads (0: runtime default)
  int32_t outer_scheme; // 0: damped Picard; 1: type-II Anderson (the paper's solver)
  int32_t anderson_m;   // Anderson memory M (paper: 4)
  int32_t anderson_start; // outer iteration from which Anderson is eligible (paper: 2)
  int32_t ls_halvings;  // backtracking alpha = 1, 1/2, ..., 2^-ls_halvings (paper: 6)
  double anderson_lambda; // regularization lambda (paper: 1e-12)
  double ls_decrease;   // sufficient-decrease coefficient (paper: 1e-4)
  double ls_growth;     // residual-growth limit (paper: 1.2)
  int32_t shape_order;  // B-spline degree r of the particle shape: 2 (the paper's; 0 selects
                        // it) or 1, the linear shape of the spline-degree comparison
  int32_t refine_levels;  // convergence-triggered particle refinement: a particle whose
                          // solve fails is retried with 2, 4, ... 2^refine_levels equal
                          // particle sub-steps (0: off; at most kMaxRefine)
};

}  // extern "C"
