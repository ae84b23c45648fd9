// Device-side data of the solver and the launch wrappers of its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amrfld {

// Scalars of one PCG solve, kept in device memory so that the iteration runs
// without host round trips; the host reads them between batches of iterations.
struct PcgScalars {
  double rho;       // (r, z) of the current iterate
  double alpha, beta;
  double rnorm0, bnorm, thresh;
  double rnorm;     // ||r_j|| of the recursive residual
  double linf;      // max |x_j - x_{j-1}| / |x_{j-1}|
  double true_rnorm;
  double min_E;
  double tol;
  double abs_floor;
  int iter;         // completed iterations
  int done;         // 1 once converged, failed or out of iterations
  int converged;
  int nonfinite;
  int max_iter;
  int linf_test;
  unsigned cnt[4];  // arrival counters of the last-block reductions
};

// One level's device arrays (slot order).
struct DevLevel {
  int n_slots;
  int n_oct;
  const int32_t* nbr;     // [n_oct*6]
  const int32_t* cnb;     // [n_oct*6]
  const int32_t* child;   // [n_slots]
  const int32_t* parent;  // [n_oct]
  double dx, vol;
};

struct CellKParams {
  int kmode;        // 0 const, 1 Levermore-Pomraning
  double K_const, kappa_R, c_light;
};

struct CouplingParams {
  const double* T;  // nullptr: no coupling
  double kappa_P, c_light, a_rad, c_v;
};

// Per-block partial sums need at most this many blocks per launch.
constexpr int kBlock = 256;

int grid_for(int64_t n);

// Cell diffusivity K of every slot of a level.
void launch_cell_K(hipStream_t s, const DevLevel& L, const double* E, const double* rho,
                   const double* E_coarse, const CellKParams& kp, double* K);

// Face coefficients C+ (3 arrays), diagonal and right-hand side.
void launch_assemble(hipStream_t s, const DevLevel& L, const double* K, const double* K_coarse,
                     const double* E, const double* E_coarse, const double* rho, const double* reg,
                     double dt, double w, const CouplingParams& cp, double* Cp, double* diag,
                     double* b);

// PCG (FP64).  x holds x0 on entry and the iterate on exit.
void launch_pcg_init(hipStream_t s, const DevLevel& L, const double* Cp, const double* diag,
                     const double* b, const double* x, double* r, double* p_clear,
                     PcgScalars* sc, double* partials);
void launch_pass_a(hipStream_t s, const DevLevel& L, const double* Cp, const double* diag,
                   const double* r, const double* p_old, double* p_new, double* q, PcgScalars* sc,
                   double* partials);
void launch_pass_b(hipStream_t s, const DevLevel& L, const double* diag, const double* p,
                   const double* q, double* x, double* r, PcgScalars* sc, double* partials);
void launch_true_residual(hipStream_t s, const DevLevel& L, const double* Cp, const double* diag,
                          const double* b, const double* x, PcgScalars* sc, double* partials);

// Post-solve: temperature update (coupling), smallest leaf energy.
void launch_post_solve(hipStream_t s, const DevLevel& L, const double* E, const double* rho,
                       const CouplingParams& cp, double dt, double* T_out, PcgScalars* sc,
                       double* partials);

// Adds the energy gained through every fine-to-coarse face of the fine level to
// the register of the coarse level (slot-major per direction: reg[d*n + slot]).
void launch_flux_register(hipStream_t s, const DevLevel& F, const double* K_f, const double* K_c,
                          const double* E_f, const double* E_c, double dt, double* reg_c,
                          int n_slots_c);

// Refined slots of the coarse level take the mean of their 8 children.
void launch_restrict(hipStream_t s, const DevLevel& F, const double* E_f, double* E_c);

void launch_fill(hipStream_t s, double* p, int64_t n, double v);

}  // namespace amrfld
