// Device-side data of the solver and the launch wrappers of its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amrfld {

constexpr int kBlock = 256;  // threads per block = slots per tile
constexpr int kMaxTilesPerBlock = 16;

// Scalars of one PCG solve in device memory.  The sweeps derive alpha, beta and
// the stopping decision themselves from the previous sweep's block partials;
// the host reads this record only between batches of iterations.
struct PcgScalars {
  double rho[2];    // (r, z) of iterate j, stored at index j & 1
  double rnorm0, bnorm, thresh;
  double tol, abs_floor;
  double rnorm;     // ||r_j|| of the recursive residual
  double linf;      // max |x_j - x_{j-1}| / |x_{j-1}|
  double true_rnorm;
  double min_E;
  int iter;         // completed iterations
  int done;         // 1 once converged, failed or out of iterations
  int converged;
  int nonfinite;
  int max_iter;
  int linf_test;
};

// One level's (or one batch's) device tables, slot order.
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
  int kmode;  // 0 const, 1 Levermore-Pomraning
  double K_const, kappa_R, c_light;
};

struct CouplingParams {
  const double* T;  // nullptr: no coupling
  double kappa_P, c_light, a_rad, c_v;
};

inline int tiles_of(int64_t n_slots) { return int((n_slots + kBlock - 1) / kBlock); }
int grid_for(int64_t n);

// ------------------------------------------------------------ setup kernels
void launch_cell_K(hipStream_t s, const DevLevel& L, const double* E, const double* rho,
                   const double* E_coarse, const CellKParams& kp, double* K);
void launch_assemble(hipStream_t s, const DevLevel& L, const double* K, const double* K_coarse,
                     const double* E, const double* E_coarse, const double* rho, const double* reg,
                     double dt, double w, const CouplingParams& cp, double* Cp, double* diag,
                     double* b);
void launch_flux_register(hipStream_t s, const DevLevel& F, const double* K_f, const double* K_c,
                          const double* E_f, const double* E_c, double dt, double* reg_c,
                          int n_slots_c);
void launch_restrict(hipStream_t s, const DevLevel& F, const double* E_f, double* E_c);
void launch_fill(hipStream_t s, double* p, int64_t n, double v);
void launch_fill_f32(hipStream_t s, float* p, int64_t n, float v);
void launch_to_f32(hipStream_t s, int64_t n, const double* Cp, const double* diag, float* Cp32,
                   float* diag32);

// -------------------------------------------------------------- PCG sweeps
// G = number of blocks of every sweep of a solve (<= tiles); partials hold
// 4 G doubles: [0, G) for the operator sweep, [G, 4G) for the update sweep.
int sweep_blocks(int n_tiles, int max_blocks);

template <typename T>
void launch_pcg_init(hipStream_t s, const DevLevel& L, int G, const T* Cp, const T* diag,
                     const T* b, const T* x, T* r, T* p_clear, double* part);
void launch_init_finish(hipStream_t s, int G, const double* part, PcgScalars* sc);
template <typename T>
void launch_pass_a(hipStream_t s, const DevLevel& L, int G, int it, const T* Cp, const T* diag,
                   const T* r, const T* p_old, T* p_new, T* q, PcgScalars* sc, double* part);
template <typename T>
void launch_pass_b(hipStream_t s, const DevLevel& L, int G, int it, const T* diag, const T* p,
                   const T* q, T* x, T* r, PcgScalars* sc, double* part);
void launch_check(hipStream_t s, int G, int it_last, PcgScalars* sc, const double* part);
void launch_true_residual(hipStream_t s, const DevLevel& L, int G, const double* Cp,
                          const double* diag, const double* b, const double* x, PcgScalars* sc,
                          double* part);
void launch_post_solve(hipStream_t s, const DevLevel& L, int G, const double* E, const double* rho,
                       const CouplingParams& cp, double dt, double* T_out, PcgScalars* sc,
                       double* part);

// ------------------------------------------- mixed precision (FP32 inner solve)
// Outer sweep: x_new = x_old + d (d in FP32, may be null), r = b - A x_new in
// FP64, r32 = (float) r; partials ||r||^2, ||b||^2, max |d| / |x_old|; then the
// finisher applies the outer stopping test and prepares the inner scalars.
void launch_ir_sweep(hipStream_t s, const DevLevel& L, int G, const double* Cp, const double* diag,
                     const double* b, const double* x_old, const float* d, double* x_new,
                     float* r32, double* part);
void launch_ir_finish(hipStream_t s, int G, int first, double inner_tol, int inner_max,
                      PcgScalars* outer, PcgScalars* inner, const double* part);
// Inner start: d = 0, p = 0; partials (r, r / diag), ||r||^2 of the FP32 residual.
void launch_inner_init(hipStream_t s, const DevLevel& L, int G, const float* diag32, const float* r32,
                       float* d, float* p_clear, double* part);

}  // namespace amrfld
