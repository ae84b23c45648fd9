// Device-side data of the solver and the launch wrappers of its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amrfld {

constexpr int kBlock = 256;  // threads per block = slots per tile
// LDS of one block's staged range of one vector in the staged sweeps: at most 16
// tiles per block in the FP64 sweeps and, in the same bytes, 32 in the FP32 ones
// (fewer, longer ranges: fewer faces gathered across range ends).
constexpr int kStageBytes = 32768;
constexpr int kMaxTilesPerBlock = kStageBytes / (kBlock * int(sizeof(double)));
constexpr int kMaxTilesPerBlock32 = kStageBytes / (kBlock * int(sizeof(float)));

// Words of the persistent launch's control buffer (unsigned), each on its own
// 256-byte line: grid-barrier arrivals (of the XCD groups) and releases, the count
// of problems whose PCG (or inner PCG) stopped, the count of problems whose
// refinement loop stopped (mixed precision), the first barrier's arrivals and
// release, then per XCD (up to kMaxXcd) its count of resident blocks, its arrivals
// and its release, and last the abort flag.  The first kBarAbort words are zeroed
// before every persistent launch.
constexpr int kMaxXcd = 16;
constexpr int kBarArrive = 0, kBarRelease = 64, kBarDone = 128, kBarOuterDone = 192, kBarFirstArrive = 256,
              kBarFirstRelease = 320, kBarXcdCount = 384, kBarXcdArrive = kBarXcdCount + 64 * kMaxXcd,
              kBarXcdRelease = kBarXcdArrive + 64 * kMaxXcd, kBarAbort = kBarXcdRelease + 64 * kMaxXcd,
              kBarWords = kBarAbort + 64;

// Scalars of one PCG solve in device memory.  The sweeps derive alpha, beta and
// the stopping decision themselves from the previous sweep's block partials;
// the host reads this record only between batches of iterations.
struct PcgScalars {
  double gam[2];    // (r^, r^) of iterate j (scaled residual), stored at index j & 1
  double alpha[2];  // step alpha_j that takes iterate j to j + 1, at index j & 1
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
  int counted;      // this problem's stop has been added to the plan's done counter
  int inner_total;  // mixed precision, outer record: inner iterations of the refinement so far
  // mixed precision, inner record: 0 = the inner CG starts afresh (p = 0); 1 or 2 =
  // it continues its search direction after a residual replacement, with s^ of the
  // last iteration in buffer cont - 1 (gam[1], alpha[1] hold that iteration's scalars)
  int cont;
  int pad_;
};

// Parameters of one independent patch of a batch: a box of cells of size dx
// whose boundary faces carry a Dirichlet, Neumann or Robin condition (the
// interface rows of Sect. 3.2 with a given ghost value and inflow).
struct PatchParams {
  double dx, vol, coef;  // coef = dt / dx^2
  double kappa_R, c_light, K_const;
  double ghost[6], flux[6];
  int mode[6];
  int kmode;
  double K_exp;  // composite system: the level's power-law exponent (boundary diffusivity)
};

// One level's (or one batch's) device tables, slot order.  child: >= 0 child
// oct (refined slot), -1 leaf, -2 padding slot of a batch (identity row).
struct DevLevel {
  int n_slots = 0;
  int n_oct = 0;
  const int32_t* nbr = nullptr;       // [n_oct*6]
  const int32_t* cnb = nullptr;       // [n_oct*6]
  const int32_t* child = nullptr;     // [n_slots]
  const int32_t* parent = nullptr;    // [n_oct]
  double dx = 1.0, vol = 1.0;
  const int32_t* oct_prob = nullptr;  // batch: patch of each oct; composite: level of each oct
  const PatchParams* pp = nullptr;    // batch: per-patch parameters; composite: per-level dx, vol, coef
  // Composite system of all levels (unique time step), else nullptr: cif[a * n + i]
  // is the volume-scaled coefficient of slot i's out-of-oct face on axis a when that
  // face looks at a coarser leaf (0 otherwise); bit d of c2f[i] is set when the
  // same-level neighbour in direction d is refined, whose four finer cells on that
  // face are then coupled to i with their own cif.  nbr, cnb and child then hold
  // indices into the concatenated slot space of all levels.
  const double* cif = nullptr;
  const uint8_t* c2f = nullptr;
  // Composite: the rows with couplings to other levels, row if_row[t] holding
  // entries [if_ptr[t], if_ptr[t+1]) of column if_col and coefficient cif[if_src].
  int n_if_rows = 0;
  const int32_t* if_row = nullptr;
  const int32_t* if_ptr = nullptr;
  const int32_t* if_col = nullptr;
  const int32_t* if_src = nullptr;
  const double* if_val = nullptr;  // cif[if_src[e]], gathered once per solve
  double* if_part = nullptr;       // partials of the interface kernel
};

// How the blocks of a sweep are spread over independent problems (a level is
// one problem).  Problem q owns blocks [blk0[q], blk0[q+1]) and tiles
// [tile0[q], tile0[q+1]); blocks never straddle problems, so block partials
// and scalars are per problem.
struct SweepPlan {
  int n_prob = 1;
  int G = 1;                          // total blocks
  int n_tiles = 0;                    // used when the arrays are null (one problem)
  int tpb_max = 1;                    // largest tile count of one block (sizes the LDS of the staged sweeps)
  const int32_t* blk_prob = nullptr;  // [G] or nullptr
  const int32_t* blk0 = nullptr;      // [n_prob + 1] or nullptr
  const int32_t* tile0 = nullptr;     // [n_prob + 1] or nullptr
  unsigned* done_count = nullptr;     // counts problems that stopped (read by the persistent sweep)
  // one problem only: more (w^, r^) partials that the iteration sweep's head adds to
  // its own (the couplings of the composite system to other levels)
  const double* extra_part = nullptr;
  int n_extra = 0;
};
inline SweepPlan single_plan(int G, int n_tiles) {
  SweepPlan p;
  p.n_prob = 1;
  p.G = G;
  p.n_tiles = n_tiles;
  p.tpb_max = (n_tiles + G - 1) / G;
  p.blk_prob = nullptr;
  p.blk0 = nullptr;
  p.tile0 = nullptr;
  p.done_count = nullptr;
  return p;
}

struct CellKParams {
  int kmode;  // 0 const, 1 Levermore-Pomraning, 2 Minerbo, 3 power law K_const E^K_exp
  double K_const, kappa_R, c_light;
  double K_exp = 0.0;
};

// Faces of the unit box (directions -x, +x, -y, +y, -z, +z): bit d of mask set
// means a Dirichlet energy val[d] held at that face, dx / 2 from the cell centres;
// the other faces carry no flux.
struct OuterBC {
  unsigned mask = 0;
  double val[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
};

// Face coefficients of the operator of a solve, stored or formed in every sweep.
// Stored (Cp set): Cp[a][i] is the coefficient of the +a face of slot i, zero
// unless both sides are leaves of the level.  Formed (K set): the face of slot i
// in direction d couples it to its neighbour j when bit d of mask[i] is set, with
// coefficient harmonic(K_i, K_j) * scale, times theta when theta != 1: the very
// expression of the assembly, so both forms give the same bits while the sweeps
// read one diffusivity per slot instead of three coefficients.  scale = dt / dx^2
// of the level, or per problem from the batch table (per_problem).
template <typename T>
struct FaceCoefs {
  const T* Cp = nullptr;
  const T* K = nullptr;
  const uint8_t* mask = nullptr;
  double scale = 1.0;
  double theta = 1.0;
  bool per_problem = false;
};

// The Jacobi-scaled operator A^ = S A S, S = diag(rs), rs = 1 / sqrt(diag A), of a
// solve, as the CG sweeps read it: its diagonal is 1 on every row and the
// coefficient of a face is C_f rs_i rs_j.  Stored (Ch set): Ch[a][i] for the +a face
// of slot i, zero unless both sides are leaves.  Formed (K set): from the two
// diffusivities with the assembly's expression, times rs_i rs_j, the same bits.
template <typename T>
struct ScaledOp {
  const T* Ch = nullptr;
  const T* K = nullptr;
  const uint8_t* mask = nullptr;
  const T* rs = nullptr;  // always set
  double scale = 1.0;
  double theta = 1.0;
  bool per_problem = false;
};

// Vectors of the CG iteration on the scaled system: residual r^, w^ = A^ r^ and
// s^ = A^ p^ in two buffers each (the sweep of iteration it reads buffer
// (it - 1) & 1 and writes it & 1, so values that other blocks recompute across
// their range boundaries are never overwritten during a sweep), search direction p^.
template <typename T>
struct CgVecs {
  T* r[2] = {nullptr, nullptr};
  T* w[2] = {nullptr, nullptr};
  T* s[2] = {nullptr, nullptr};
  T* p = nullptr;
};

struct CouplingParams {
  const double* T;  // nullptr: no coupling
  double kappa_P, c_light, a_rad, c_v;
};

inline int tiles_of(int64_t n_slots) { return int((n_slots + kBlock - 1) / kBlock); }
int grid_for(int64_t n);

// ------------------------------------------------------------ setup kernels
void launch_cell_K(hipStream_t s, const DevLevel& L, const double* E, const double* rho,
                   const double* E_coarse, const CellKParams& kp, const OuterBC& ob, double* K);
// w: weight of the coarse-to-fine Dirichlet part (1 D, 0 N, alpha R); alpha: Robin
// weight of batch patch faces whose mode is Robin; kp and ob: the diffusivity law and
// the box faces' Dirichlet values (no patch table).
// mask: bit d of slot i set when its face in direction d couples two leaves.
void launch_assemble(hipStream_t s, const DevLevel& L, const double* K, const double* K_coarse,
                     const double* E, const double* E_coarse, const double* rho, const double* reg,
                     double dt, double w, double alpha, const CouplingParams& cp, const CellKParams& kp,
                     const OuterBC& ob, double* Cp, uint8_t* mask, double* diag, double* b);
// Theta-weighted step (Crank-Nicolson at 1/2) from an assembled backward-Euler
// level system: b -= (1 - theta) (A E - E) on the leaves, then A = I + theta (A - I).
void launch_theta_step(hipStream_t s, const DevLevel& L, double theta, const double* E,
                       const FaceCoefs<double>& A1, double* Cp, double* diag, double* b);
// Composite system of all levels advanced with one dt (unique time step): per slot
// the volume-scaled same-level coefficients Cp, interface coefficients cif, the
// refined-neighbour mask c2f, diagonal and right-hand side; E is the concatenated
// energy, K the concatenated diffusivity of every level.
void launch_assemble_composite(hipStream_t s, const DevLevel& C, const double* K, const double* E,
                               const double* rho, const CouplingParams& cp, const OuterBC& ob, double dt,
                               double* Cp, double* cif, uint8_t* c2f, double* diag, double* b);
void launch_flux_register(hipStream_t s, const DevLevel& F, const double* K_f, const double* K_c,
                          const double* E_f, const double* E_c, double dt, double* reg_c,
                          int n_slots_c);
void launch_restrict(hipStream_t s, const DevLevel& F, const double* E_f, double* E_c);
void launch_fill(hipStream_t s, double* p, int64_t n, double v);
// dst[i] = src[i] for n device doubles (a plain streaming copy; the runtime's
// generic copy runs far below HBM rate at these sizes).
void launch_copy_f64(hipStream_t s, double* dst, const double* src, int64_t n);
void launch_fill_f32(hipStream_t s, float* p, int64_t n, float v);
// Jacobi scaling of an assembled operator: rs = 1 / sqrt(diag) on every slot and,
// when Cp is given, Ch[a][i] = Cp[a][i] rs_i rs_j for the +a neighbour j.
void launch_jacobi_scale(hipStream_t s, const DevLevel& L, const double* Cp, const double* diag, double* rs,
                         double* Ch);
// FP32 copies of a scaled operator: Ch (stored form) or K (formed), and rs.
void launch_to_f32(hipStream_t s, int64_t n, const double* Ch, const double* K, const double* rs, float* Ch32,
                   float* K32, float* rs32);

// -------------------------------------------------------------- PCG sweeps
// Jacobi PCG (Sect. 3.3.4) run as CG on the Jacobi-scaled system with the
// recurrences of Chronopoulos and Gear: one fused sweep per iteration, whose two
// dot products are reduced together at the head of the next sweep.  G = number of
// blocks of every sweep of a solve (<= tiles); partials hold 8 G doubles, 4 per
// block for each iteration parity.  max_tiles: the most tiles one block may take
// (kMaxTilesPerBlock for FP64 sweeps, kMaxTilesPerBlock32 for FP32 ones).
int sweep_blocks(int n_tiles, int max_blocks, int max_tiles = kMaxTilesPerBlock);

// Every launcher below covers all problems of the plan; sc points at n_prob
// scalar records.
// The two start sweeps of a solve without couplings to other levels, staged in LDS
// like the iteration sweep: r^_0 = rs b - A^ (x0 / rs), p^ = 0, s^ buffer 0 = 0, then
// w^_0 = A^ r^_0 and the partials the first iteration sweep reduces.
template <typename T>
void launch_cg_start(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<T>& Ah, const T* b,
                     const T* x, const CgVecs<T>& v, double* part);
// The start sweeps of the composite system (couplings to other levels included).
// Sweep 1: r^_0 = rs (b - A x0) with the unscaled operator A (diag and A), p^ = 0, s^
// buffer 0 = 0.
template <typename T>
void launch_cg_init_r(hipStream_t s, const DevLevel& L, const SweepPlan& P, const FaceCoefs<T>& A, const T* diag,
                      const T* b, const T* x, const T* rs, const CgVecs<T>& v);
// Start, sweep 2: w^_0 = A^ r^_0; partials (r^, r^), (w^, r^), ||r_0||^2, ||b||^2 over
// the unknowns.
template <typename T>
void launch_cg_init_w(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<T>& Ah, const T* b,
                      const CgVecs<T>& v, double* part);
// The iteration sweep `it` (1, 2, ...) advances every problem from iterate it - 1 to
// iterate it: at its head the stopping test on iterate it - 1 (for it = 1 the start
// of the solve: ||r_0||, the threshold and the absolute floor), beta and alpha;
// then p^ = r^ + beta p^, s^ = w^ + beta s^, x += alpha rs p^, r^ -= alpha s^,
// w^ = A^ r^; partials (r^, r^), (w^, r^), ||r||^2 = sum (r^ / rs)^2 and
// max |x - x_old| / |x_old|.  x is the unscaled iterate, updated in place.
// t0 / t1 (optional): events that the launch itself records when the kernel
// starts and ends, so that they time the kernel alone.
template <typename T>
void launch_cg_sweep(hipStream_t s, const DevLevel& L, const SweepPlan& P, int it, const ScaledOp<T>& Ah,
                     const CgVecs<T>& v, T* x, PcgScalars* sc, double* part, hipEvent_t t0 = nullptr,
                     hipEvent_t t1 = nullptr);
void launch_check(hipStream_t s, const SweepPlan& P, int it_last, PcgScalars* sc, const double* part);
// Composite system: after a sweep that wrote w^ (buffer `buf` of v, iteration `it`,
// 0 for the start), w^ -= (scaled couplings to other levels) r^ for the listed rows,
// and partials of (that part of w^, r^) in part_if (ceil(n_if_rows / kBlock) of
// them); skipped once the problem stopped.
int interface_blocks(const DevLevel& L);
// val[e] = cif[src[e]] rs_row rs_col for the interface entries of every listed row
// (once per solve).
void launch_interface_values(hipStream_t s, const DevLevel& L, int n_entries, const double* cif, const double* rs,
                             double* val);
void launch_interface(hipStream_t s, const DevLevel& L, const double* r, double* w, const PcgScalars* sc,
                      double* part_if);
// All iterations of all problems in one cooperative launch (grid barrier between
// sweeps); bar is the control buffer (kBarWords), P.done_count = bar + kBarDone;
// its first kBarAbort words are zeroed before the launch.  Returns an error if the
// device cannot run the cooperative launch.  bar[kBarAbort] becomes 1 if a grid
// barrier timed out (the launch then returns early).
// Blocks of the persistent launch for this plan (0 if the device cannot run it);
// per_cu_cap > 0 limits the resident blocks per compute unit (fewer barrier arrivals).
template <typename T>
int persistent_blocks(const SweepPlan& P, int per_cu_cap);
template <typename T>
hipError_t launch_pcg_persistent(hipStream_t s, const DevLevel& L, const SweepPlan& P, int max_iter,
                                 const ScaledOp<T>& Ah, const CgVecs<T>& v, T* x, PcgScalars* sc, double* part,
                                 unsigned* bar, int per_cu_cap);
void launch_zero_u32(hipStream_t s, unsigned* p, int n);
// Copies count scalar records between device memory and the device-mapped view of
// pinned host memory (to_host: then makes the stores visible to the host), so that
// reading or setting the scalars costs one small kernel instead of a copy engine
// transfer.
void launch_copy_scalars(hipStream_t s, const PcgScalars* src, PcgScalars* dst, int count, bool to_host);
void launch_init_scalars(hipStream_t s, PcgScalars* sc, int n, double tol, double abs_floor, int max_iter,
                         int linf_test);
// The same with the scaled operator, staged in LDS, for solves without couplings to
// other levels.
void launch_true_residual(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<double>& Ah,
                          const double* b, const double* x, PcgScalars* sc, double* part);
void launch_true_residual(hipStream_t s, const DevLevel& L, const SweepPlan& P, const FaceCoefs<double>& A,
                          const double* diag, const double* b, const double* x, PcgScalars* sc,
                          double* part);
void launch_post_solve(hipStream_t s, const DevLevel& L, const SweepPlan& P, const double* E,
                       const double* rho, const CouplingParams& cp, double dt, double* T_out,
                       PcgScalars* sc, double* part);

// ------------------------------------------- mixed precision (FP32 inner solve)
// Outer sweep: x_new = x_old + d (d in FP32, may be null), r = b - A x_new in
// FP64 (applied as S^-1 A^ (S^-1 x_new) with the FP64 scaled operator Ah),
// r32 = (float) r; partials ||r||^2, ||b||^2 and the largest relative change of the
// last inner iteration (alpha of the inner record times rs32 p32, against the
// iterate before it); then the finisher applies the outer stopping test, the caps of
// max_outer sweeps and of the outer record's max_iter inner iterations, and prepares
// the inner scalars (an inner solve of a stopped problem is off from the start).
void launch_ir_sweep(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<double>& Ah,
                     const double* b, const double* x_old, const float* d, const float* p32,
                     const float* rs32, double* x_new, float* r32, const PcgScalars* outer,
                     const PcgScalars* inner, double* part);
void launch_ir_finish(hipStream_t s, const SweepPlan& P, int first, double inner_tol, int max_outer,
                      PcgScalars* outer, PcgScalars* inner, const double* part);
// Arrays and parameters of the whole mixed-precision solve in one persistent launch.
struct MixedArgs {
  ScaledOp<double> Ah;  // FP64 scaled operator of the refinement sweeps
  const double* b = nullptr;
  double* x = nullptr;      // iterate: x_0 on entry, the result on return
  double* x_alt = nullptr;  // second buffer of the refinement sweeps
  ScaledOp<float> Ah32;     // FP32 scaled operator of the inner solves
  CgVecs<float> v32;
  float *r32 = nullptr, *d32 = nullptr;
  PcgScalars* outer = nullptr;  // n_prob outer records (tol, abs_floor, max_iter, linf_test set)
  PcgScalars* inner = nullptr;  // n_prob inner records
  double* part = nullptr;
  unsigned* bar = nullptr;      // control buffer; its first kBarAbort words zeroed before the launch
  double inner_tol = 3e-3;
  int max_outer = 30;
  int inner_cap = 10000;        // bound of the inner loop (the records' max_iter never exceeds it)
  unsigned spin_limit = 1u << 26;
};
// Blocks of the mixed persistent launch for the plans of its FP64 refinement sweeps
// (P) and of its FP32 inner sweeps (P32: the same problems, at most as many blocks)
// (0 if the device cannot run it).
int mixed_persistent_blocks(const SweepPlan& P, const SweepPlan& P32, int per_cu_cap);
// P.done_count and P32.done_count must be M.bar + kBarDone.  Returns an error if the
// device cannot run the cooperative launch; bar[kBarAbort] becomes 1 if a grid
// barrier timed out.
hipError_t launch_mixed_persistent(hipStream_t s, const DevLevel& L, const SweepPlan& P, const SweepPlan& P32,
                                   const MixedArgs& M, int per_cu_cap);
// Inner start (one sweep): d = 0, r^ = rs r32, w^ = A^ r^ (the neighbours' r^
// formed from their r32 and rs); for a fresh start (inner cont = 0) p^ = 0 and s^
// buffer 0 = 0, for a continued one s^ is moved into buffer 0 and p^ kept; partials
// (r^, r^), (w^, r^), ||r32||^2 twice (the inner ||r_0|| and ||b||), laid out for
// P, the plan of the inner sweeps that follow.  Problems whose refinement has
// stopped are left alone.
void launch_inner_init(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<float>& Ah,
                       const float* r32, float* d, const CgVecs<float>& v, const PcgScalars* outer,
                       const PcgScalars* inner, double* part);

// ------------------------------------------------------------- batch layout
// dst[i] = src[prob(i)][idx[i]] (idx < 0: padding slot, dst = pad).
void launch_batch_gather(hipStream_t s, const DevLevel& L, const int32_t* idx, const double* const* src,
                         double pad, double* dst);
// out[out_off[prob(i)] + idx[i]] = src[i] for every real slot.
void launch_batch_scatter(hipStream_t s, const DevLevel& L, const int32_t* idx, const int64_t* out_off,
                          const double* src, double* out);

}  // namespace amrfld
