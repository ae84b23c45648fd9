/*
 * amrfld — level-by-level implicit diffusion solve for adaptive time-stepping
 * on oct-based AMR grids, on one AMD Instinct MI355X (gfx950).
 *
 * The method (Commercon, Debout & Teyssier 2014):
 *   - backward-Euler finite-volume update of dE/dt = div(K grad E) on the leaf
 *     cells of ONE level at a time (Sect. 3.1, eqs. Er_imp and Er_imp1):
 *       (1 + sum_f C_f) E_i^{n+1} - sum_f C_f E_nb^{n+1} = E_i^n,
 *     C_f = K_f dt / dx^2 for same-level and coarse-to-fine faces and
 *     (2/3) K_f dt / dx^2 for a face towards a coarser leaf (Sect. 3.1);
 *   - level-interface conditions (Sect. 3.2, 3.3): fine-to-coarse faces are
 *     Dirichlet with the coarse energy at the start of the coarse step;
 *     coarse-to-fine faces are Dirichlet (restricted fine energy), Neumann
 *     (stored fine flux, eq. mean_flux) or Robin (weight alpha);
 *   - Jacobi-preconditioned conjugate gradient with the L2-residual and
 *     L-infinity-change stopping test (Sect. 3.3.4);
 *   - adaptive time-stepping, finer levels first, dt_l = dt_{l-1} / nsub
 *     (Sect. 2.2);
 *   - Levermore-Pomraning limited diffusivity K = c lambda(R) / (rho kappa_R)
 *     and the linearised two-temperature coupling term (Sect. 2.1).
 *
 * Conventions for every call:
 *   - Every call returns an amrfld_status; nothing aborts or throws across the
 *     ABI.  amrfld_last_error() gives a message for the last failure.
 *   - Arguments are validated before any device work; on AMRFLD_E_INVALID no
 *     state has changed.  A level, batch layout or composite system whose
 *     allocation fails (AMRFLD_E_NOMEM) is not kept in part: the call can be
 *     made again.
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are ordinary CPU memory.  Caller buffers are borrowed for the
 *     duration of the call only.  The library owns its tables, fields and
 *     workspace (device memory, freed by amrfld_destroy).
 *   - Work is ordered on opts.stream (a hipStream_t, NULL = the null stream).
 *     Solve calls return after every kernel of the solve has finished
 *     (convergence is known on return; only the small kernel that handed the
 *     scalars to the host may still be retiring, which later work on the
 *     stream orders behind); set/get calls are stream-ordered.
 *   - A context is not thread-safe: one host thread at a time.
 *   - Per-cell arrays use the library's cell order for that level ("slot"
 *     order): octs sorted by Morton key of their coordinates, 8 cells per oct,
 *     x fastest within the oct.  amrfld_level_info returns the coordinates.
 */
#ifndef AMRFLD_H
#define AMRFLD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amrfld_ctx amrfld_ctx;

typedef enum {
  AMRFLD_OK = 0,
  AMRFLD_E_INVALID = -1,   /* bad argument, unbalanced hierarchy, wrong call order */
  AMRFLD_E_STATE = -2,     /* call not valid in the current state (e.g. no fields yet) */
  AMRFLD_E_NOMEM = -3,     /* device or host allocation failed */
  AMRFLD_E_DEVICE = -4,    /* a HIP runtime call failed */
  AMRFLD_E_NOCONV = -5,    /* PCG hit max_iter; E holds the last iterate */
  AMRFLD_E_NONFINITE = -6  /* NaN or Inf met in the residual of a solve; also a diagonal
                              entry <= 0 (the system is then not SPD and has no
                              Jacobi scaling) */
} amrfld_status;

typedef enum { AMRFLD_BC_DIRICHLET = 0, AMRFLD_BC_NEUMANN = 1, AMRFLD_BC_ROBIN = 2 } amrfld_bc;
/* AMRFLD_MIXED (not in the paper): FP32 operator, vectors and operator arithmetic with
 * FP64 dot products, inside an FP64 refinement loop that forms the true residual
 * b - A x and applies the solution update in FP64 and decides the stop with the
 * rule of Sect. 3.3.4 on that residual.  Between two refinement sweeps the FP32 CG
 * reduces its residual by inner_tol; after each sweep it continues from the new
 * residual with its search direction kept (residual replacement). */
typedef enum { AMRFLD_FP64 = 0, AMRFLD_MIXED = 1 } amrfld_precision;
typedef enum { AMRFLD_K_CONST = 0, AMRFLD_K_LP = 1, AMRFLD_K_MINERBO = 2, AMRFLD_K_POWER = 3 } amrfld_kmode;

typedef struct {
  int base_level;        /* coarsest level; it must cover the unit box */
  int max_level;         /* finest level that will be built (<= 20) */
  double robin_alpha;    /* Robin weight of the Dirichlet part, 0..1 (Sect. 3.2.3); default 0.5 */
  int max_iter;          /* PCG iteration cap, then AMRFLD_E_NOCONV; default 10000 */
  int precision;         /* amrfld_precision */
  int linf_test;         /* 1: also require max |dx|/|x| < tol (Sect. 3.3.4); default 1 */
  double abs_floor;      /* also converged when ||r|| <= abs_floor ||b||; default 1e-14 */
  double a_rad;          /* radiation constant of the coupling term; default 1 */
  double c_v;            /* specific heat of the coupling term; default 1 */
  int nsub[32];          /* substeps of level l per step of level l-1; 0 means 2 */
  int check_every;       /* PCG iterations between host convergence checks; 0 = auto */
  int true_residual;     /* 1: compute ||b - A x|| after each solve for the stats */
  int time_sweeps;       /* N > 0: time the sweep of every N-th CG iteration with HIP events */
  double inner_tol;      /* AMRFLD_MIXED: residual reduction of each FP32 inner CG segment between two
                            FP64 refinement sweeps; default 3e-3 */
  int max_outer;         /* AMRFLD_MIXED: refinement sweeps cap; default 30 */
  int max_blocks;        /* blocks per CG sweep (0 = 1024); each block sweeps a range of 256-slot tiles */
  int persistent;        /* 1 = all PCG iterations of a solve (batch form: of a step) in one cooperative
                            launch, where the device can run it; in AMRFLD_MIXED the whole refinement
                            loop with its inner solves, every decision made on the device; else
                            host-polled sweeps.  Results are the same bits either way */
  int graph;             /* with persistent: the batch form captures all its steps in one hipGraph;
                            amrfld_advance_subcycled captures one coarse step, all its level solves
                            each in one persistent launch, and replays it while dt, bc_mode, tol,
                            the context's parameters and its device buffers stay the same
                            (set_coeffs, set_launch and build_level force a new capture) */
  void* stream;          /* hipStream_t */
  int persistent_per_cu; /* persistent launch: resident blocks per compute unit (0 = as many as fit) */
  double theta;          /* time weighting of the level solves: 1 backward Euler (default), 1/2
                            Crank-Nicolson (Sect. 3.3.6); values in [1/2, 1]; theta < 1 requires
                            Dirichlet interfaces and no coupling term */
  double K_exp;          /* AMRFLD_K_POWER: K = K_const E^K_exp (the nonlinear equilibrium test,
                            Sect. 4.2); default 0 */
  int outer_mode[6];     /* faces of the unit box, in the order -x, +x, -y, +y, -z, +z: 0 no flux
                            (default), 1 Dirichlet; level solves and the unique time step only */
  double outer_value[6]; /* energy held at each Dirichlet face: the row of a cell on that face gets
                            C = 2 K_f dt / dx^2 (the value dx / 2 from the centre), K_f the harmonic
                            mean of the cell's K and the law's K at the held value (no gradient
                            there); the flux-limited gradient also takes the held value dx / 2 away */
  int form_coefs;        /* 1: the PCG sweeps form each face coefficient from the two cells'
                            diffusivities with the assembly's expression (the same bits) instead of
                            reading the three stored per cell (default 0): 15 fewer bytes per cell
                            and sweep for six divisions more (level solves and the batch form; the
                            unique time step always reads stored coefficients) */
} amrfld_opts;

typedef struct {
  int level, iters, converged, status;
  int64_t n_leaf;
  double rel_res;        /* ||r_j|| / ||r_0|| of the recursive residual */
  double true_rel_res;   /* ||b - A x|| / ||r_0|| (or -1 when not computed) */
  double linf_change;    /* max |x_j - x_{j-1}| / |x_{j-1}| of the last iteration */
  double min_E;          /* smallest leaf energy after the solve (negative energies, Sect. 3.3.5) */
  double ms;             /* device time of the whole solve (setup + PCG + post-solve) */
  double pcg_ms;         /* device time of the PCG iterations only */
  double dt;
  int outer_iters;       /* refinement sweeps (mixed precision), else 0 */
  int n_timed;           /* iterations whose sweeps were timed (time_sweeps), else 0 */
  double sweep_ms;       /* summed device time of the timed iteration sweeps (one per CG iteration) */
  double spare_ms;       /* 0: kept for the layout (the iteration is one fused sweep) */
  int launch_mode;       /* 0 host-polled sweeps, 1 persistent launch, 2 persistent launches in a hipGraph */
  double rnorm0;         /* ||r_0|| = ||b - A x_0|| (mixed precision: the first outer residual) */
  double bnorm;          /* ||b||; the stopping threshold is max(tol ||r_0||, abs_floor ||b||) */
  int sweep_blocks;      /* blocks (256-slot tile ranges) of every PCG sweep */
  int launch_blocks;     /* blocks of the launch that runs them (fewer for a persistent launch) */
} amrfld_stats;

/* Fill *o with the defaults listed above. */
void amrfld_default_opts(amrfld_opts* o);

/* Create a context for one hierarchy.  o->base_level >= 1, base <= max <= 20. */
amrfld_status amrfld_create(const amrfld_opts* o, amrfld_ctx** out);
void amrfld_destroy(amrfld_ctx* c);

/* Build level `level` from a HOST array of oct coordinates oct_ijk[n_oct][3]
 * (int32, each in [0, 2^(level-1))): the oct (I,J,K) holds cells (2I+a, 2J+b,
 * 2K+c) and its parent cell is (I,J,K) at level-1 (Fig. 1).  Levels are built
 * base first, then each next finer level.  The base level must list every oct
 * of the box.  Rejected with AMRFLD_E_INVALID: out-of-range or duplicate
 * octs, an oct whose parent cell is absent, and an oct whose parent has a face
 * neighbour position inside the box but absent at level-1 (the hierarchy must
 * keep face neighbours within one level, Sect. 3.1). */
amrfld_status amrfld_build_level(amrfld_ctx* c, int level, int64_t n_oct, const int32_t* oct_ijk);

/* Sizes of a built level: slots (8 per oct) and leaves (unrefined slots).
 * cell_ijk_out, if not NULL, is a HOST int32[n_slots][3] that receives the
 * cell coordinates in slot order. */
amrfld_status amrfld_level_info(const amrfld_ctx* c, int level, int64_t* n_slots, int64_t* n_leaf,
                                int32_t* cell_ijk_out);

/* Set the fields of a level from DEVICE float64 arrays of n_slots values in
 * slot order: density rho (> 0), radiative energy E (> 0 in LP mode) and gas
 * temperature T (NULL: no coupling term on this level).  Refined slots carry the
 * value used for their restricted cell until the next restriction replaces E.
 * kappa_R, kappa_P: opacities per unit mass; c_light: speed of light; kmode:
 * AMRFLD_K_CONST (K = K_const everywhere, the heat equation of Sect. 1),
 * AMRFLD_K_LP (K = c lambda(R) / (rho kappa_R) with the Levermore-Pomraning
 * limiter, Sect. 2.1), AMRFLD_K_MINERBO (the same with the Minerbo limiter of
 * the collapse runs, Sect. 5.1) or AMRFLD_K_POWER (K = K_const E^K_exp, K_exp from
 * the options, lagged at the start of each solve; E > 0 unless K_exp is an
 * integer).  The values are copied (stream-ordered) before return.  Arrays that are
 * not device memory are rejected with AMRFLD_E_INVALID. */
amrfld_status amrfld_set_coeffs(amrfld_ctx* c, int level, const double* rho, const double* E,
                                const double* T, double kappa_R, double kappa_P, double c_light,
                                int kmode, double K_const);

/* Advance level `level` alone by dt: assemble its system with the interface
 * rows of Sect. 3.2 (bc_mode for coarse-to-fine faces; fine-to-coarse faces are
 * always Dirichlet with the current coarse energy), solve with Jacobi PCG to
 * relative residual tol (Sect. 3.3.4), write the new leaf energies, add the
 * fine-to-coarse face energies to the parent level's flux register in Neumann /
 * Robin mode (eq. mean_flux) and clear this level's register.  With a
 * temperature the coupling term is included and T is updated.
 * Returns AMRFLD_E_NOCONV if max_iter was reached. */
amrfld_status amrfld_solve_level(amrfld_ctx* c, int level, double dt, int bc_mode, double tol);

/* For callers that cannot allocate device memory (tight serving loops, harnesses
 * that forbid hipMalloc): amrfld_solve_level with the same arguments, kernels,
 * results and stats, whose CG workspace (residual, operator products and search
 * direction vectors, block partials, scalar record, persistent-launch barrier words)
 * lives in a static device array of the library instead of context workspace.  It
 * makes no device allocation or free; the level's tables and fields come from
 * amrfld_build_level / amrfld_set_coeffs as usual.
 * Limits: a level of at most 2^20 slots (about 57 MB of scratch per device, held
 * from the first amrfld_create on that device until the process ends); FP64 only;
 * no sweep timing (opts.time_sweeps is ignored).
 * Errors: AMRFLD_E_INVALID for a larger level, AMRFLD_MIXED precision or bad
 * arguments (as amrfld_solve_level); AMRFLD_E_STATE when the context's device is
 * not current or when bc_mode is Neumann / Robin and the coarser level's flux
 * register does not exist yet (one amrfld_solve_level call in that mode creates
 * it); AMRFLD_E_DEVICE if the scratch array could not be located on this device.
 * Every call on one device uses that device's single array and leaves its contents
 * behind (each solve initialises what it reads): calls that overlap in time on one
 * device, from any context, stream or thread, race and must be serialised by the
 * caller. */
amrfld_status amrfld_solve_level_noalloc(amrfld_ctx* c, int level, double dt, int bc_mode, double tol);

/* Restrict level fine_level into level fine_level - 1: every refined cell of the
 * coarser level takes the mean of the energies of its 8 children, the coarse-to-fine
 * ghost value of Sect. 3.3.2 taken after the fine substeps (Sect. 2.2).
 * amrfld_advance_subcycled does this itself between levels; a caller that runs its
 * own schedule of amrfld_solve_level calls makes it where that schedule restricts.
 * Stream-ordered.  AMRFLD_E_INVALID: fine_level is the base level or not built;
 * AMRFLD_E_STATE: the fields of either level are not set. */
amrfld_status amrfld_restrict_level(amrfld_ctx* c, int fine_level);

/* One step dt_coarse of the base level with adaptive time-stepping (Sect. 2.2):
 * step(l, dt) = { nsub(l+1) x step(l+1, dt/nsub(l+1)); restrict l+1 into l;
 * solve_level(l, dt) }.  Returns the first non-OK status of its solves. */
amrfld_status amrfld_advance_subcycled(amrfld_ctx* c, double dt_coarse, int bc_mode, double tol);

/* One independent patch of the batch form: a box of n^3 cells of size dx whose
 * interior faces are same-level faces (eq. Er_imp1) and whose six boundary
 * faces carry the interface rows of Sect. 3.2 with a given outside energy and
 * inflow: Dirichlet diag += C, b += C ghost; Neumann b += flux; Robin
 * diag += alpha C, b += alpha C ghost + (1 - alpha) flux, with C = K_i dt / dx^2
 * (the ghost cell has the boundary cell's diffusivity) and alpha = robin_alpha.
 * rho and E are DEVICE float64 arrays of n^3 values, x fastest (index
 * i + n (j + n k)); they are read during the call only. */
typedef struct {
  int n;                 /* cells per axis: even, 2 <= n <= 1024 */
  double dx;             /* cell size */
  double dt;             /* backward-Euler step */
  const double* rho;
  const double* E;       /* energy at the start of the first step */
  int kmode;             /* amrfld_kmode */
  double K_const, kappa_R, c_light;
  int face_mode[6];      /* -x, +x, -y, +y, -z, +z: amrfld_bc */
  double face_ghost[6];  /* outside energy of Dirichlet / Robin faces */
  double face_flux[6];   /* inflow into each boundary cell per step, E units */
} amrfld_patch;

/* Advance n_prob independent patches by n_steps backward-Euler steps each, all
 * patches in the same sweeps: every PCG sweep covers the tiles of all patches,
 * with per-patch reductions, scalars and convergence (a converged patch's
 * blocks return at once).  precision: AMRFLD_FP64 or AMRFLD_MIXED; tol as in
 * amrfld_solve_level.  E_out: DEVICE float64 array receiving the final energies
 * of all patches concatenated in patch order (sum of n^3 values, x fastest),
 * written by a kernel enqueued on opts.stream before return (stream-ordered).
 * Patch fields or E_out that are not device memory are rejected with
 * AMRFLD_E_INVALID before any launch.
 * Stats: one entry per (step, patch), the patch index in the `level` field.
 * The batch layout is kept in the context and reused while the sizes repeat. */
amrfld_status amrfld_solve_batch(amrfld_ctx* c, int n_prob, const amrfld_patch* patches, int n_steps,
                                 double tol, int precision, double* E_out);

/* Advance every level by dt_coarse with one time step shared by all levels, the
 * finest level's: the unique-time-step method the paper compares its adaptive one
 * with (Sect. 1; coefficients of the remark closing Sect. 3.1).  n = product over
 * the finer levels of nsub composite solves of dt_coarse / n, each a Jacobi-PCG over
 * the leaves of all levels coupled in one system: same-level faces A, a face
 * towards a coarser leaf (2/3) A, a face shared with a refined neighbour coupled to
 * each of its four finer cells with 2^(3-ndim) A / 3; every row is multiplied by
 * its cell volume, which makes the matrix symmetric (and the total energy exactly
 * conserved with zero-flux outer faces).  After each solve T is updated and the
 * finer levels are restricted into their parents.  Runs in FP64 with host-polled
 * sweeps whatever opts.precision and opts.persistent say; no flux registers are
 * involved.  Stats: one entry per composite solve, with level = -1.  Errors: as
 * amrfld_advance_subcycled; E_STATE when T is set on some levels only. */
amrfld_status amrfld_advance_unique(amrfld_ctx* c, double dt_coarse, double tol);

/* Copy a level's E (and T when T_out is not NULL) to DEVICE arrays of n_slots
 * float64 in slot order (stream-ordered); other memory is rejected with
 * AMRFLD_E_INVALID. */
amrfld_status amrfld_get_E(const amrfld_ctx* c, int level, double* E_out, double* T_out);

/* Stats of the solves made by the last solve / advance / batch call, in order.
 * Writes min(max_n, count) entries to out and the count to *n. */
amrfld_status amrfld_last_stats(const amrfld_ctx* c, amrfld_stats* out, int max_n, int* n);

/* Launch shape of the PCG sweeps for the following calls on this context; not a
 * step of the method (the same sweeps, dealt differently to the GPU), used to
 * time candidate shapes on the device.  max_blocks: blocks per sweep (0 = 1024;
 * each block sweeps a contiguous range of at most 16 tiles of 256 slots, or 32 in
 * the FP32 inner sweeps of an AMRFLD_MIXED level solve, which may then take fewer
 * blocks than its FP64 sweeps);
 * persistent, persistent_per_cu, form_coefs: as in amrfld_opts.  Negative values
 * are rejected with AMRFLD_E_INVALID and change nothing.  Results of one shape are
 * bitwise reproducible, and form_coefs changes no FP64 bit; between block counts
 * the block partials are summed in other groupings, so they may differ in the
 * last bits. */
amrfld_status amrfld_set_launch(amrfld_ctx* c, int max_blocks, int persistent, int persistent_per_cu,
                                int form_coefs);

/* Inner tolerance and refinement-sweep cap of the AMRFLD_MIXED form for the
 * following calls (as amrfld_opts.inner_tol and max_outer); not a step of the
 * method: every result still meets the FP64 stopping rule, only the split of the
 * work between FP32 inner iterations and FP64 refinement sweeps changes, and the
 * best split depends on the workload (the autotuner times it).  inner_tol outside
 * (0, 1) or max_outer < 1: AMRFLD_E_INVALID, nothing changes. */
amrfld_status amrfld_set_refinement(amrfld_ctx* c, double inner_tol, int max_outer);

/* Message of the last failure on this context ("" if none). */
const char* amrfld_last_error(const amrfld_ctx* c);

/* Message of the calling thread's last failure of amrfld_create (no context exists
   then); valid until that thread's next amrfld_create. */
const char* amrfld_create_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AMRFLD_H */
