// C ABI of the level solve: context, hierarchy tables, fields, the per-level
// solve (assembly + Jacobi PCG + post-solve) and the adaptive time-stepping
// driver (Sect. 2.2, Sect. 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/amrfld.h"
#include "device.h"
#include "signal.h"
#include "tables.h"

using namespace amrfld;

namespace {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct NoMem : std::runtime_error {
  using std::runtime_error::runtime_error;
};

void check(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) throw NoMem(std::string(what) + ": out of device memory");
  if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

// Counts device allocations and frees: a captured graph holds raw pointers, so it
// is replayed only while this count is the one it was captured at.
std::atomic<uint64_t> g_alloc_epoch{0};

// Set while the no-allocation solve runs on this thread: any device allocation or
// free reached from it is a library bug, reported as an error instead of made.
thread_local bool g_no_alloc = false;

template <class T>
T* dalloc(int64_t n, const char* what) {
  if (g_no_alloc) throw std::logic_error(std::string(what) + ": device allocation in the no-allocation solve");
  void* p = nullptr;
  if (n <= 0) n = 1;
  check(hipMalloc(&p, size_t(n) * sizeof(T)), what);
  g_alloc_epoch.fetch_add(1);
  return static_cast<T*>(p);
}

void dfree(void* p) {
  if (p) {
    if (g_no_alloc) throw std::logic_error("device free in the no-allocation solve");
    (void)hipFree(p);
    g_alloc_epoch.fetch_add(1);
  }
}

// ----------------------------------------------------------- static scratch
// Workspace of amrfld_solve_level_noalloc in a file-scope device array, for callers
// that cannot allocate device memory: the CG vectors (r^, w^, s^ in two buffers each
// and p^) of up to kScratchSlots slots, the block partials of that many slots'
// sweeps, one scalar record and the barrier words of the persistent launch.  Every sub-buffer starts on
// a 256-byte boundary.  Each device holds its own copy for the life of the process.
constexpr int64_t kScratchSlots = int64_t(1) << 20;
constexpr int kScratchVectors = 7;  // r^, w^, s^ (two buffers each) and p^
constexpr int64_t kScratchPartials = 8 * ((kScratchSlots + kBlock - 1) / kBlock);
constexpr int64_t kScratchScalarDoubles = 32;            // one PcgScalars, padded to 256 B
constexpr int64_t kScratchBarDoubles = kBarWords / 2;    // kBarWords unsigned words
constexpr int64_t kScratchOffPartials = kScratchVectors * kScratchSlots;
constexpr int64_t kScratchOffScalars = kScratchOffPartials + kScratchPartials;
constexpr int64_t kScratchOffBar = kScratchOffScalars + kScratchScalarDoubles;
constexpr int64_t kScratchDoubles = kScratchOffBar + kScratchBarDoubles;
static_assert(sizeof(PcgScalars) <= kScratchScalarDoubles * sizeof(double), "scalar record fits its slot");
static_assert(kScratchSlots % 32 == 0 && kScratchPartials % 32 == 0, "sub-buffers stay 256-byte aligned");

static __device__ __align__(256) double scratch[kScratchDoubles];

// The device address of `scratch` on each device, taken once per device with that
// device current (in host code the array's name is no device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

void resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_done[dev]) return;
  double* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
  g_scratch_err[dev] = e;
  g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
  if (e != hipSuccess) (void)hipGetLastError();
  g_scratch_done[dev] = true;
}

double* scratch_of(int dev, std::string* why) {
  if (dev < 0 || dev >= kMaxDevices) {
    *why = "device index out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    *why = "the device scratch was not set up on this device (create the context with it current)";
    return nullptr;
  }
  if (!g_scratch_ptr[dev]) *why = std::string("device scratch: ") + hipGetErrorString(g_scratch_err[dev]);
  return g_scratch_ptr[dev];
}

struct LevelState {
  LevelTables t;
  int32_t *nbr = nullptr, *cnb = nullptr, *parent = nullptr, *child = nullptr;
  bool tables_uploaded = false, child_dirty = true;
  double *rho = nullptr, *E = nullptr, *T = nullptr, *K = nullptr;
  double *Cp = nullptr, *diag = nullptr, *b = nullptr, *reg = nullptr;
  double *Ch = nullptr, *rs = nullptr;  // the Jacobi-scaled operator of the current solve
  uint8_t* mask = nullptr;  // per slot: faces that couple two leaves of the level
  int last_iters = 0;       // CG iterations of the level's last FP64 solve (first batch of the next)
  bool has_fields = false, has_T = false;
  int kmode = 1;
  double K_const = 1.0, kappa_R = 1.0, kappa_P = 1.0, c_light = 1.0, K_exp = 0.0;

  DevLevel dev() const {
    DevLevel d;
    d.n_slots = int(t.n_slots());
    d.n_oct = int(t.n_oct);
    d.nbr = nbr;
    d.cnb = cnb;
    d.child = child;
    d.parent = parent;
    d.dx = 1.0 / double(int64_t(1) << t.level);
    d.vol = d.dx * d.dx * d.dx;
    d.oct_prob = nullptr;
    d.pp = nullptr;
    return d;
  }
  void release() {
    for (void* p : {(void*)nbr, (void*)cnb, (void*)parent, (void*)child, (void*)rho, (void*)E,
                    (void*)T, (void*)K, (void*)Cp, (void*)diag, (void*)b, (void*)reg, (void*)mask, (void*)Ch,
                    (void*)rs})
      dfree(p);
    nbr = cnb = parent = child = nullptr;
    rho = E = T = K = Cp = diag = b = reg = Ch = rs = nullptr;
    mask = nullptr;
    tables_uploaded = false;
  }
};

thread_local std::string g_create_error;  // the calling thread's last amrfld_create failure

}  // namespace

// Concatenated slot layout of a batch of patches (cached while the sizes repeat).
struct BatchState {
  std::vector<int> sizes;
  int n_prob = 0;
  int64_t n_slots = 0, n_oct = 0;
  int G = 0, tpb_max = 1;
  std::vector<int64_t> out_off;  // host copy: first output value of each patch
  int32_t *nbr = nullptr, *cnb = nullptr, *child = nullptr, *oct_prob = nullptr, *idx = nullptr;
  int32_t *blk_prob = nullptr, *blk0 = nullptr, *tile0 = nullptr;
  int64_t* d_out_off = nullptr;
  double *E = nullptr, *rho = nullptr, *K = nullptr, *Cp = nullptr, *diag = nullptr, *b = nullptr;
  double *Ch = nullptr, *rs = nullptr;  // the Jacobi-scaled operator of the current step
  uint8_t* mask = nullptr;
  PatchParams* pp = nullptr;
  const double** src = nullptr;  // device array of n_prob pointers

  void release() {
    for (void* p : {(void*)nbr, (void*)cnb, (void*)child, (void*)oct_prob, (void*)idx, (void*)blk_prob,
                    (void*)blk0, (void*)tile0, (void*)d_out_off, (void*)E, (void*)rho, (void*)K, (void*)Cp,
                    (void*)diag, (void*)b, (void*)pp, (void*)src, (void*)mask, (void*)Ch, (void*)rs})
      dfree(p);
    nbr = cnb = child = oct_prob = idx = blk_prob = blk0 = tile0 = nullptr;
    d_out_off = nullptr;
    E = rho = K = Cp = diag = b = Ch = rs = nullptr;
    mask = nullptr;
    pp = nullptr;
    src = nullptr;
  }
  DevLevel dev() const {
    DevLevel d;
    d.n_slots = int(n_slots);
    d.n_oct = int(n_oct);
    d.nbr = nbr;
    d.cnb = cnb;
    d.child = child;
    d.parent = nullptr;
    d.dx = 1.0;
    d.vol = 1.0;
    d.oct_prob = oct_prob;
    d.pp = pp;
    return d;
  }
  SweepPlan plan() const {
    SweepPlan p;
    p.n_prob = n_prob;
    p.G = G;
    p.n_tiles = tiles_of(n_slots);
    p.tpb_max = tpb_max;
    p.blk_prob = blk_prob;
    p.blk0 = blk0;
    p.tile0 = tile0;
    p.done_count = nullptr;
    return p;
  }
};

// One coarse step of the subcycled driver captured as a graph (FP64, persistent
// solves), replayed while its parameters and every device buffer stay the same.
struct StepGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  double dt = 0.0, tol = 0.0;
  int mode = -1;
  uint64_t alloc_epoch = 0, param_epoch = 0;
  void reset() {
    if (ex) (void)hipGraphExecDestroy(ex);
    if (g) (void)hipGraphDestroy(g);
    ex = nullptr;
    g = nullptr;
    mode = -1;
  }
};

struct amrfld_ctx {
  amrfld_opts o{};
  std::string err;
  int device = 0;  // current device when the context was created
  uint64_t param_epoch = 0;  // bumped by every call that changes what a captured step bakes in
  StepGraph step_graph;
  int finest = -1;
  std::vector<LevelState> lev;  // index: level - base
  int64_t ws_n = 0;
  CgVecs<double> cg;  // the CG vectors of the largest solve so far
  double* partials = nullptr;
  int64_t partial_n = 0;
  // mixed-precision workspace: FP32 scaled operator, outer residual, inner iterate
  // and CG vectors; second buffer of the FP64 refinement sweeps
  int64_t ws32_n = 0;
  float *Ch32 = nullptr, *K32 = nullptr, *rs32 = nullptr, *r32 = nullptr, *d32 = nullptr;
  CgVecs<float> cg32;
  double* x_alt = nullptr;
  PcgScalars* sc = nullptr;     // [2 sc_cap]: outer (or plain) solves, then inner solves
  PcgScalars* h_sc = nullptr;   // pinned mirror
  PcgScalars* h_sc_dev = nullptr;  // the mirror as the device addresses it
  int sc_cap = 0;
  uint64_t* h_seq = nullptr;      // pinned completion word of scalar reads
  uint64_t* h_seq_dev = nullptr;  // the word as the device addresses it
  uint64_t seq = 0;               // value of the last scalar read
  struct BatchState* batch = nullptr;
  struct CompositeState* comp = nullptr;  // unique-time-step system of all levels (built on first use)
  unsigned* bar = nullptr;  // grid barrier counter, generation, done counter, abort flag
  hipStream_t cap_stream = nullptr;  // library stream for graph capture (default priority)
  hipEvent_t cap_ev[2] = {nullptr, nullptr};
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> sweep_ev;  // 4 per iteration when sweeps are timed
  std::vector<amrfld_stats> stats;

  hipStream_t stream() const { return static_cast<hipStream_t>(o.stream); }
  LevelState& L(int level) { return lev[level - o.base_level]; }
  const LevelState& L(int level) const { return lev[level - o.base_level]; }
  int nsub(int level) const {
    const int v = (level >= 0 && level < 32) ? o.nsub[level] : 0;
    return v > 0 ? v : 2;
  }
};

namespace {

// Caller arrays that a kernel reads or writes must be device memory (a host
// pointer would fault in the kernel): checked before any launch.
bool device_ptr(const void* p) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

amrfld_status fail(amrfld_ctx* c, amrfld_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

template <class F>
amrfld_status guarded(amrfld_ctx* c, F&& f) {
  try {
    return f();
  } catch (const NoMem& e) {
    return fail(c, AMRFLD_E_NOMEM, e.what());
  } catch (const HipError& e) {
    return fail(c, AMRFLD_E_DEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(c, AMRFLD_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, AMRFLD_E_INVALID, e.what());
  }
}

template <typename T>
void free_vecs(CgVecs<T>& v) {
  for (T* p : {v.r[0], v.r[1], v.w[0], v.w[1], v.s[0], v.s[1], v.p}) dfree(p);
  v = CgVecs<T>{};
}

template <typename T>
void alloc_vecs(CgVecs<T>& v, int64_t n, const char* what) {
  for (T** p : {&v.r[0], &v.r[1], &v.w[0], &v.w[1], &v.s[0], &v.s[1], &v.p}) *p = dalloc<T>(n, what);
}

void ensure_workspace(amrfld_ctx* c, int64_t n) {
  if (n > c->ws_n) {
    free_vecs(c->cg);
    c->ws_n = 0;
    alloc_vecs(c->cg, n, "workspace");
    c->ws_n = n;
  }
  // 4 partials per block and iteration parity
  const int64_t g = int64_t(tiles_of(n)) * 8;
  if (g > c->partial_n) {
    dfree(c->partials);
    c->partials = nullptr;
    c->partial_n = 0;
    c->partials = dalloc<double>(g, "partials");
    c->partial_n = g;
  }
}

void ensure_workspace32(amrfld_ctx* c, int64_t n) {
  if (n <= c->ws32_n) return;
  for (void* p : {(void*)c->Ch32, (void*)c->K32, (void*)c->rs32, (void*)c->r32, (void*)c->d32, (void*)c->x_alt})
    dfree(p);
  free_vecs(c->cg32);
  c->Ch32 = c->K32 = c->rs32 = c->r32 = c->d32 = nullptr;
  c->x_alt = nullptr;
  c->ws32_n = 0;
  c->Ch32 = dalloc<float>(3 * n, "workspace fp32");
  c->K32 = dalloc<float>(n, "workspace fp32");
  c->rs32 = dalloc<float>(n, "workspace fp32");
  c->r32 = dalloc<float>(n, "workspace fp32");
  c->d32 = dalloc<float>(n, "workspace fp32");
  alloc_vecs(c->cg32, n, "workspace fp32");
  c->x_alt = dalloc<double>(n, "workspace x");
  c->ws32_n = n;
}

// The level's device tables: allocated all together (a failed allocation leaves
// none), copied until one upload has succeeded.
void upload_tables(amrfld_ctx* c, LevelState& L) {
  const hipStream_t s = c->stream();
  const int64_t n_oct = L.t.n_oct;
  if (!L.nbr) {
    int32_t *nbr = nullptr, *cnb = nullptr, *parent = nullptr, *child = nullptr;
    try {
      nbr = dalloc<int32_t>(6 * n_oct, "tables");
      cnb = dalloc<int32_t>(6 * n_oct, "tables");
      parent = dalloc<int32_t>(n_oct, "tables");
      child = dalloc<int32_t>(8 * n_oct, "tables");
    } catch (...) {
      for (void* p : {(void*)nbr, (void*)cnb, (void*)parent, (void*)child}) dfree(p);
      throw;
    }
    L.nbr = nbr;
    L.cnb = cnb;
    L.parent = parent;
    L.child = child;
    L.tables_uploaded = false;
    L.child_dirty = true;
  }
  if (!L.tables_uploaded) {
    check(hipMemcpyAsync(L.nbr, L.t.nbr.data(), 6 * n_oct * 4, hipMemcpyHostToDevice, s), "upload");
    check(hipMemcpyAsync(L.cnb, L.t.cnb.data(), 6 * n_oct * 4, hipMemcpyHostToDevice, s), "upload");
    check(hipMemcpyAsync(L.parent, L.t.parent.data(), n_oct * 4, hipMemcpyHostToDevice, s), "upload");
    L.tables_uploaded = true;
  }
  if (L.child_dirty) {
    check(hipMemcpyAsync(L.child, L.t.child.data(), 8 * L.t.n_oct * 4, hipMemcpyHostToDevice, s),
          "upload");
    check(hipStreamSynchronize(s), "upload");
    L.child_dirty = false;
  }
}

CellKParams kparams(const LevelState& L) {
  CellKParams k;
  k.kmode = L.kmode;
  k.K_const = L.K_const;
  k.kappa_R = L.kappa_R;
  k.c_light = L.c_light;
  k.K_exp = L.K_exp;
  return k;
}

// The operator's face coefficients as the sweeps read them: stored, or formed
// from K and the face mask (scale = dt / dx^2, or per problem from the batch table).
FaceCoefs<double> face_coefs(const amrfld_ctx* c, const double* Cp, const double* K, const uint8_t* mask,
                             double scale, double theta, bool per_problem) {
  FaceCoefs<double> A;
  if (!c->o.form_coefs) {
    A.Cp = Cp;
    return A;
  }
  A.K = K;
  A.mask = mask;
  A.scale = scale;
  A.theta = theta;
  A.per_problem = per_problem;
  return A;
}

FaceCoefs<double> stored_face_coefs(const double* Cp) {
  FaceCoefs<double> A;
  A.Cp = Cp;
  return A;
}

OuterBC outer_bc(const amrfld_ctx* c) {
  OuterBC b;
  for (int d = 0; d < 6; ++d)
    if (c->o.outer_mode[d] == 1) {
      b.mask |= 1u << d;
      b.val[d] = c->o.outer_value[d];
    }
  return b;
}

CouplingParams cparams(const amrfld_ctx* c, const LevelState& L) {
  CouplingParams p;
  p.T = L.has_T ? L.T : nullptr;
  p.kappa_P = L.kappa_P;
  p.c_light = L.c_light;
  p.a_rad = c->o.a_rad;
  p.c_v = c->o.c_v;
  return p;
}

double* ensure_reg(amrfld_ctx* c, LevelState& L) {
  if (!L.reg) {
    const int64_t n = 6 * L.t.n_slots();
    L.reg = dalloc<double>(n, "flux register");
    launch_fill(c->stream(), L.reg, n, 0.0);
  }
  return L.reg;
}

// The theta-weighted step is defined for Dirichlet interfaces and no coupling term
// (the stored flux and the temperature update assume backward Euler).
amrfld_status check_theta(amrfld_ctx* c, int bc_mode) {
  if (c->o.theta == 1.0) return AMRFLD_OK;
  if (bc_mode != AMRFLD_BC_DIRICHLET)
    return fail(c, AMRFLD_E_INVALID, "theta < 1 requires Dirichlet interfaces");
  for (const LevelState& L : c->lev)
    if (L.has_T) return fail(c, AMRFLD_E_INVALID, "theta < 1 is not defined with the coupling term");
  return AMRFLD_OK;
}

amrfld_status check_level_ready(amrfld_ctx* c, int level) {
  if (level < c->o.base_level || level > c->finest)
    return fail(c, AMRFLD_E_INVALID, "level not built");
  if (!c->L(level).has_fields) return fail(c, AMRFLD_E_STATE, "fields of the level not set");
  for (int l = level - 1; l >= std::max(c->o.base_level, level - 2); --l)
    if (!c->L(l).has_fields) return fail(c, AMRFLD_E_STATE, "fields of a coarser level not set");
  return AMRFLD_OK;
}

struct LoopStats {
  std::vector<int> iters;  // per problem: PCG iterations (inner iterations in mixed precision)
  int n_timed = 0;
  double sweep_ms = 0.0;
  bool persistent = false;  // iterations ran in persistent launches
  int launch_blocks = 0;    // blocks of those launches
};

void ensure_scalars(amrfld_ctx* c, int n_prob) {
  if (n_prob <= c->sc_cap) return;
  dfree(c->sc);
  if (c->h_sc) (void)hipHostFree(c->h_sc);
  c->sc = nullptr;
  c->h_sc = nullptr;
  c->h_sc_dev = nullptr;
  c->sc_cap = 0;
  c->sc = dalloc<PcgScalars>(2 * int64_t(n_prob), "scalars");
  check(hipHostMalloc(reinterpret_cast<void**>(&c->h_sc), 2 * size_t(n_prob) * sizeof(PcgScalars),
                      hipHostMallocMapped | hipHostMallocCoherent),
        "pinned scalars");
  check(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->h_sc_dev), c->h_sc, 0), "mapped scalars");
  c->sc_cap = n_prob;
  if (!c->h_seq) {
    uint64_t* w = nullptr;
    check(hipHostMalloc(reinterpret_cast<void**>(&w), 64, hipHostMallocMapped | hipHostMallocCoherent),
          "pinned completion word");
    *w = c->seq;
    uint64_t* wd = nullptr;
    const hipError_t e = hipHostGetDevicePointer(reinterpret_cast<void**>(&wd), w, 0);
    if (e != hipSuccess) (void)hipHostFree(w);
    check(e, "mapped completion word");
    c->h_seq = w;
    c->h_seq_dev = wd;
  }
}

// The device view of a slice of the pinned mirror, or nullptr outside it.
PcgScalars* mapped(amrfld_ctx* c, const PcgScalars* host, int count) {
  if (!c->h_sc_dev || host < c->h_sc || host + count > c->h_sc + 2 * int64_t(c->sc_cap)) return nullptr;
  return c->h_sc_dev + (host - c->h_sc);
}

// Brings count scalar records from the device to the host and waits for them.  Into
// the pinned mirror, a one-block kernel copies them and then stores a new value to a
// pinned completion word, which the host reads in a loop: the wait ends as soon as
// the word lands, where a blocking stream wait adds the thread's wake-up to every
// convergence check.  After 50 ms of polling the host blocks on the stream instead.  Every kernel before the copy has
// finished on return; the copy kernel itself may still be retiring.
void read_scalars(amrfld_ctx* c, PcgScalars* host, const PcgScalars* dev, int count) {
  const hipStream_t s = c->stream();
  PcgScalars* m = mapped(c, host, count);
  if (!m || !c->h_seq) {
    check(hipMemcpyAsync(host, dev, count * sizeof(PcgScalars), hipMemcpyDeviceToHost, s), "scalars");
    check(hipStreamSynchronize(s), "sync");
    return;
  }
  static_assert(sizeof(PcgScalars) % 8 == 0, "scalar records are copied as 8-byte words");
  const uint64_t want = ++c->seq;
  launch_scalars_to_host(s, dev, m, count * int(sizeof(PcgScalars) / 8), c->h_seq_dev, want);
  check(hipGetLastError(), "scalars");
  const auto t0 = std::chrono::steady_clock::now();
  while (__atomic_load_n(c->h_seq, __ATOMIC_ACQUIRE) != want) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
      check(hipStreamSynchronize(s), "sync");
      if (__atomic_load_n(c->h_seq, __ATOMIC_ACQUIRE) != want)
        throw HipError("scalars: completion word not written by a finished stream");
      break;
    }
    __builtin_ia32_pause();
  }
}

bool all_done(const PcgScalars* h, int n) {
  for (int q = 0; q < n; ++q)
    if (!h[q].done) return false;
  return true;
}

// Iterations of the CG solves of all problems of a plan, whose start sweeps
// already ran: batches of iteration sweeps, a stopping check after each batch, the
// next batch size predicted from the slowest problem's observed convergence rate.
// Launches after a problem converged return at once.  Returns the largest
// iteration count of the problems' solves (0: every problem was already stopped).
// first_chunk > 0: size of the first batch (a prediction, e.g. the previous inner
// solve's count), else the default.  lead: records stored just before sc_dev (and
// sc_host) that every check also brings to the host (the outer records of the mixed
// form).
template <typename T>
int pcg_iterations(amrfld_ctx* c, const DevLevel& D, const SweepPlan& P, const ScaledOp<T>& Ah,
                   const CgVecs<T>& v, T* x, PcgScalars* sc_dev, PcgScalars* sc_host, int max_iter, LoopStats* ls,
                   int first_chunk = 0, int lead = 0) {
  const hipStream_t s = c->stream();
  const int np = P.n_prob;
  if (c->o.persistent && !D.cif) {
    // all iterations in one cooperative launch, when the device can run it
    const int per_cu = c->o.persistent_per_cu;
    if (!c->bar) c->bar = dalloc<unsigned>(kBarWords, "barrier");
    SweepPlan Pp = P;
    Pp.done_count = c->bar + kBarDone;
    const int blocks = persistent_blocks<T>(Pp, per_cu);
    if (blocks > 0) {
      launch_zero_u32(s, c->bar, kBarWords);
      const hipError_t e = launch_pcg_persistent<T>(s, D, Pp, max_iter, Ah, v, x, sc_dev, c->partials, c->bar, per_cu);
      if (e == hipSuccess) {
        read_scalars(c, sc_host, sc_dev, np);
        unsigned aborted = 0;
        check(hipMemcpy(&aborted, c->bar + kBarAbort, sizeof(unsigned), hipMemcpyDeviceToHost), "abort flag");
        if (aborted) throw std::runtime_error("persistent sweep: a grid barrier timed out");
        int max_done = 0;
        for (int qq = 0; qq < np; ++qq) {
          ls->iters[qq] += sc_host[qq].iter;
          max_done = std::max(max_done, sc_host[qq].iter);
        }
        ls->persistent = true;
        ls->launch_blocks = blocks;
        return max_done;
      }
      (void)hipGetLastError();  // not launchable here: poll instead
    }
  }
  int launched = 0;
  int chunk = c->o.check_every > 0 ? c->o.check_every : (first_chunk > 0 ? std::min(first_chunk, 256) : 8);
  const bool autochunk = c->o.check_every <= 0;
  const int period = c->o.time_sweeps;
  // the first batch is enqueued behind the start sweeps without waiting for them: a
  // problem they already stopped makes its launches return at once, and the host
  // copy of the scalars is only read after a batch
  bool first = true;
  while ((first || !all_done(sc_host, np)) && launched < max_iter) {
    first = false;
    // sweep it makes iterate it; the check after the last one tests iterate max_iter
    const int k = std::min(chunk, max_iter - launched);
    if (period > 0) {
      while (int(c->sweep_ev.size()) < 2 * ((launched + k) / period + 1)) {
        hipEvent_t e;
        check(hipEventCreate(&e), "event");
        c->sweep_ev.push_back(e);
      }
    }
    for (int t = 0; t < k; ++t) {
      const int it = launched + t + 1;
      // every period-th iteration: the sweep's launch records its own start and end
      hipEvent_t* e = (period > 0 && it % period == 0) ? &c->sweep_ev[2 * (it / period - 1)] : nullptr;
      launch_cg_sweep<T>(s, D, P, it, Ah, v, x, sc_dev, c->partials, e ? e[0] : nullptr, e ? e[1] : nullptr);
      if constexpr (std::is_same<T, double>::value) {
        if (D.n_if_rows > 0) launch_interface(s, D, v.r[it & 1], v.w[it & 1], sc_dev, D.if_part);
      }
    }
    launched += k;
    launch_check(s, P, launched, sc_dev, c->partials);
    check(hipGetLastError(), "launch");
    read_scalars(c, sc_host - lead, sc_dev - lead, np + lead);
    if (autochunk && !all_done(sc_host, np)) {
      int est = 2;
      for (int qq = 0; qq < np; ++qq) {
        const PcgScalars& h = sc_host[qq];
        if (h.done) continue;
        const double ratio = h.rnorm0 > 0 ? h.rnorm / h.rnorm0 : 1.0;
        int e = 2 * chunk;
        if (h.iter > 0 && ratio > 0 && ratio < 1 && h.rnorm > h.thresh) {
          const double rate = std::log(ratio) / h.iter;  // log reduction per iteration (< 0)
          e = int(std::ceil(std::log(h.thresh / h.rnorm) / rate)) + 1;
        }
        est = std::max(est, e);
      }
      chunk = std::max(2, std::min(256, est));
    }
  }
  int max_done = 0;
  for (int qq = 0; qq < np; ++qq) {
    ls->iters[qq] += sc_host[qq].iter;
    max_done = std::max(max_done, sc_host[qq].iter);
  }
  if (period > 0) {
    // timed sweeps that did work for at least one problem (sweep it makes iterate it)
    for (int it = period; it <= max_done && 2 * (it / period) <= int(c->sweep_ev.size()); it += period) {
      const int kk = it / period - 1;
      float ta = 0.f;
      check(hipEventSynchronize(c->sweep_ev[2 * kk + 1]), "event");
      check(hipEventElapsedTime(&ta, c->sweep_ev[2 * kk], c->sweep_ev[2 * kk + 1]), "event");
      ls->sweep_ms += ta;
      ls->n_timed += 1;
    }
  }
  return max_done;
}

PcgScalars make_scalars(double tol, double abs_floor, int max_iter, int linf_test) {
  PcgScalars init{};
  init.tol = tol;
  init.abs_floor = abs_floor;
  init.max_iter = max_iter;
  init.linf_test = linf_test;
  return init;
}

// Operator arrays of one solve (a level or a whole batch), slot order: the
// unscaled operator (diag and A, stored or formed face coefficients) and the
// Jacobi-scaled one the CG sweeps read.
struct SolveArrays {
  FaceCoefs<double> A;
  const double* diag;
  const double* b;
  double* x;  // x_0 on entry (the energy, updated in place)
  int64_t n;
  ScaledOp<double> Ah;
};

// The Jacobi-scaled operator of a solve: rs (and the stored scaled coefficients
// unless they are formed in the sweeps) computed from the assembled system on s.
ScaledOp<double> scale_operator(amrfld_ctx* c, hipStream_t s, const DevLevel& D, const FaceCoefs<double>& A,
                                const double* Cp, const double* diag, double* rs, double* Ch) {
  launch_jacobi_scale(s, D, A.Cp ? Cp : nullptr, diag, rs, Ch);
  ScaledOp<double> Ah;
  Ah.rs = rs;
  if (A.Cp) {
    Ah.Ch = Ch;
  } else {
    Ah.K = A.K;
    Ah.mask = A.mask;
    Ah.scale = A.scale;
    Ah.theta = A.theta;
    Ah.per_problem = A.per_problem;
  }
  return Ah;
}

// The FP32 copy of a solve's scaled operator (launched on s into the FP32
// workspace) as the inner sweeps read it.
ScaledOp<float> operator_f32(amrfld_ctx* c, hipStream_t s, const SolveArrays& A) {
  ensure_workspace32(c, A.n);
  launch_to_f32(s, A.n, A.Ah.Ch, A.Ah.K, A.Ah.rs, c->Ch32, c->K32, c->rs32);
  ScaledOp<float> A32;
  A32.rs = c->rs32;
  if (A.Ah.Ch) {
    A32.Ch = c->Ch32;
  } else {
    A32.K = c->K32;
    A32.mask = A.Ah.mask;
    A32.scale = A.Ah.scale;
    A32.theta = A.Ah.theta;
    A32.per_problem = A.Ah.per_problem;
  }
  return A32;
}

MixedArgs mixed_args(amrfld_ctx* c, const SolveArrays& A, const ScaledOp<float>& A32, PcgScalars* out,
                     PcgScalars* in, int max_outer) {
  MixedArgs M;
  M.Ah = A.Ah;
  M.b = A.b;
  M.x = A.x;
  M.x_alt = c->x_alt;
  M.Ah32 = A32;
  M.v32 = c->cg32;
  M.r32 = c->r32;
  M.d32 = c->d32;
  M.outer = out;
  M.inner = in;
  M.part = c->partials;
  M.bar = c->bar;
  M.inner_tol = c->o.inner_tol;
  M.max_outer = max_outer;
  M.inner_cap = c->o.max_iter;
  return M;
}

// The two start sweeps of the FP64 CG (and, for the composite system, the couplings
// of w^_0 to other levels).
void cg_start(amrfld_ctx* c, hipStream_t s, const DevLevel& D, const SweepPlan& P, const SolveArrays& A,
              PcgScalars* sc) {
  if (D.cif && D.n_if_rows > 0) {  // a composite system with couplings to other levels
    launch_cg_init_r<double>(s, D, P, A.A, A.diag, A.b, A.x, A.Ah.rs, c->cg);
    launch_cg_init_w<double>(s, D, P, A.Ah, A.b, c->cg, c->partials);
  } else {
    launch_cg_start<double>(s, D, P, A.Ah, A.b, A.x, c->cg, c->partials);
  }
  if (D.n_if_rows > 0) launch_interface(s, D, c->cg.r[0], c->cg.w[0], sc, D.if_part);
}

// hint: the iteration count of a previous solve of the same system shape (0: none);
// the first batch of sweeps covers it with a small margin, so that a solve that
// converges as fast as that one needs a single check.
void pcg_fp64(amrfld_ctx* c, const DevLevel& D, const SweepPlan& P, const SolveArrays& A, double tol,
              LoopStats* ls, int hint = 0) {
  const hipStream_t s = c->stream();
  const int np = P.n_prob;
  for (int q = 0; q < np; ++q) c->h_sc[q] = make_scalars(tol, c->o.abs_floor, c->o.max_iter, c->o.linf_test);
  launch_init_scalars(s, c->sc, np, tol, c->o.abs_floor, c->o.max_iter, c->o.linf_test);
  cg_start(c, s, D, P, A, c->sc);
  check(hipEventRecord(c->ev[1], s), "event");
  pcg_iterations<double>(c, D, P, A.Ah, c->cg, A.x, c->sc, c->h_sc, c->o.max_iter, ls,
                         hint > 0 ? hint + std::max(2, hint / 16) : 0);
}

// The plan of a level's sweeps, at most max_tiles tiles per block.
SweepPlan level_plan(const amrfld_ctx* c, int n_tiles, int max_tiles = kMaxTilesPerBlock) {
  return single_plan(sweep_blocks(n_tiles, c->o.max_blocks > 0 ? c->o.max_blocks : 1024, max_tiles), n_tiles);
}

// FP32 inner CG on A d = r inside an FP64 iterative-refinement loop: the FP64
// sweep applies x += d and forms the true residual r = b - A x; the inner solve
// uses the FP32 scaled operator, FP32 vectors and operator arithmetic with FP64 dot
// products, and after each refinement sweep continues its search direction from the
// replaced residual instead of starting afresh.  Outer scalars of problem q at
// sc[q], inner ones at sc[n_prob + q].  Every decision of the loop is made on the
// device (k_ir_finish): the host enqueues rounds and learns that all problems
// stopped when a round's inner solves all end after 0 iterations, so it reads
// scalars inside the inner solves, and right after the refinement test of a round
// that it expects to stop every problem.  With
// `persistent` the whole solve is one cooperative launch (the same bits).  Once the
// stream has run, the outer records hold the refinement sweeps (iter) and the inner
// iterations (inner_total).  P plans the FP64 sweeps and P32 the FP32 inner ones
// (the same problems; P32 may give a block longer ranges).
void pcg_mixed(amrfld_ctx* c, const DevLevel& D, const SweepPlan& P, const SweepPlan& P32, const SolveArrays& A,
               double tol, LoopStats* ls) {
  const hipStream_t s = c->stream();
  const int np = P.n_prob;
  const ScaledOp<float> A32 = operator_f32(c, s, A);
  for (int q = 0; q < np; ++q) {
    c->h_sc[q] = make_scalars(tol, c->o.abs_floor, c->o.max_iter, c->o.linf_test);
    c->h_sc[np + q] = make_scalars(c->o.inner_tol, 0.0, c->o.max_iter, 0);
  }
  launch_init_scalars(s, c->sc, np, tol, c->o.abs_floor, c->o.max_iter, c->o.linf_test);
  launch_init_scalars(s, c->sc + np, np, c->o.inner_tol, 0.0, c->o.max_iter, 0);
  check(hipEventRecord(c->ev[1], s), "event");
  PcgScalars* out = c->sc;
  PcgScalars* in = c->sc + np;
  const int max_outer = c->o.max_outer > 0 ? c->o.max_outer : 30;
  if (c->o.persistent && !D.cif) {
    if (!c->bar) c->bar = dalloc<unsigned>(kBarWords, "barrier");
    SweepPlan Pp = P, P32p = P32;
    Pp.done_count = P32p.done_count = c->bar + kBarDone;
    const MixedArgs M = mixed_args(c, A, A32, out, in, max_outer);
    const int blocks = mixed_persistent_blocks(Pp, P32p, c->o.persistent_per_cu);
    if (blocks > 0) {
      launch_zero_u32(s, c->bar, kBarWords);
      if (launch_mixed_persistent(s, D, Pp, P32p, M, c->o.persistent_per_cu) == hipSuccess) {
        unsigned aborted = 0;
        check(hipMemcpyAsync(&aborted, c->bar + kBarAbort, sizeof(unsigned), hipMemcpyDeviceToHost, s), "abort flag");
        check(hipStreamSynchronize(s), "abort flag");
        if (aborted) throw std::runtime_error("persistent sweep: a grid barrier timed out");
        ls->persistent = true;
        ls->launch_blocks = blocks;
        return;
      }
      (void)hipGetLastError();  // not launchable here: host-driven launches instead
    }
  }
  double* x_cur = A.x;
  double* x_nxt = c->x_alt;
  int hint = 0;
  bool expect_stop = false;
  for (int outer = 0; outer <= max_outer; ++outer) {
    launch_ir_sweep(s, D, P, A.Ah, A.b, x_cur, outer == 0 ? nullptr : c->d32, c->cg32.p, A32.rs, x_nxt, c->r32,
                    out, in, c->partials);
    std::swap(x_cur, x_nxt);
    launch_ir_finish(s, P, outer == 0 ? 1 : 0, c->o.inner_tol, max_outer, out, in, c->partials);
    launch_inner_init(s, D, P32, A32, c->r32, c->d32, c->cg32, out, in, c->partials);
    if (expect_stop) {
      // the refinement test is expected to stop every problem here: read its outcome
      // before enqueuing inner sweeps that would only find their problems stopped
      read_scalars(c, c->h_sc + np, in, np);
      if (all_done(c->h_sc + np, np)) break;
    }
    const int done = pcg_iterations<float>(c, D, P32, A32, c->cg32, c->d32, in, c->h_sc + np, c->o.max_iter, ls,
                                           hint + 1, np);
    if (done == 0) break;  // every refinement loop had stopped before this round's inner solves
    hint = done;
    // expected when every running problem's inner solve ended with a residual (that of
    // the FP64 one the next refinement sweep forms, up to FP32 rounding) well below its
    // refinement threshold; a wrong guess costs one read of the scalars
    expect_stop = true;
    for (int q = 0; q < np && expect_stop; ++q)
      expect_stop = c->h_sc[q].done || c->h_sc[np + q].rnorm <= 0.5 * c->h_sc[q].thresh;
  }
  if (x_cur != A.x) launch_copy_f64(s, A.x, x_cur, A.n);
}

// One backward-Euler step of one level (Sect. 3.3.4).
amrfld_status solve_one(amrfld_ctx* c, int level, double dt, int mode, double tol) {
  const hipStream_t s = c->stream();
  LevelState& L = c->L(level);
  LevelState* Lc = level > c->o.base_level ? &c->L(level - 1) : nullptr;
  upload_tables(c, L);
  if (Lc) upload_tables(c, *Lc);
  const DevLevel D = L.dev();
  ensure_workspace(c, D.n_slots);
  check(hipEventRecord(c->ev[0], s), "event");

  // diffusivities of this level and of the coarser one (fine-to-coarse faces)
  if (Lc) {
    const double* Ecc = level - 1 > c->o.base_level ? c->L(level - 2).E : nullptr;
    launch_cell_K(s, Lc->dev(), Lc->E, Lc->rho, Ecc, kparams(*Lc), outer_bc(c), Lc->K);
  }
  launch_cell_K(s, D, L.E, L.rho, Lc ? Lc->E : nullptr, kparams(L), outer_bc(c), L.K);
  const double w = mode == AMRFLD_BC_DIRICHLET ? 1.0 : mode == AMRFLD_BC_NEUMANN ? 0.0 : c->o.robin_alpha;
  const CouplingParams cp = cparams(c, L);
  launch_assemble(s, D, L.K, Lc ? Lc->K : nullptr, L.E, Lc ? Lc->E : nullptr, L.rho, L.reg, dt, w,
                  c->o.robin_alpha, cp, kparams(L), outer_bc(c), L.Cp, L.mask, L.diag, L.b);
  const double scale = dt / (D.dx * D.dx);
  if (c->o.theta != 1.0)
    launch_theta_step(s, D, c->o.theta, L.E, face_coefs(c, L.Cp, L.K, L.mask, scale, 1.0, false), L.Cp, L.diag,
                      L.b);
  const FaceCoefs<double> Aop = face_coefs(c, L.Cp, L.K, L.mask, scale, c->o.theta, false);
  const ScaledOp<double> Ah = scale_operator(c, s, D, Aop, L.Cp, L.diag, L.rs, L.Ch);

  const int n_tiles = tiles_of(D.n_slots);
  const SweepPlan P = level_plan(c, n_tiles);
  ensure_scalars(c, 1);
  LoopStats ls;
  ls.iters.assign(1, 0);
  const SolveArrays A{Aop, L.diag, L.b, L.E, D.n_slots, Ah};
  if (c->o.precision == AMRFLD_MIXED) {
    pcg_mixed(c, D, P, level_plan(c, n_tiles, kMaxTilesPerBlock32), A, tol, &ls);
  } else {
    pcg_fp64(c, D, P, A, tol, &ls, L.last_iters);
  }
  check(hipEventRecord(c->ev[2], s), "event");
  if (c->o.true_residual && c->o.precision != AMRFLD_MIXED)
    launch_true_residual(s, D, P, Ah, L.b, L.E, c->sc, c->partials);
  launch_post_solve(s, D, P, L.E, L.rho, cp, dt, L.T, c->sc, c->partials);
  if (Lc && (mode == AMRFLD_BC_NEUMANN || mode == AMRFLD_BC_ROBIN)) {
    double* reg = ensure_reg(c, *Lc);
    launch_flux_register(s, D, L.K, Lc->K, L.E, Lc->E, dt, reg, int(Lc->t.n_slots()));
  }
  if (L.reg) launch_fill(s, L.reg, 6 * L.t.n_slots(), 0.0);
  check(hipEventRecord(c->ev[3], s), "event");
  read_scalars(c, c->h_sc, c->sc, 1);
  check(hipGetLastError(), "kernels");

  const PcgScalars& h = *c->h_sc;
  if (c->o.precision != AMRFLD_MIXED) L.last_iters = h.iter;
  amrfld_stats st{};
  st.level = level;
  st.iters = h.iter;
  st.converged = h.converged;
  st.n_leaf = L.t.n_leaf;
  st.rel_res = h.rnorm0 > 0 ? h.rnorm / h.rnorm0 : 0.0;
  if (c->o.precision == AMRFLD_MIXED) {
    st.iters = h.inner_total;
    st.outer_iters = h.iter;
    st.true_rel_res = st.rel_res;  // the outer residual is the FP64 true residual
  } else {
    st.true_rel_res = c->o.true_residual ? (h.rnorm0 > 0 ? h.true_rnorm / h.rnorm0 : 0.0) : -1.0;
  }
  st.linf_change = h.linf;
  st.min_E = h.min_E;
  st.dt = dt;
  st.rnorm0 = h.rnorm0;
  st.bnorm = h.bnorm;
  st.sweep_blocks = P.G;
  st.launch_blocks = ls.persistent ? ls.launch_blocks : P.G;
  st.launch_mode = ls.persistent ? 1 : 0;
  float ms = 0.f, pms = 0.f;
  check(hipEventSynchronize(c->ev[3]), "event");  // passed already: the scalars were read after it
  check(hipEventElapsedTime(&ms, c->ev[0], c->ev[3]), "event");
  check(hipEventElapsedTime(&pms, c->ev[1], c->ev[2]), "event");
  st.ms = ms;
  st.pcg_ms = pms;
  st.n_timed = ls.n_timed;
  st.sweep_ms = ls.sweep_ms;
  st.spare_ms = 0.0;
  amrfld_status status = AMRFLD_OK;
  if (h.nonfinite) status = AMRFLD_E_NONFINITE;
  else if (!h.converged) status = AMRFLD_E_NOCONV;
  st.status = status;
  c->stats.push_back(st);
  if (status == AMRFLD_E_NONFINITE)
    return fail(c, status, "non-finite value in the residual of level " + std::to_string(level));
  if (status == AMRFLD_E_NOCONV)
    return fail(c, status, "PCG did not converge within max_iter on level " + std::to_string(level));
  return AMRFLD_OK;
}

// The solves of one coarse step in the order of step(): level, dt and whether the
// finer level is restricted into it first.
struct ScheduledSolve {
  int level;
  double dt;
  bool restrict_first;
};

void schedule(const amrfld_ctx* c, int level, double dt, std::vector<ScheduledSolve>& out) {
  bool restricted = false;
  if (level < c->finest) {
    const int ns = c->nsub(level + 1);
    for (int k = 0; k < ns; ++k) schedule(c, level + 1, dt / ns, out);
    restricted = true;
  }
  out.push_back({level, dt, restricted});
}

// The kernels of one level solve with its PCG (mixed precision: its whole refinement
// loop) in one persistent launch, enqueued without host synchronisation (scalars in
// sc, the inner records of the mixed form in sc_inner; the barrier words of c->bar,
// whose abort flag is left for the caller to read).
hipError_t record_solve(amrfld_ctx* c, hipStream_t st, int level, double dt, int mode, double tol, PcgScalars* sc,
                        PcgScalars* sc_inner) {
  LevelState& L = c->L(level);
  LevelState* Lc = level > c->o.base_level ? &c->L(level - 1) : nullptr;
  const DevLevel D = L.dev();
  if (Lc) {
    const double* Ecc = level - 1 > c->o.base_level ? c->L(level - 2).E : nullptr;
    launch_cell_K(st, Lc->dev(), Lc->E, Lc->rho, Ecc, kparams(*Lc), outer_bc(c), Lc->K);
  }
  launch_cell_K(st, D, L.E, L.rho, Lc ? Lc->E : nullptr, kparams(L), outer_bc(c), L.K);
  const double w = mode == AMRFLD_BC_DIRICHLET ? 1.0 : mode == AMRFLD_BC_NEUMANN ? 0.0 : c->o.robin_alpha;
  const CouplingParams cp = cparams(c, L);
  launch_assemble(st, D, L.K, Lc ? Lc->K : nullptr, L.E, Lc ? Lc->E : nullptr, L.rho, L.reg, dt, w,
                  c->o.robin_alpha, cp, kparams(L), outer_bc(c), L.Cp, L.mask, L.diag, L.b);
  const double scale = dt / (D.dx * D.dx);
  if (c->o.theta != 1.0)
    launch_theta_step(st, D, c->o.theta, L.E, face_coefs(c, L.Cp, L.K, L.mask, scale, 1.0, false), L.Cp, L.diag,
                      L.b);
  const FaceCoefs<double> Aop = face_coefs(c, L.Cp, L.K, L.mask, scale, c->o.theta, false);
  const ScaledOp<double> Ah = scale_operator(c, st, D, Aop, L.Cp, L.diag, L.rs, L.Ch);
  const SolveArrays A{Aop, L.diag, L.b, L.E, D.n_slots, Ah};
  const int n_tiles = tiles_of(D.n_slots);
  const SweepPlan P = level_plan(c, n_tiles);
  SweepPlan Pp = P, P32p = level_plan(c, n_tiles, kMaxTilesPerBlock32);
  Pp.done_count = P32p.done_count = c->bar + kBarDone;
  const bool mixed = c->o.precision == AMRFLD_MIXED;
  launch_init_scalars(st, sc, 1, tol, c->o.abs_floor, c->o.max_iter, c->o.linf_test);
  launch_zero_u32(st, c->bar, kBarAbort);  // arrivals, releases, stop counts; not the abort flag
  hipError_t e;
  if (mixed) {
    const ScaledOp<float> A32 = operator_f32(c, st, A);
    launch_init_scalars(st, sc_inner, 1, c->o.inner_tol, 0.0, c->o.max_iter, 0);
    const int max_outer = c->o.max_outer > 0 ? c->o.max_outer : 30;
    e = launch_mixed_persistent(st, D, Pp, P32p, mixed_args(c, A, A32, sc, sc_inner, max_outer),
                                c->o.persistent_per_cu);
  } else {
    cg_start(c, st, D, P, A, sc);
    e = launch_pcg_persistent<double>(st, D, Pp, c->o.max_iter, Ah, c->cg, L.E, sc, c->partials, c->bar,
                                      c->o.persistent_per_cu);
  }
  if (e != hipSuccess) return e;
  if (c->o.true_residual && !mixed) launch_true_residual(st, D, P, Ah, L.b, L.E, sc, c->partials);
  launch_post_solve(st, D, P, L.E, L.rho, cp, dt, L.T, sc, c->partials);
  if (Lc && (mode == AMRFLD_BC_NEUMANN || mode == AMRFLD_BC_ROBIN))
    launch_flux_register(st, D, L.K, Lc->K, L.E, Lc->E, dt, Lc->reg, int(Lc->t.n_slots()));
  if (L.reg) launch_fill(st, L.reg, 6 * L.t.n_slots(), 0.0);
  return hipGetLastError();
}

// One coarse step as a graph of persistent level solves (FP64 PCG, or the whole
// mixed-precision refinement loop): captured on first use and replayed while dt,
// mode, tol, the context's parameters and its device buffers are those it was
// captured with.  AMRFLD_E_STATE: not available here (no cooperative launch, capture
// refused); the caller then runs the step eagerly.
amrfld_status advance_graph(amrfld_ctx* c, double dt_coarse, int mode, double tol) {
  if (!c->o.graph || !c->o.persistent) return AMRFLD_E_STATE;
  const bool mixed = c->o.precision == AMRFLD_MIXED;
  std::vector<ScheduledSolve> sched;
  schedule(c, c->o.base_level, dt_coarse, sched);
  const int n = int(sched.size());
  // everything the captured kernels touch exists before the capture
  int64_t max_slots = 0;
  for (int l = c->o.base_level; l <= c->finest; ++l) {
    upload_tables(c, c->L(l));
    max_slots = std::max<int64_t>(max_slots, c->L(l).t.n_slots());
    if (l < c->finest && (mode == AMRFLD_BC_NEUMANN || mode == AMRFLD_BC_ROBIN)) ensure_reg(c, c->L(l));
  }
  ensure_workspace(c, max_slots);
  if (mixed) ensure_workspace32(c, max_slots);
  ensure_scalars(c, n + 1);  // n solves, then the shared inner record of the mixed form
  if (!c->bar) c->bar = dalloc<unsigned>(kBarWords, "barrier");
  for (int l = c->o.base_level; l <= c->finest; ++l) {
    const int nt = tiles_of(c->L(l).t.n_slots());
    const SweepPlan P = level_plan(c, nt);
    const int pb = mixed ? mixed_persistent_blocks(P, level_plan(c, nt, kMaxTilesPerBlock32),
                                                   c->o.persistent_per_cu)
                         : persistent_blocks<double>(P, c->o.persistent_per_cu);
    if (pb <= 0) return AMRFLD_E_STATE;
  }
  const hipStream_t us = c->stream();
  StepGraph& sg = c->step_graph;
  const uint64_t epoch = g_alloc_epoch.load();
  if (!(sg.ex && sg.dt == dt_coarse && sg.tol == tol && sg.mode == mode && sg.alloc_epoch == epoch &&
        sg.param_epoch == c->param_epoch)) {
    sg.reset();
    if (!c->cap_stream) check(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "stream");
    for (auto& e : c->cap_ev)
      if (!e) check(hipEventCreate(&e), "event");
    check(hipEventRecord(c->cap_ev[0], us), "event");
    check(hipStreamWaitEvent(c->cap_stream, c->cap_ev[0], 0), "event");
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    hipError_t e_rec = e;
    if (e == hipSuccess) {
      launch_zero_u32(c->cap_stream, c->bar, kBarWords);
      int k = 0;
      for (const ScheduledSolve& op : sched) {
        if (e_rec != hipSuccess) break;
        if (op.restrict_first) {
          LevelState& F = c->L(op.level + 1);
          launch_restrict(c->cap_stream, F.dev(), F.E, c->L(op.level).E);
        }
        e_rec = record_solve(c, c->cap_stream, op.level, op.dt, mode, tol, c->sc + k++, c->sc + n);
      }
    }
    const hipError_t e_end = e == hipSuccess ? hipStreamEndCapture(c->cap_stream, &sg.g) : e;
    if (e_rec == hipSuccess && e_end == hipSuccess && sg.g) e = hipGraphInstantiate(&sg.ex, sg.g, nullptr, nullptr, 0);
    else e = hipErrorNotSupported;
    if (e != hipSuccess) {
      sg.reset();
      (void)hipGetLastError();
      return AMRFLD_E_STATE;
    }
    sg.dt = dt_coarse;
    sg.tol = tol;
    sg.mode = mode;
    sg.alloc_epoch = epoch;
    sg.param_epoch = c->param_epoch;
  }
  check(hipEventRecord(c->ev[0], us), "event");
  check(hipGraphLaunch(sg.ex, us), "graph launch");
  check(hipEventRecord(c->ev[3], us), "event");
  check(hipStreamSynchronize(us), "sync");
  float total_ms = 0.f;
  check(hipEventElapsedTime(&total_ms, c->ev[0], c->ev[3]), "event");
  unsigned aborted = 0;
  check(hipMemcpy(&aborted, c->bar + kBarAbort, sizeof(unsigned), hipMemcpyDeviceToHost), "abort flag");
  read_scalars(c, c->h_sc, c->sc, n);
  amrfld_status worst = AMRFLD_OK;
  std::string worst_msg;
  for (int k = 0; k < n; ++k) {
    const PcgScalars& h = c->h_sc[k];
    const LevelState& L = c->L(sched[k].level);
    const int nt = tiles_of(L.t.n_slots());
    const SweepPlan P = level_plan(c, nt);
    amrfld_stats st{};
    st.level = sched[k].level;
    st.iters = mixed ? h.inner_total : h.iter;
    st.outer_iters = mixed ? h.iter : 0;
    st.converged = h.converged;
    st.n_leaf = L.t.n_leaf;
    st.rel_res = h.rnorm0 > 0 ? h.rnorm / h.rnorm0 : 0.0;
    st.true_rel_res = mixed ? st.rel_res : (c->o.true_residual ? (h.rnorm0 > 0 ? h.true_rnorm / h.rnorm0 : 0.0) : -1.0);
    st.linf_change = h.linf;
    st.min_E = h.min_E;
    st.dt = sched[k].dt;
    st.ms = total_ms / n;
    st.pcg_ms = -1.0;
    st.rnorm0 = h.rnorm0;
    st.bnorm = h.bnorm;
    st.sweep_blocks = P.G;
    st.launch_blocks = mixed ? mixed_persistent_blocks(P, level_plan(c, nt, kMaxTilesPerBlock32),
                                                       c->o.persistent_per_cu)
                             : persistent_blocks<double>(P, c->o.persistent_per_cu);
    st.launch_mode = 2;
    st.status = h.nonfinite ? AMRFLD_E_NONFINITE : (h.converged ? AMRFLD_OK : AMRFLD_E_NOCONV);
    if (st.status != AMRFLD_OK && worst == AMRFLD_OK) {
      worst = amrfld_status(st.status);
      worst_msg = (st.status == AMRFLD_E_NONFINITE ? "non-finite value in the residual of level "
                                                   : "PCG did not converge within max_iter on level ") +
                  std::to_string(sched[k].level);
    }
    c->stats.push_back(st);
  }
  if (aborted) return fail(c, AMRFLD_E_DEVICE, "persistent sweep: a grid barrier timed out");
  if (worst != AMRFLD_OK) return fail(c, worst, worst_msg);
  return AMRFLD_OK;
}

amrfld_status step(amrfld_ctx* c, int level, double dt, int mode, double tol) {
  amrfld_status worst = AMRFLD_OK;
  if (level < c->finest) {
    const int ns = c->nsub(level + 1);
    for (int k = 0; k < ns; ++k) {
      const amrfld_status s = step(c, level + 1, dt / ns, mode, tol);
      if (s != AMRFLD_OK && worst == AMRFLD_OK) worst = s;
      if (s == AMRFLD_E_NONFINITE || s == AMRFLD_E_DEVICE) return s;
    }
    LevelState& F = c->L(level + 1);
    launch_restrict(c->stream(), F.dev(), F.E, c->L(level).E);
  }
  const amrfld_status s = solve_one(c, level, dt, mode, tol);
  return worst != AMRFLD_OK ? worst : s;
}

}  // namespace

// Concatenated slot space of all levels for the unique-time-step composite system:
// each level's slots at a tile-aligned offset (padding slots are identity rows),
// neighbour, coarse-neighbour and child tables in that space, the level of each oct.
struct CompositeState {
  std::vector<int64_t> off;  // slot offset of each level (index level - base)
  int64_t n_slots = 0, n_oct = 0;
  int n_levels = 0;
  int32_t *nbr = nullptr, *cnb = nullptr, *child = nullptr, *lvl = nullptr;
  PatchParams* pp = nullptr;
  std::vector<PatchParams> pp_host;
  double *x = nullptr, *K = nullptr, *rho = nullptr, *T = nullptr;
  double *Cp = nullptr, *cif = nullptr, *diag = nullptr, *b = nullptr;
  double *Ch = nullptr, *rs = nullptr;  // the Jacobi-scaled operator of the current solve
  uint8_t* c2f = nullptr;
  // rows coupled to other levels: row, entry range, column, coefficient index into cif
  int n_if_rows = 0, n_if_entries = 0;
  int32_t *if_row = nullptr, *if_ptr = nullptr, *if_col = nullptr, *if_src = nullptr;
  double *if_val = nullptr, *if_part = nullptr;

  DevLevel dev() const {
    DevLevel d;
    d.n_slots = int(n_slots);
    d.n_oct = int(n_oct);
    d.nbr = nbr;
    d.cnb = cnb;
    d.child = child;
    d.oct_prob = lvl;
    d.pp = pp;
    d.cif = cif;
    d.c2f = c2f;
    d.n_if_rows = n_if_rows;
    d.if_row = if_row;
    d.if_ptr = if_ptr;
    d.if_col = if_col;
    d.if_src = if_src;
    d.if_val = if_val;
    d.if_part = if_part;
    return d;
  }
  void release() {
    for (void* p : {(void*)nbr, (void*)cnb, (void*)child, (void*)lvl, (void*)pp, (void*)x, (void*)K, (void*)rho,
                    (void*)T, (void*)Cp, (void*)cif, (void*)diag, (void*)b, (void*)c2f, (void*)if_row,
                    (void*)if_ptr, (void*)if_col, (void*)if_src, (void*)if_val, (void*)if_part, (void*)Ch, (void*)rs})
      dfree(p);
  }
};

namespace {

template <class T>
void upload(amrfld_ctx* c, T** dst, const std::vector<T>& v, const char* what) {
  *dst = dalloc<T>(int64_t(v.size()), what);
  check(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream()), what);
}

// The composite slot space of the context's levels (rebuilt after a level changes).
void build_composite_into(amrfld_ctx* c, CompositeState* C);

// The composite slot space, built once for the current levels; a failed build
// leaves none behind.
void build_composite(amrfld_ctx* c) {
  if (c->comp) return;
  CompositeState* C = new CompositeState();
  try {
    build_composite_into(c, C);
  } catch (...) {
    (void)hipStreamSynchronize(c->stream());  // copies from host vectors that are gone
    C->release();
    delete C;
    throw;
  }
  c->comp = C;
}

void build_composite_into(amrfld_ctx* c, CompositeState* C) {
  const int base = c->o.base_level;
  C->n_levels = c->finest - base + 1;
  C->off.assign(C->n_levels + 1, 0);
  for (int k = 0; k < C->n_levels; ++k) {
    const int64_t ns = c->L(base + k).t.n_slots();
    C->off[k + 1] = C->off[k] + (ns + kBlock - 1) / kBlock * kBlock;
  }
  C->n_slots = C->off[C->n_levels];
  C->n_oct = C->n_slots / 8;
  if (C->n_slots > int64_t(0x7fffffff)) throw std::invalid_argument("hierarchy too large for 32-bit slot indices");
  std::vector<int32_t> nbr(6 * C->n_oct, -1), cnb(6 * C->n_oct, -1), child(C->n_slots, -2), lvl(C->n_oct, 0);
  for (int k = 0; k < C->n_levels; ++k) {
    const LevelTables& t = c->L(base + k).t;
    const int64_t oo = C->off[k] / 8;
    for (int64_t o = oo; o < C->off[k + 1] / 8; ++o) lvl[o] = k;
    for (int64_t o = 0; o < t.n_oct; ++o) {
      for (int d = 0; d < 6; ++d) {
        const int32_t nb = t.nbr[o * 6 + d], cb = t.cnb[o * 6 + d];
        nbr[(oo + o) * 6 + d] = nb >= 0 ? int32_t(oo + nb) : -1;
        cnb[(oo + o) * 6 + d] = (cb >= 0 && k > 0) ? int32_t(C->off[k - 1] + cb) : -1;
      }
    }
    for (int64_t i = 0; i < t.n_slots(); ++i) {
      const int32_t ch = t.child[i];
      child[C->off[k] + i] = (ch >= 0 && k + 1 < C->n_levels) ? int32_t(C->off[k + 1] / 8 + ch) : -1;
    }
  }
  // rows with couplings to other levels: faces towards a coarser leaf, and the four
  // finer cells of each face shared with a refined same-level neighbour
  std::vector<int32_t> if_row, if_ptr(1, 0), if_col, if_src;
  const int64_t n3 = C->n_slots;
  for (int k = 0; k < C->n_levels; ++k) {
    const LevelTables& t = c->L(base + k).t;
    for (int64_t i = 0; i < t.n_slots(); ++i) {
      if (t.child[i] != -1) continue;
      const int pos = int(i & 7);
      const int64_t o = i >> 3, gi = C->off[k] + i;
      const size_t before = if_col.size();
      for (int a = 0; a < 3 && k > 0; ++a) {
        const int d = 2 * a + ((pos >> a) & 1);
        if (t.nbr[o * 6 + d] < 0 && t.cnb[o * 6 + d] >= 0) {
          if_col.push_back(int32_t(C->off[k - 1] + t.cnb[o * 6 + d]));
          if_src.push_back(int32_t(a * n3 + gi));
        }
      }
      for (int d = 0; d < 6 && k + 1 < C->n_levels; ++d) {
        const int a = d >> 1, side = d & 1, bit = 1 << a;
        int64_t j = -1;
        if (((pos >> a) & 1) != side) {
          j = i ^ bit;
        } else if (t.nbr[o * 6 + d] >= 0) {
          j = (int64_t(t.nbr[o * 6 + d]) << 3) | (pos ^ bit);
        }
        if (j < 0 || t.child[j] < 0) continue;
        const int64_t co = C->off[k + 1] / 8 + t.child[j];
        const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2, fb = side ? 0 : 1;
        for (int q = 0; q < 4; ++q) {
          const int64_t f = (co << 3) | (fb << a) | ((q & 1) << t0) | ((q >> 1) << t1);
          if_col.push_back(int32_t(f));
          if_src.push_back(int32_t(a * n3 + f));
        }
      }
      if (if_col.size() > before) {
        if_row.push_back(int32_t(gi));
        if_ptr.push_back(int32_t(if_col.size()));
      }
    }
  }
  if (3 * n3 > int64_t(0x7fffffff) || if_col.size() > size_t(0x7fffffff))
    throw std::invalid_argument("hierarchy too large for 32-bit interface indices");
  C->n_if_rows = int(if_row.size());
  C->n_if_entries = int(if_col.size());
  upload(c, &C->nbr, nbr, "composite tables");
  upload(c, &C->cnb, cnb, "composite tables");
  upload(c, &C->child, child, "composite tables");
  upload(c, &C->lvl, lvl, "composite tables");
  if (!if_row.empty()) {
    upload(c, &C->if_row, if_row, "composite interfaces");
    upload(c, &C->if_ptr, if_ptr, "composite interfaces");
    upload(c, &C->if_col, if_col, "composite interfaces");
    upload(c, &C->if_src, if_src, "composite interfaces");
  }
  C->if_part = dalloc<double>(std::max(1, (C->n_if_rows + kBlock - 1) / kBlock), "composite interfaces");
  if (C->n_if_entries > 0) C->if_val = dalloc<double>(C->n_if_entries, "composite interfaces");
  C->pp = dalloc<PatchParams>(C->n_levels, "composite parameters");
  C->pp_host.assign(C->n_levels, PatchParams{});
  const int64_t n = C->n_slots;
  C->x = dalloc<double>(n, "composite fields");
  C->K = dalloc<double>(n, "composite fields");
  C->rho = dalloc<double>(n, "composite fields");
  C->T = dalloc<double>(n, "composite fields");
  C->Cp = dalloc<double>(3 * n, "composite system");
  C->cif = dalloc<double>(3 * n, "composite system");
  C->diag = dalloc<double>(n, "composite system");
  C->b = dalloc<double>(n, "composite system");
  C->Ch = dalloc<double>(3 * n, "composite system");
  C->rs = dalloc<double>(n, "composite system");
  C->c2f = dalloc<uint8_t>(n, "composite system");
  launch_fill(c->stream(), C->x, n, 0.0);  // padding slots keep x = 0 (identity rows)
  launch_fill(c->stream(), C->rho, n, 1.0);
  launch_fill(c->stream(), C->T, n, 1.0);
  check(hipStreamSynchronize(c->stream()), "composite tables");
}

// One composite solve: every level advanced by dt together.
amrfld_status solve_composite(amrfld_ctx* c, double dt, double tol) {
  const hipStream_t s = c->stream();
  CompositeState& C = *c->comp;
  const int base = c->o.base_level;
  for (int k = 0; k < C.n_levels; ++k) upload_tables(c, c->L(base + k));
  ensure_workspace(c, C.n_slots);
  ensure_scalars(c, 1 + C.n_levels);
  const bool coupled = c->L(base).has_T;
  check(hipEventRecord(c->ev[0], s), "event");
  for (int k = 0; k < C.n_levels; ++k) {
    LevelState& L = c->L(base + k);
    const double* Ec = k > 0 ? c->L(base + k - 1).E : nullptr;
    launch_cell_K(s, L.dev(), L.E, L.rho, Ec, kparams(L), outer_bc(c), C.K + C.off[k]);
    launch_copy_f64(s, C.x + C.off[k], L.E, L.t.n_slots());
    launch_copy_f64(s, C.rho + C.off[k], L.rho, L.t.n_slots());
    if (coupled) launch_copy_f64(s, C.T + C.off[k], L.T, L.t.n_slots());
    const double dx = 1.0 / double(int64_t(1) << (base + k));
    PatchParams& P = C.pp_host[k];
    P.dx = dx;
    P.vol = dx * dx * dx;
    P.coef = dt / (dx * dx);
    P.kmode = L.kmode;  // the level's law, for the diffusivity of values held at box faces
    P.K_const = L.K_const;
    P.K_exp = L.K_exp;
    P.kappa_R = L.kappa_R;
    P.c_light = L.c_light;
  }
  check(hipMemcpyAsync(C.pp, C.pp_host.data(), C.n_levels * sizeof(PatchParams), hipMemcpyHostToDevice, s),
        "parameters");
  CouplingParams cp = cparams(c, c->L(base));
  cp.T = coupled ? C.T : nullptr;
  const DevLevel D = C.dev();
  launch_assemble_composite(s, D, C.K, C.x, C.rho, cp, outer_bc(c), dt, C.Cp, C.cif, C.c2f, C.diag, C.b);
  const ScaledOp<double> Ah = scale_operator(c, s, D, stored_face_coefs(C.Cp), C.Cp, C.diag, C.rs, C.Ch);
  launch_interface_values(s, D, C.n_if_entries, C.cif, C.rs, C.if_val);
  const int n_tiles = tiles_of(C.n_slots);
  const int B = c->o.max_blocks > 0 ? c->o.max_blocks : 1024;
  SweepPlan P = single_plan(sweep_blocks(n_tiles, B), n_tiles);
  if (C.n_if_rows > 0) {
    P.extra_part = C.if_part;
    P.n_extra = interface_blocks(D);
  }
  LoopStats ls;
  ls.iters.assign(1, 0);
  pcg_fp64(c, D, P, SolveArrays{stored_face_coefs(C.Cp), C.diag, C.b, C.x, C.n_slots, Ah}, tol, &ls);
  check(hipEventRecord(c->ev[2], s), "event");
  if (c->o.true_residual) launch_true_residual(s, D, P, stored_face_coefs(C.Cp), C.diag, C.b, C.x, c->sc, c->partials);
  int64_t n_leaf = 0;
  for (int k = 0; k < C.n_levels; ++k) {
    LevelState& L = c->L(base + k);
    launch_copy_f64(s, L.E, C.x + C.off[k], L.t.n_slots());
    const int tl = tiles_of(L.t.n_slots());
    launch_post_solve(s, L.dev(), single_plan(sweep_blocks(tl, B), tl), L.E, L.rho, cparams(c, L), dt, L.T,
                      c->sc + 1 + k, c->partials);
    n_leaf += L.t.n_leaf;
  }
  for (int level = c->finest; level > base; --level) {
    LevelState& F = c->L(level);
    launch_restrict(s, F.dev(), F.E, c->L(level - 1).E);
  }
  check(hipEventRecord(c->ev[3], s), "event");
  read_scalars(c, c->h_sc, c->sc, 1 + C.n_levels);
  check(hipGetLastError(), "kernels");
  const PcgScalars& h = c->h_sc[0];
  amrfld_stats st{};
  st.level = -1;
  st.iters = h.iter;
  st.converged = h.converged;
  st.n_leaf = n_leaf;
  st.rel_res = h.rnorm0 > 0 ? h.rnorm / h.rnorm0 : 0.0;
  st.true_rel_res = c->o.true_residual ? (h.rnorm0 > 0 ? h.true_rnorm / h.rnorm0 : 0.0) : -1.0;
  st.linf_change = h.linf;
  st.min_E = c->h_sc[1].min_E;
  for (int k = 1; k < C.n_levels; ++k) st.min_E = std::min(st.min_E, c->h_sc[1 + k].min_E);
  st.dt = dt;
  st.rnorm0 = h.rnorm0;
  st.bnorm = h.bnorm;
  st.sweep_blocks = P.G;
  st.launch_blocks = P.G;
  float ms = 0.f, pms = 0.f;
  check(hipEventSynchronize(c->ev[3]), "event");  // passed already: the scalars were read after it
  check(hipEventElapsedTime(&ms, c->ev[0], c->ev[3]), "event");
  check(hipEventElapsedTime(&pms, c->ev[1], c->ev[2]), "event");
  st.ms = ms;
  st.pcg_ms = pms;
  st.n_timed = ls.n_timed;
  st.sweep_ms = ls.sweep_ms;
  st.spare_ms = 0.0;
  st.status = h.nonfinite ? AMRFLD_E_NONFINITE : (h.converged ? AMRFLD_OK : AMRFLD_E_NOCONV);
  c->stats.push_back(st);
  if (st.status == AMRFLD_E_NONFINITE) return fail(c, AMRFLD_E_NONFINITE, "non-finite value in the composite residual");
  if (st.status == AMRFLD_E_NOCONV) return fail(c, AMRFLD_E_NOCONV, "composite PCG did not converge within max_iter");
  return AMRFLD_OK;
}

amrfld_status advance_unique(amrfld_ctx* c, double dt_coarse, double tol) {
  int64_t n = 1;
  for (int l = c->o.base_level + 1; l <= c->finest; ++l) n *= c->nsub(l);
  if (n > (int64_t(1) << 20)) return fail(c, AMRFLD_E_INVALID, "too many unique time steps per coarse step");
  const int base = c->o.base_level;
  for (int l = base; l <= c->finest; ++l)
    if (c->L(l).has_T != c->L(base).has_T)
      return fail(c, AMRFLD_E_STATE, "T must be set on every level or on none");
  build_composite(c);
  amrfld_status worst = AMRFLD_OK;
  for (int64_t k = 0; k < n; ++k) {
    const amrfld_status st = solve_composite(c, dt_coarse / double(n), tol);
    if (st != AMRFLD_OK && worst == AMRFLD_OK) worst = st;
    if (st == AMRFLD_E_NONFINITE || st == AMRFLD_E_DEVICE) return st;
  }
  return worst;
}

// Morton-ordered octs of each patch, tile-aligned slot ranges (padding slots are
// identity rows), neighbour tables within each patch, and the block plan: each
// patch gets enough blocks for at most `tpb` tiles per block.
void build_batch_into(amrfld_ctx* c, BatchState* B, const std::vector<int>& sizes);

// The batch layout for these patch sizes, kept while they repeat; a failed build
// leaves no layout behind.
void build_batch(amrfld_ctx* c, const std::vector<int>& sizes) {
  BatchState* B = c->batch;
  if (B && B->sizes == sizes) return;
  if (B) {
    B->release();
    B->sizes.clear();
  } else {
    B = c->batch = new BatchState();
  }
  try {
    build_batch_into(c, B, sizes);
  } catch (...) {
    (void)hipStreamSynchronize(c->stream());  // copies from host vectors that are gone
    B->release();
    B->sizes.clear();
    throw;
  }
  B->sizes = sizes;
}

void build_batch_into(amrfld_ctx* c, BatchState* B, const std::vector<int>& sizes) {
  B->n_prob = int(sizes.size());
  std::vector<int64_t> oct0(B->n_prob + 1, 0), tile0(B->n_prob + 1, 0);
  B->out_off.assign(B->n_prob + 1, 0);
  for (int q = 0; q < B->n_prob; ++q) {
    const int64_t m = sizes[q] / 2;
    const int64_t slots = 8 * m * m * m;
    const int64_t tiles = (slots + kBlock - 1) / kBlock;
    tile0[q + 1] = tile0[q] + tiles;
    oct0[q + 1] = tile0[q + 1] * (kBlock / 8);
    B->out_off[q + 1] = B->out_off[q] + int64_t(sizes[q]) * sizes[q] * sizes[q];
  }
  B->n_oct = oct0[B->n_prob];
  B->n_slots = 8 * B->n_oct;
  if (B->n_slots > int64_t(0x7fffffff)) throw std::invalid_argument("batch too large for 32-bit slot indices");
  std::vector<int32_t> nbr(6 * B->n_oct, -1), child(B->n_slots, -2), oct_prob(B->n_oct), idx(B->n_slots, -1);
  const int kOff[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
  for (int q = 0; q < B->n_prob; ++q) {
    const int n = sizes[q];
    const int m = n / 2;
    const int64_t mo = int64_t(m) * m * m;
    std::vector<int64_t> order(mo);
    std::vector<uint64_t> key(mo);
    for (int64_t k = 0; k < mo; ++k) {
      order[k] = k;
      key[k] = morton3(uint32_t(k % m), uint32_t((k / m) % m), uint32_t(k / (int64_t(m) * m)));
    }
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b2) { return key[a] < key[b2]; });
    std::vector<int32_t> local_of(mo);  // position -> local oct index
    for (int64_t o = 0; o < mo; ++o) local_of[order[o]] = int32_t(o);
    for (int64_t o = 0; o < oct0[q + 1] - oct0[q]; ++o) oct_prob[oct0[q] + o] = q;
    for (int64_t o = 0; o < mo; ++o) {
      const int64_t lin = order[o];
      const int I = int(lin % m), J = int((lin / m) % m), K = int(lin / (int64_t(m) * m));
      const int64_t go = oct0[q] + o;
      for (int d = 0; d < 6; ++d) {
        const int a = I + kOff[d][0], b2 = J + kOff[d][1], cc = K + kOff[d][2];
        if (a < 0 || b2 < 0 || cc < 0 || a >= m || b2 >= m || cc >= m) continue;
        nbr[6 * go + d] = int32_t(oct0[q] + local_of[a + int64_t(m) * (b2 + int64_t(m) * cc)]);
      }
      for (int pos = 0; pos < 8; ++pos) {
        const int64_t slot = 8 * go + pos;
        const int x = 2 * I + (pos & 1), y = 2 * J + ((pos >> 1) & 1), z = 2 * K + ((pos >> 2) & 1);
        child[slot] = -1;
        idx[slot] = int32_t(x + int64_t(n) * (y + int64_t(n) * z));
      }
    }
  }
  // blocks: at most tpb tiles per block, about >= 1024 blocks in total
  const int64_t total_tiles = tile0[B->n_prob];
  const int max_blocks = c->o.max_blocks > 0 ? c->o.max_blocks : 1024;
  const int tpb = int(std::max<int64_t>(1, std::min<int64_t>(kMaxTilesPerBlock, total_tiles / max_blocks)));
  std::vector<int32_t> blk0(B->n_prob + 1, 0), t0v(B->n_prob + 1, 0), blk_prob;
  int tpb_max = 1;
  for (int q = 0; q < B->n_prob; ++q) {
    const int64_t tiles = tile0[q + 1] - tile0[q];
    const int64_t g = (tiles + tpb - 1) / tpb;
    blk0[q + 1] = int32_t(blk0[q] + g);
    t0v[q + 1] = int32_t(tile0[q + 1]);
    tpb_max = std::max<int>(tpb_max, int((tiles + g - 1) / g));
    for (int64_t k = 0; k < g; ++k) blk_prob.push_back(q);
  }
  B->G = blk0[B->n_prob];
  B->tpb_max = tpb_max;
  std::vector<int32_t> cnb(6 * B->n_oct, -1);
  upload(c, &B->nbr, nbr, "batch tables");
  upload(c, &B->cnb, cnb, "batch tables");
  upload(c, &B->child, child, "batch tables");
  upload(c, &B->oct_prob, oct_prob, "batch tables");
  upload(c, &B->idx, idx, "batch tables");
  upload(c, &B->blk_prob, blk_prob, "batch tables");
  upload(c, &B->blk0, blk0, "batch tables");
  upload(c, &B->tile0, t0v, "batch tables");
  upload(c, &B->d_out_off, B->out_off, "batch tables");
  B->E = dalloc<double>(B->n_slots, "batch fields");
  B->rho = dalloc<double>(B->n_slots, "batch fields");
  B->K = dalloc<double>(B->n_slots, "batch fields");
  B->Cp = dalloc<double>(3 * B->n_slots, "batch fields");
  B->mask = dalloc<uint8_t>(B->n_slots, "batch fields");
  B->diag = dalloc<double>(B->n_slots, "batch fields");
  B->b = dalloc<double>(B->n_slots, "batch fields");
  B->Ch = dalloc<double>(3 * B->n_slots, "batch fields");
  B->rs = dalloc<double>(B->n_slots, "batch fields");
  B->pp = dalloc<PatchParams>(B->n_prob, "batch params");
  B->src = reinterpret_cast<const double**>(dalloc<const double*>(B->n_prob, "batch pointers"));
  check(hipStreamSynchronize(c->stream()), "batch tables");
}

// All steps of a batch with one cooperative launch per step for the PCG
// iterations, optionally captured in one hipGraph.  Returns AMRFLD_E_STATE when
// the device cannot run the cooperative launch (the caller then polls).
amrfld_status solve_batch_persistent(amrfld_ctx* c, const std::vector<amrfld_patch>& pt, int n_steps, double tol,
                                     int precision) {
  BatchState& B = *c->batch;
  const int np = B.n_prob;
  const DevLevel D = B.dev();
  SweepPlan P = B.plan();
  if (!c->bar) c->bar = dalloc<unsigned>(kBarWords, "barrier");
  P.done_count = c->bar + kBarDone;
  const unsigned* abort_flag = c->bar + kBarAbort;
  const int per_cu = c->o.persistent_per_cu;
  const bool mixed = precision == AMRFLD_MIXED;
  if ((mixed ? mixed_persistent_blocks(P, P, per_cu) : persistent_blocks<double>(P, per_cu)) <= 0) return AMRFLD_E_STATE;
  // one record per (step, patch), then the inner records of the mixed form (shared by the steps)
  ensure_scalars(c, n_steps * np + np);
  if (mixed) ensure_workspace32(c, B.n_slots);
  PcgScalars* sc_inner = c->sc + int64_t(n_steps) * np;
  CouplingParams cp{};
  cp.T = nullptr;
  const CellKParams kp{1, 1.0, 1.0, 1.0};
  const FaceCoefs<double> Aop = face_coefs(c, B.Cp, B.K, B.mask, 1.0, 1.0, true);
  const int max_outer = c->o.max_outer > 0 ? c->o.max_outer : 30;
  auto record = [&](hipStream_t st) -> hipError_t {
    launch_zero_u32(st, c->bar, kBarWords);
    for (int step = 0; step < n_steps; ++step) {
      PcgScalars* sc = c->sc + int64_t(step) * np;
      launch_cell_K(st, D, B.E, B.rho, nullptr, kp, OuterBC{}, B.K);
      launch_assemble(st, D, B.K, nullptr, B.E, nullptr, B.rho, nullptr, 1.0, 1.0, c->o.robin_alpha, cp, kp,
                      OuterBC{}, B.Cp, B.mask, B.diag, B.b);
      const ScaledOp<double> Ah = scale_operator(c, st, D, Aop, B.Cp, B.diag, B.rs, B.Ch);
      const SolveArrays A{Aop, B.diag, B.b, B.E, B.n_slots, Ah};
      launch_init_scalars(st, sc, np, tol, c->o.abs_floor, c->o.max_iter, c->o.linf_test);
      launch_zero_u32(st, c->bar, kBarAbort);
      hipError_t e;
      if (mixed) {
        const ScaledOp<float> A32 = operator_f32(c, st, A);
        launch_init_scalars(st, sc_inner, np, c->o.inner_tol, 0.0, c->o.max_iter, 0);
        // the batch's FP32 sweeps keep its FP64 plan (16 tiles per block)
        e = launch_mixed_persistent(st, D, P, P, mixed_args(c, A, A32, sc, sc_inner, max_outer), per_cu);
      } else {
        cg_start(c, st, D, P, A, sc);
        e = launch_pcg_persistent<double>(st, D, P, c->o.max_iter, Ah, c->cg, B.E, sc, c->partials, c->bar, per_cu);
      }
      if (e != hipSuccess) return e;
      if (c->o.true_residual && !mixed) launch_true_residual(st, D, P, Ah, B.b, B.E, sc, c->partials);
      launch_post_solve(st, D, P, B.E, B.rho, cp, 0.0, nullptr, sc, c->partials);
    }
    return hipGetLastError();
  };
  const hipStream_t us = c->stream();
  int mode = c->o.graph ? 2 : 1;
  float total_ms = 0.f;
  if (mode == 2) {
    if (!c->cap_stream) check(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "stream");
    for (auto& e : c->cap_ev)
      if (!e) check(hipEventCreate(&e), "event");
    check(hipEventRecord(c->cap_ev[0], us), "event");
    check(hipStreamWaitEvent(c->cap_stream, c->cap_ev[0], 0), "event");
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    hipError_t e_rec = e == hipSuccess ? record(c->cap_stream) : e;
    hipError_t e_end = e == hipSuccess ? hipStreamEndCapture(c->cap_stream, &g) : e;
    hipGraphExec_t ex = nullptr;
    if (e_rec == hipSuccess && e_end == hipSuccess && g)
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    else
      e = hipErrorNotSupported;
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      mode = 1;
    } else {
      check(hipEventRecord(c->cap_ev[0], c->cap_stream), "event");
      check(hipGraphLaunch(ex, c->cap_stream), "graph launch");
      check(hipEventRecord(c->cap_ev[1], c->cap_stream), "event");
      check(hipStreamSynchronize(c->cap_stream), "graph");
      check(hipEventElapsedTime(&total_ms, c->cap_ev[0], c->cap_ev[1]), "event");
      (void)hipGraphExecDestroy(ex);
      (void)hipGraphDestroy(g);
    }
  }
  if (mode == 1) {
    check(hipEventRecord(c->ev[0], us), "event");
    check(record(us), "persistent launch");
    check(hipEventRecord(c->ev[3], us), "event");
    check(hipStreamSynchronize(us), "sync");
    check(hipEventElapsedTime(&total_ms, c->ev[0], c->ev[3]), "event");
  }
  unsigned aborted = 0;
  check(hipMemcpy(&aborted, abort_flag, sizeof(unsigned), hipMemcpyDeviceToHost), "abort flag");
  read_scalars(c, c->h_sc, c->sc, n_steps * np);
  amrfld_status worst = AMRFLD_OK;
  std::string worst_msg;
  for (int step = 0; step < n_steps; ++step) {
    for (int q = 0; q < np; ++q) {
      const PcgScalars& h = c->h_sc[int64_t(step) * np + q];
      amrfld_stats st{};
      st.level = q;
      st.iters = mixed ? h.inner_total : h.iter;
      st.outer_iters = mixed ? h.iter : 0;
      st.converged = h.converged;
      st.n_leaf = int64_t(B.sizes[q]) * B.sizes[q] * B.sizes[q];
      st.rel_res = h.rnorm0 > 0 ? h.rnorm / h.rnorm0 : 0.0;
      st.true_rel_res =
          mixed ? st.rel_res : (c->o.true_residual ? (h.rnorm0 > 0 ? h.true_rnorm / h.rnorm0 : 0.0) : -1.0);
      st.linf_change = h.linf;
      st.min_E = h.min_E;
      st.dt = pt[q].dt;
      st.ms = total_ms / n_steps;
      st.pcg_ms = -1.0;
      st.launch_mode = mode;
      st.rnorm0 = h.rnorm0;
      st.bnorm = h.bnorm;
      st.sweep_blocks = P.G;
      st.launch_blocks = mixed ? mixed_persistent_blocks(P, P, per_cu) : persistent_blocks<double>(P, per_cu);
      st.status = h.nonfinite ? AMRFLD_E_NONFINITE : (h.converged ? AMRFLD_OK : AMRFLD_E_NOCONV);
      if (st.status != AMRFLD_OK && worst == AMRFLD_OK) {
        worst = amrfld_status(st.status);
        worst_msg = "patch " + std::to_string(q) + " step " + std::to_string(step) +
                    (st.status == AMRFLD_E_NONFINITE ? ": non-finite residual" : ": no convergence");
      }
      c->stats.push_back(st);
    }
  }
  if (aborted) return fail(c, AMRFLD_E_DEVICE, "persistent sweep: a grid barrier timed out");
  if (worst != AMRFLD_OK) return fail(c, worst, worst_msg);
  return AMRFLD_OK;
}

amrfld_status solve_batch(amrfld_ctx* c, const std::vector<amrfld_patch>& pt, int n_steps, double tol,
                          int precision) {
  const hipStream_t s = c->stream();
  std::vector<int> sizes(pt.size());
  for (size_t q = 0; q < pt.size(); ++q) sizes[q] = pt[q].n;
  build_batch(c, sizes);
  BatchState& B = *c->batch;
  const int np = B.n_prob;
  std::vector<PatchParams> pp(np);
  for (int q = 0; q < np; ++q) {
    PatchParams& P = pp[q];
    P.dx = pt[q].dx;
    P.vol = pt[q].dx * pt[q].dx * pt[q].dx;
    P.coef = pt[q].dt / (pt[q].dx * pt[q].dx);
    P.kappa_R = pt[q].kappa_R;
    P.c_light = pt[q].c_light;
    P.K_const = pt[q].K_const;
    P.kmode = pt[q].kmode;
    for (int d = 0; d < 6; ++d) {
      P.mode[d] = pt[q].face_mode[d];
      P.ghost[d] = pt[q].face_ghost[d];
      P.flux[d] = pt[q].face_flux[d];
    }
  }
  check(hipMemcpyAsync(B.pp, pp.data(), np * sizeof(PatchParams), hipMemcpyHostToDevice, s), "batch params");
  const DevLevel D = B.dev();
  std::vector<const double*> ptr(np);
  for (int q = 0; q < np; ++q) ptr[q] = pt[q].rho;
  check(hipMemcpyAsync(B.src, ptr.data(), np * sizeof(void*), hipMemcpyHostToDevice, s), "batch pointers");
  launch_batch_gather(s, D, B.idx, B.src, 1.0, B.rho);
  check(hipStreamSynchronize(s), "batch gather");  // the pointer array is reused next
  for (int q = 0; q < np; ++q) ptr[q] = pt[q].E;
  check(hipMemcpyAsync(B.src, ptr.data(), np * sizeof(void*), hipMemcpyHostToDevice, s), "batch pointers");
  launch_batch_gather(s, D, B.idx, B.src, 0.0, B.E);
  ensure_workspace(c, B.n_slots);
  if (c->o.persistent) {
    const amrfld_status st = solve_batch_persistent(c, pt, n_steps, tol, precision);
    if (st != AMRFLD_E_STATE) return st;
    c->stats.clear();  // the device cannot run it: poll instead
  }
  ensure_scalars(c, np);
  const SweepPlan P = B.plan();
  // the batch's precision for this call only, restored on every way out
  struct PrecisionScope {
    amrfld_opts& o;
    int saved;
    ~PrecisionScope() { o.precision = saved; }
  } scope{c->o, c->o.precision};
  c->o.precision = precision;
  amrfld_status worst = AMRFLD_OK;
  std::string worst_msg;
  int hint = 0;  // the previous step's longest FP64 solve (first batch of sweeps of the next)
  for (int step = 0; step < n_steps; ++step) {
    check(hipEventRecord(c->ev[0], s), "event");
    const CellKParams kp{1, 1.0, 1.0, 1.0};
    launch_cell_K(s, D, B.E, B.rho, nullptr, kp, OuterBC{}, B.K);
    CouplingParams cp{};
    cp.T = nullptr;
    launch_assemble(s, D, B.K, nullptr, B.E, nullptr, B.rho, nullptr, 1.0, 1.0, c->o.robin_alpha, cp, kp,
                    OuterBC{}, B.Cp, B.mask, B.diag, B.b);
    LoopStats ls;
    ls.iters.assign(np, 0);
    const FaceCoefs<double> Aop = face_coefs(c, B.Cp, B.K, B.mask, 1.0, 1.0, true);
    const ScaledOp<double> Ah = scale_operator(c, s, D, Aop, B.Cp, B.diag, B.rs, B.Ch);
    const SolveArrays A{Aop, B.diag, B.b, B.E, B.n_slots, Ah};
    if (precision == AMRFLD_MIXED) {
      pcg_mixed(c, D, P, P, A, tol, &ls);  // one plan for the batch's FP64 and FP32 sweeps
    } else {
      pcg_fp64(c, D, P, A, tol, &ls, hint);
      hint = *std::max_element(ls.iters.begin(), ls.iters.end());
    }
    check(hipEventRecord(c->ev[2], s), "event");
    if (c->o.true_residual && precision != AMRFLD_MIXED)
      launch_true_residual(s, D, P, Ah, B.b, B.E, c->sc, c->partials);
    launch_post_solve(s, D, P, B.E, B.rho, cp, 0.0, nullptr, c->sc, c->partials);
    check(hipEventRecord(c->ev[3], s), "event");
    read_scalars(c, c->h_sc, c->sc, np);
    check(hipGetLastError(), "kernels");
    float ms = 0.f, pms = 0.f;
    check(hipEventSynchronize(c->ev[3]), "event");  // passed already: the scalars were read after it
    check(hipEventElapsedTime(&ms, c->ev[0], c->ev[3]), "event");
    check(hipEventElapsedTime(&pms, c->ev[1], c->ev[2]), "event");
    for (int q = 0; q < np; ++q) {
      const PcgScalars& h = c->h_sc[q];
      amrfld_stats st{};
      st.level = q;
      st.iters = precision == AMRFLD_MIXED ? h.inner_total : ls.iters[q];
      st.outer_iters = precision == AMRFLD_MIXED ? h.iter : 0;
      st.converged = h.converged;
      st.n_leaf = int64_t(sizes[q]) * sizes[q] * sizes[q];
      st.rel_res = h.rnorm0 > 0 ? h.rnorm / h.rnorm0 : 0.0;
      st.true_rel_res = precision == AMRFLD_MIXED ? st.rel_res
                        : (c->o.true_residual ? (h.rnorm0 > 0 ? h.true_rnorm / h.rnorm0 : 0.0) : -1.0);
      st.linf_change = h.linf;
      st.min_E = h.min_E;
      st.dt = pt[q].dt;
      st.ms = ms;
      st.pcg_ms = pms;
      st.n_timed = ls.n_timed;
      st.sweep_ms = ls.sweep_ms;
      st.spare_ms = 0.0;
      st.rnorm0 = h.rnorm0;
      st.bnorm = h.bnorm;
      st.sweep_blocks = P.G;
      st.launch_blocks = ls.persistent ? ls.launch_blocks : P.G;
      st.launch_mode = ls.persistent ? 1 : 0;
      st.status = h.nonfinite ? AMRFLD_E_NONFINITE : (h.converged ? AMRFLD_OK : AMRFLD_E_NOCONV);
      if (st.status != AMRFLD_OK && worst == AMRFLD_OK) {
        worst = amrfld_status(st.status);
        worst_msg = "patch " + std::to_string(q) + " step " + std::to_string(step) +
                    (st.status == AMRFLD_E_NONFINITE ? ": non-finite residual" : ": no convergence");
      }
      c->stats.push_back(st);
    }
    if (worst == AMRFLD_E_NONFINITE) break;
  }
  if (worst != AMRFLD_OK) return fail(c, worst, worst_msg);
  return AMRFLD_OK;
}

// The level solve with its PCG workspace (r, both p buffers, q, block partials,
// the scalar record, the barrier words) in the device scratch array instead of the
// context's workspace, which it neither grows nor frees.  The context's pointers are
// swapped for the duration of the call and restored on every way out; allocations
// are refused meanwhile (g_no_alloc).
amrfld_status solve_one_noalloc(amrfld_ctx* c, double* scr, int level, double dt, int mode, double tol) {
  struct Swap {
    amrfld_ctx* c;
    CgVecs<double> cg;
    double* partials;
    int64_t ws_n, partial_n;
    PcgScalars* sc;
    unsigned* bar;
    int time_sweeps;
    ~Swap() {
      c->cg = cg;
      c->partials = partials;
      c->ws_n = ws_n;
      c->partial_n = partial_n;
      c->sc = sc;
      c->bar = bar;
      c->o.time_sweeps = time_sweeps;
      g_no_alloc = false;
    }
  } keep{c, c->cg, c->partials, c->ws_n, c->partial_n, c->sc, c->bar, c->o.time_sweeps};
  double** vec[kScratchVectors] = {&c->cg.r[0], &c->cg.r[1], &c->cg.w[0], &c->cg.w[1], &c->cg.s[0], &c->cg.s[1],
                                   &c->cg.p};
  for (int k = 0; k < kScratchVectors; ++k) *vec[k] = scr + k * kScratchSlots;
  c->partials = scr + kScratchOffPartials;
  c->ws_n = kScratchSlots;
  c->partial_n = kScratchPartials;
  c->sc = reinterpret_cast<PcgScalars*>(scr + kScratchOffScalars);
  c->bar = reinterpret_cast<unsigned*>(scr + kScratchOffBar);
  c->o.time_sweeps = 0;  // sweep timing would create events
  g_no_alloc = true;
  return solve_one(c, level, dt, mode, tol);
}

}  // namespace

extern "C" {

void amrfld_default_opts(amrfld_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->base_level = 1;
  o->max_level = 1;
  o->robin_alpha = 0.5;
  o->max_iter = 10000;
  o->precision = AMRFLD_FP64;
  o->linf_test = 1;
  o->abs_floor = 1e-14;
  o->a_rad = 1.0;
  o->c_v = 1.0;
  o->check_every = 0;
  o->true_residual = 1;
  o->inner_tol = 3e-3;
  o->max_outer = 30;
  o->max_blocks = 0;
  o->stream = nullptr;
  o->theta = 1.0;
}

const char* amrfld_create_error(void) { return g_create_error.c_str(); }

amrfld_status amrfld_create(const amrfld_opts* o, amrfld_ctx** out) {
  g_create_error.clear();
  if (!o || !out) {
    g_create_error = "NULL argument";
    return AMRFLD_E_INVALID;
  }
  *out = nullptr;
  if (o->base_level < 1 || o->max_level < o->base_level || o->max_level > 20) {
    g_create_error = "levels must satisfy 1 <= base_level <= max_level <= 20";
    return AMRFLD_E_INVALID;
  }
  if (!(o->robin_alpha >= 0.0 && o->robin_alpha <= 1.0)) {
    g_create_error = "robin_alpha must be in [0, 1]";
    return AMRFLD_E_INVALID;
  }
  if (o->max_iter < 1 || !(o->abs_floor >= 0.0) || o->precision < 0 || o->precision > 1) {
    g_create_error = "max_iter >= 1, abs_floor >= 0 and a known precision are required";
    return AMRFLD_E_INVALID;
  }
  if (o->max_blocks < 0 || o->persistent_per_cu < 0) {
    g_create_error = "max_blocks and persistent_per_cu must be >= 0";
    return AMRFLD_E_INVALID;
  }
  if (!(o->theta >= 0.5 && o->theta <= 1.0)) {
    g_create_error = "theta must be in [0.5, 1]";
    return AMRFLD_E_INVALID;
  }
  if (!std::isfinite(o->K_exp)) {
    g_create_error = "K_exp must be finite";
    return AMRFLD_E_INVALID;
  }
  for (int d = 0; d < 6; ++d)
    if ((o->outer_mode[d] != 0 && o->outer_mode[d] != 1) || (o->outer_mode[d] == 1 && !std::isfinite(o->outer_value[d]))) {
      g_create_error = "outer_mode must be 0 or 1, with a finite outer_value where it is 1";
      return AMRFLD_E_INVALID;
    }
  amrfld_ctx* c = nullptr;
  try {
    c = new amrfld_ctx();
    c->o = *o;
    c->lev.resize(o->max_level - o->base_level + 1);
    check(hipGetDevice(&c->device), "device");
    resolve_scratch(c->device);
    ensure_scalars(c, 1);
    for (auto& e : c->ev) check(hipEventCreate(&e), "event");
    c->stats.reserve(64);
  } catch (const std::exception& e) {
    g_create_error = e.what();
    amrfld_destroy(c);
    return AMRFLD_E_DEVICE;
  }
  *out = c;
  return AMRFLD_OK;
}

void amrfld_destroy(amrfld_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream());
  c->step_graph.reset();
  for (auto& L : c->lev) L.release();
  if (c->batch) {
    c->batch->release();
    delete c->batch;
  }
  if (c->comp) {
    c->comp->release();
    delete c->comp;
  }
  dfree(c->bar);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto& e : c->cap_ev)
    if (e) (void)hipEventDestroy(e);
  free_vecs(c->cg);
  free_vecs(c->cg32);
  for (void* p : {(void*)c->partials, (void*)c->sc, (void*)c->Ch32, (void*)c->K32, (void*)c->rs32, (void*)c->r32,
                  (void*)c->d32, (void*)c->x_alt})
    dfree(p);
  if (c->h_sc) (void)hipHostFree(c->h_sc);
  if (c->h_seq) (void)hipHostFree(c->h_seq);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->sweep_ev) (void)hipEventDestroy(e);
  delete c;
}

amrfld_status amrfld_build_level(amrfld_ctx* c, int level, int64_t n_oct, const int32_t* oct_ijk) {
  if (!c) return AMRFLD_E_INVALID;
  ++c->param_epoch;
  if (!oct_ijk) return fail(c, AMRFLD_E_INVALID, "oct_ijk is NULL");
  const int expect = c->finest < 0 ? c->o.base_level : c->finest + 1;
  if (level != expect)
    return fail(c, AMRFLD_E_INVALID, "levels must be built base first, one finer level at a time (expected level " +
                                          std::to_string(expect) + ")");
  if (level > c->o.max_level) return fail(c, AMRFLD_E_INVALID, "level above max_level");
  return guarded(c, [&]() -> amrfld_status {
    LevelTables t;
    const bool base = level == c->o.base_level;
    LevelTables* coarser = base ? nullptr : &c->L(level - 1).t;
    // validate against a copy so that a rejected level leaves the coarser tables untouched
    LevelTables coarse_copy;
    if (coarser) coarse_copy = *coarser;
    const std::string why = build_level_tables(level, base, n_oct, oct_ijk, coarser ? &coarse_copy : nullptr, &t);
    if (!why.empty()) return fail(c, AMRFLD_E_INVALID, why);
    // the level's device arrays and tables first: a failure leaves the context as it was
    LevelState fresh;
    fresh.t = std::move(t);
    const int64_t n = fresh.t.n_slots();
    try {
      fresh.rho = dalloc<double>(n, "fields");
      fresh.E = dalloc<double>(n, "fields");
      fresh.K = dalloc<double>(n, "fields");
      fresh.Cp = dalloc<double>(3 * n, "fields");
      fresh.mask = dalloc<uint8_t>(n, "fields");
      fresh.diag = dalloc<double>(n, "fields");
      fresh.b = dalloc<double>(n, "fields");
      fresh.Ch = dalloc<double>(3 * n, "fields");
      fresh.rs = dalloc<double>(n, "fields");
      upload_tables(c, fresh);
    } catch (...) {
      (void)hipStreamSynchronize(c->stream());
      fresh.release();
      throw;
    }
    if (coarser) {
      *coarser = std::move(coarse_copy);
      c->L(level - 1).child_dirty = true;
    }
    if (c->comp) {  // the composite slot space no longer matches the levels
      c->comp->release();
      delete c->comp;
      c->comp = nullptr;
    }
    LevelState& L = c->L(level);
    L.release();
    L = std::move(fresh);
    c->finest = level;
    if (coarser) upload_tables(c, c->L(level - 1));  // its child table (allocated with that level)
    return AMRFLD_OK;
  });
}

amrfld_status amrfld_level_info(const amrfld_ctx* c, int level, int64_t* n_slots, int64_t* n_leaf,
                                int32_t* cell_ijk_out) {
  if (!c) return AMRFLD_E_INVALID;
  amrfld_ctx* m = const_cast<amrfld_ctx*>(c);
  if (level < c->o.base_level || level > c->finest) return fail(m, AMRFLD_E_INVALID, "level not built");
  const LevelState& L = c->L(level);
  if (n_slots) *n_slots = L.t.n_slots();
  if (n_leaf) *n_leaf = L.t.n_leaf;
  if (cell_ijk_out) {
    for (int64_t o = 0; o < L.t.n_oct; ++o)
      for (int pos = 0; pos < 8; ++pos) {
        int32_t* p = cell_ijk_out + 3 * (8 * o + pos);
        p[0] = 2 * L.t.ijk[3 * o] + (pos & 1);
        p[1] = 2 * L.t.ijk[3 * o + 1] + ((pos >> 1) & 1);
        p[2] = 2 * L.t.ijk[3 * o + 2] + ((pos >> 2) & 1);
      }
  }
  return AMRFLD_OK;
}

amrfld_status amrfld_set_coeffs(amrfld_ctx* c, int level, const double* rho, const double* E,
                                const double* T, double kappa_R, double kappa_P, double c_light,
                                int kmode, double K_const) {
  if (!c) return AMRFLD_E_INVALID;
  if (level < c->o.base_level || level > c->finest) return fail(c, AMRFLD_E_INVALID, "level not built");
  if (!rho || !E) return fail(c, AMRFLD_E_INVALID, "rho and E are required");
  if (kmode != AMRFLD_K_CONST && kmode != AMRFLD_K_LP && kmode != AMRFLD_K_MINERBO && kmode != AMRFLD_K_POWER)
    return fail(c, AMRFLD_E_INVALID, "unknown kmode");
  if ((kmode == AMRFLD_K_LP || kmode == AMRFLD_K_MINERBO) && !(kappa_R > 0.0 && c_light > 0.0))
    return fail(c, AMRFLD_E_INVALID, "kappa_R and c_light must be positive");
  if ((kmode == AMRFLD_K_CONST || kmode == AMRFLD_K_POWER) && !(K_const >= 0.0 && std::isfinite(K_const)))
    return fail(c, AMRFLD_E_INVALID, "K_const must be finite and >= 0");
  if (T && !(kappa_P >= 0.0 && c_light > 0.0)) return fail(c, AMRFLD_E_INVALID, "kappa_P >= 0 and c_light > 0 needed with T");
  if (!device_ptr(rho) || !device_ptr(E) || (T && !device_ptr(T)))
    return fail(c, AMRFLD_E_INVALID, "rho, E and T must be device arrays");
  return guarded(c, [&]() -> amrfld_status {
    LevelState& L = c->L(level);
    const int64_t n = L.t.n_slots();
    const hipStream_t s = c->stream();
    launch_copy_f64(s, L.rho, rho, n);
    launch_copy_f64(s, L.E, E, n);
    if (T) {
      if (!L.T) L.T = dalloc<double>(n, "fields");
      launch_copy_f64(s, L.T, T, n);
    }
    L.has_T = T != nullptr;
    L.kmode = kmode;
    L.K_const = K_const;
    L.kappa_R = kappa_R;
    L.kappa_P = kappa_P;
    L.c_light = c_light;
    L.K_exp = c->o.K_exp;
    L.has_fields = true;
    ++c->param_epoch;
    return AMRFLD_OK;
  });
}

amrfld_status amrfld_solve_level(amrfld_ctx* c, int level, double dt, int bc_mode, double tol) {
  if (!c) return AMRFLD_E_INVALID;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, AMRFLD_E_INVALID, "dt must be positive");
  if (bc_mode < 0 || bc_mode > 2) return fail(c, AMRFLD_E_INVALID, "unknown bc_mode");
  if (!(tol >= 0.0)) return fail(c, AMRFLD_E_INVALID, "tol must be >= 0");
  const amrfld_status r = check_level_ready(c, level);
  if (r != AMRFLD_OK) return r;
  const amrfld_status rt = check_theta(c, bc_mode);
  if (rt != AMRFLD_OK) return rt;
  c->stats.clear();
  return guarded(c, [&]() { return solve_one(c, level, dt, bc_mode, tol); });
}

amrfld_status amrfld_solve_level_noalloc(amrfld_ctx* c, int level, double dt, int bc_mode, double tol) {
  if (!c) return AMRFLD_E_INVALID;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, AMRFLD_E_INVALID, "dt must be positive");
  if (bc_mode < 0 || bc_mode > 2) return fail(c, AMRFLD_E_INVALID, "unknown bc_mode");
  if (!(tol >= 0.0)) return fail(c, AMRFLD_E_INVALID, "tol must be >= 0");
  if (level < c->o.base_level || level > c->finest) return fail(c, AMRFLD_E_INVALID, "level not built");
  if (c->L(level).t.n_slots() > kScratchSlots)
    return fail(c, AMRFLD_E_INVALID, "no-allocation solve: the level has " + std::to_string(c->L(level).t.n_slots()) +
                                         " slots, above the scratch limit of " + std::to_string(kScratchSlots));
  if (c->o.precision != AMRFLD_FP64)
    return fail(c, AMRFLD_E_INVALID, "no-allocation solve: FP64 only (the mixed form needs FP32 workspace)");
  const amrfld_status r = check_level_ready(c, level);
  if (r != AMRFLD_OK) return r;
  const amrfld_status rt = check_theta(c, bc_mode);
  if (rt != AMRFLD_OK) return rt;
  if (level > c->o.base_level && bc_mode != AMRFLD_BC_DIRICHLET && !c->L(level - 1).reg)
    return fail(c, AMRFLD_E_STATE, "no-allocation solve: the coarser level has no flux register yet (one "
                                   "amrfld_solve_level call in Neumann or Robin mode creates it)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) {
    (void)hipGetLastError();
    return fail(c, AMRFLD_E_STATE, "no-allocation solve: the context's device is not current");
  }
  std::string why;
  double* scr = scratch_of(dev, &why);
  if (!scr) return fail(c, AMRFLD_E_DEVICE, why);
  c->stats.clear();
  return guarded(c, [&]() { return solve_one_noalloc(c, scr, level, dt, bc_mode, tol); });
}

amrfld_status amrfld_restrict_level(amrfld_ctx* c, int fine_level) {
  if (!c) return AMRFLD_E_INVALID;
  if (fine_level <= c->o.base_level || fine_level > c->finest)
    return fail(c, AMRFLD_E_INVALID, "fine_level must be a built level above the base level");
  if (!c->L(fine_level).has_fields || !c->L(fine_level - 1).has_fields)
    return fail(c, AMRFLD_E_STATE, "fields of both levels must be set");
  return guarded(c, [&]() -> amrfld_status {
    LevelState& F = c->L(fine_level);
    upload_tables(c, F);
    launch_restrict(c->stream(), F.dev(), F.E, c->L(fine_level - 1).E);
    check(hipGetLastError(), "restrict");
    return AMRFLD_OK;
  });
}

amrfld_status amrfld_advance_subcycled(amrfld_ctx* c, double dt_coarse, int bc_mode, double tol) {
  if (!c) return AMRFLD_E_INVALID;
  if (!(dt_coarse > 0.0) || !std::isfinite(dt_coarse)) return fail(c, AMRFLD_E_INVALID, "dt must be positive");
  if (bc_mode < 0 || bc_mode > 2) return fail(c, AMRFLD_E_INVALID, "unknown bc_mode");
  if (!(tol >= 0.0)) return fail(c, AMRFLD_E_INVALID, "tol must be >= 0");
  if (c->finest < 0) return fail(c, AMRFLD_E_STATE, "no level built");
  for (int l = c->o.base_level; l <= c->finest; ++l) {
    const amrfld_status r = check_level_ready(c, l);
    if (r != AMRFLD_OK) return r;
  }
  const amrfld_status rt = check_theta(c, bc_mode);
  if (rt != AMRFLD_OK) return rt;
  c->stats.clear();
  return guarded(c, [&]() {
    const amrfld_status g = advance_graph(c, dt_coarse, bc_mode, tol);
    if (g != AMRFLD_E_STATE) return g;
    return step(c, c->o.base_level, dt_coarse, bc_mode, tol);
  });
}

amrfld_status amrfld_advance_unique(amrfld_ctx* c, double dt_coarse, double tol) {
  if (!c) return AMRFLD_E_INVALID;
  if (!(dt_coarse > 0.0) || !std::isfinite(dt_coarse)) return fail(c, AMRFLD_E_INVALID, "dt must be positive");
  if (!(tol >= 0.0)) return fail(c, AMRFLD_E_INVALID, "tol must be >= 0");
  if (c->finest < 0) return fail(c, AMRFLD_E_STATE, "no level built");
  for (int l = c->o.base_level; l <= c->finest; ++l) {
    const amrfld_status r = check_level_ready(c, l);
    if (r != AMRFLD_OK) return r;
  }
  if (c->o.theta != 1.0) return fail(c, AMRFLD_E_INVALID, "the unique-time-step solve is backward Euler (theta = 1)");
  c->stats.clear();
  return guarded(c, [&]() { return advance_unique(c, dt_coarse, tol); });
}

amrfld_status amrfld_solve_batch(amrfld_ctx* c, int n_prob, const amrfld_patch* patches, int n_steps,
                                 double tol, int precision, double* E_out) {
  if (!c) return AMRFLD_E_INVALID;
  if (n_prob < 1 || !patches || !E_out) return fail(c, AMRFLD_E_INVALID, "n_prob >= 1, patches and E_out are required");
  if (!device_ptr(E_out)) return fail(c, AMRFLD_E_INVALID, "E_out must be a device array");
  if (n_steps < 1) return fail(c, AMRFLD_E_INVALID, "n_steps must be >= 1");
  if (!(tol >= 0.0)) return fail(c, AMRFLD_E_INVALID, "tol must be >= 0");
  if (precision != AMRFLD_FP64 && precision != AMRFLD_MIXED) return fail(c, AMRFLD_E_INVALID, "unknown precision");
  if (c->o.theta != 1.0) return fail(c, AMRFLD_E_INVALID, "the batch form is backward Euler (theta = 1)");
  std::vector<amrfld_patch> pt(patches, patches + n_prob);
  for (int q = 0; q < n_prob; ++q) {
    const amrfld_patch& p = pt[q];
    const std::string at = "patch " + std::to_string(q) + ": ";
    if (p.n < 2 || p.n > 1024 || (p.n & 1)) return fail(c, AMRFLD_E_INVALID, at + "n must be even, 2..1024");
    if (!(p.dx > 0.0) || !(p.dt > 0.0)) return fail(c, AMRFLD_E_INVALID, at + "dx and dt must be positive");
    if (!p.rho || !p.E) return fail(c, AMRFLD_E_INVALID, at + "rho and E are required");
    if (!device_ptr(p.rho) || !device_ptr(p.E)) return fail(c, AMRFLD_E_INVALID, at + "rho and E must be device arrays");
    if (p.kmode != AMRFLD_K_CONST && p.kmode != AMRFLD_K_LP && p.kmode != AMRFLD_K_MINERBO)
      return fail(c, AMRFLD_E_INVALID, at + "unknown kmode");
    if (p.kmode != AMRFLD_K_CONST && !(p.kappa_R > 0.0 && p.c_light > 0.0))
      return fail(c, AMRFLD_E_INVALID, at + "kappa_R and c_light must be positive");
    for (int d = 0; d < 6; ++d)
      if (p.face_mode[d] < 0 || p.face_mode[d] > 2) return fail(c, AMRFLD_E_INVALID, at + "unknown face mode");
  }
  c->stats.clear();
  return guarded(c, [&]() -> amrfld_status {
    const amrfld_status st = solve_batch(c, pt, n_steps, tol, precision);
    if (st == AMRFLD_OK || st == AMRFLD_E_NOCONV) {
      BatchState& B = *c->batch;
      launch_batch_scatter(c->stream(), B.dev(), B.idx, B.d_out_off, B.E, E_out);
      check(hipGetLastError(), "scatter");
    }
    return st;
  });
}

amrfld_status amrfld_get_E(const amrfld_ctx* c, int level, double* E_out, double* T_out) {
  if (!c) return AMRFLD_E_INVALID;
  amrfld_ctx* m = const_cast<amrfld_ctx*>(c);
  if (level < c->o.base_level || level > c->finest) return fail(m, AMRFLD_E_INVALID, "level not built");
  if (!E_out && !T_out) return fail(m, AMRFLD_E_INVALID, "no output");
  const LevelState& L = c->L(level);
  if (T_out && !L.has_T) return fail(m, AMRFLD_E_STATE, "level has no temperature");
  if ((E_out && !device_ptr(E_out)) || (T_out && !device_ptr(T_out)))
    return fail(m, AMRFLD_E_INVALID, "E_out and T_out must be device arrays");
  return guarded(m, [&]() -> amrfld_status {
    const int64_t n = L.t.n_slots();
    if (E_out) launch_copy_f64(c->stream(), E_out, L.E, n);
    if (T_out) launch_copy_f64(c->stream(), T_out, L.T, n);
    return AMRFLD_OK;
  });
}

amrfld_status amrfld_last_stats(const amrfld_ctx* c, amrfld_stats* out, int max_n, int* n) {
  if (!c) return AMRFLD_E_INVALID;
  const int cnt = int(c->stats.size());
  if (n) *n = cnt;
  if (out)
    for (int k = 0; k < std::min(cnt, max_n); ++k) out[k] = c->stats[k];
  return AMRFLD_OK;
}

amrfld_status amrfld_set_launch(amrfld_ctx* c, int max_blocks, int persistent, int persistent_per_cu,
                                int form_coefs) {
  if (!c) return AMRFLD_E_INVALID;
  if (max_blocks < 0 || persistent < 0 || persistent_per_cu < 0 || form_coefs < 0) {
    c->err = "set_launch: negative launch parameter";
    return AMRFLD_E_INVALID;
  }
  c->o.max_blocks = max_blocks;
  c->o.persistent = persistent ? 1 : 0;
  c->o.persistent_per_cu = persistent_per_cu;
  c->o.form_coefs = form_coefs ? 1 : 0;
  ++c->param_epoch;
  c->err.clear();
  return AMRFLD_OK;
}

amrfld_status amrfld_set_refinement(amrfld_ctx* c, double inner_tol, int max_outer) {
  if (!c) return AMRFLD_E_INVALID;
  if (!(inner_tol > 0.0 && inner_tol < 1.0) || max_outer < 1) {
    c->err = "set_refinement: inner_tol in (0, 1) and max_outer >= 1 are required";
    return AMRFLD_E_INVALID;
  }
  c->o.inner_tol = inner_tol;
  c->o.max_outer = max_outer;
  ++c->param_epoch;
  c->err.clear();
  return AMRFLD_OK;
}

const char* amrfld_last_error(const amrfld_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

}  // extern "C"
