// Device helpers shared by the setup and PCG kernels.
//
// Layout: a level's cells are "slots", 8 per oct, octs in Morton order, x
// fastest inside an oct, so slot i lives in oct i >> 3 at position i & 7 and
// its in-oct face neighbour along axis a is slot i ^ (1 << a).  A 64-wide
// wavefront therefore holds 8 whole octs and in-oct neighbours are exchanged
// with cross-lane shuffles; the three faces of a cell that leave its oct go
// through the per-oct neighbour table.
//
// The operator is stored symmetric: Cp[a][i] is the coefficient of the face
// between slot i and its +a neighbour when both are leaves of the level and
// zero otherwise; the -a face of slot i is Cp[a] of the -a neighbour.  Refined
// slots carry an identity row (diag 1, all coefficients 0, r = 0), so sweeps run
// over every slot without branching on the cell type.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>

#include "device.h"

namespace amrfld {
namespace dev {

__device__ __forceinline__ int same_level_nb(const int32_t* __restrict__ nbr, int i, int dir) {
  const int pos = i & 7, axis = dir >> 1, side = dir & 1, bit = 1 << axis;
  if (((pos >> axis) & 1) != side) return i ^ bit;
  const int n = nbr[(i >> 3) * 6 + dir];
  return n < 0 ? -1 : ((n << 3) | (pos ^ bit));
}

template <typename T>
__device__ __forceinline__ T harmonic(T a, T b) {
  const T s = a + b;
  return s != T(0) ? (T(2) * a * b) / s : T(0);
}

// Coefficient of a face formed from the diffusivities of its two cells (the
// assembly's expression; harmonic is symmetric bit for bit).
template <typename T>
__device__ __forceinline__ T face_coef(T Ki, T Kj, T scale, T theta) {
  T c = harmonic(Ki, Kj) * scale;
  if (theta != T(1)) c *= theta;
  return c;
}

// Coefficient of a face of the Jacobi-scaled operator formed from the two cells'
// diffusivities and scale factors: the assembly's coefficient times rs_i rs_j (the
// stored scaled coefficients are computed with the same expression).
template <typename T>
__device__ __forceinline__ T scaled_face(T Ki, T Kj, T rsi, T rsj, T scale, T theta) {
  return face_coef(Ki, Kj, scale, theta) * (rsi * rsj);
}

// dt / dx^2 of problem `prob` of a solve.
template <typename T>
__device__ __forceinline__ T coef_scale(const FaceCoefs<T>& A, const DevLevel& L, int prob) {
  return T(A.per_problem ? L.pp[prob].coef : A.scale);
}
template <typename T>
__device__ __forceinline__ T coef_scale(const ScaledOp<T>& A, const DevLevel& L, int prob) {
  return T(A.per_problem ? L.pp[prob].coef : A.scale);
}

// Block-wide reduction; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const bool (&is_max)[NV], double* lds) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_down(v[k], off, 64);
      v[k] = is_max[k] ? fmax(v[k], o) : v[k] + o;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[wid * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = lds[k];
      for (int w = 1; w < kBlock / 64; ++w) t = is_max[k] ? fmax(t, lds[w * NV + k]) : t + lds[w * NV + k];
      v[k] = t;
    }
  }
  __syncthreads();
}

// A flag that another block may set while this block runs, read once for the
// whole block.  Waves that each read it at a different moment could see
// different values and take different paths around the block barriers that
// follow; in a persistent launch (waves that return go on to the next virtual
// block) that would pair unrelated barriers.
__device__ __forceinline__ bool block_read_flag(const int* f) {
  __shared__ int v;
  if (threadIdx.x == 0) v = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const bool r = v != 0;
  __syncthreads();
  return r;
}

// Sum (or max) of the NV-wide partials of the G blocks of the previous sweep,
// in a fixed order, made available to every thread of the block.  Every block
// computes the same bits, so the scalars derived from it agree everywhere.  Up to
// kPartialRounds * kBlock blocks, every thread issues all its loads at once (one
// memory latency instead of one per round), and the loads can be issued early
// (load_partials) and summed later (reduce_loaded); the order of the sums is the
// same in every case.
constexpr int kPartialRounds = 4;
template <int NV>
struct LoadedPartials {
  double t[kPartialRounds][NV];
};

template <int NV>
__device__ __forceinline__ LoadedPartials<NV> load_partials(const double* __restrict__ part, int G,
                                                            const bool (&is_max)[NV]) {
  LoadedPartials<NV> lp;
  if (G <= kPartialRounds * kBlock) {
#pragma unroll
    for (int r = 0; r < kPartialRounds; ++r) {
      const int g = int(threadIdx.x) + r * kBlock;
#pragma unroll
      for (int k = 0; k < NV; ++k) lp.t[r][k] = g < G ? part[g * NV + k] : (is_max[k] ? -DBL_MAX : 0.0);
    }
  }
  return lp;
}

template <int NV>
__device__ __forceinline__ void reduce_loaded(const LoadedPartials<NV>& lp, const double* __restrict__ part, int G,
                                              const bool (&is_max)[NV], double (&out)[NV], double* lds) {
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = is_max[k] ? -DBL_MAX : 0.0;
  if (G <= kPartialRounds * kBlock) {
#pragma unroll
    for (int r = 0; r < kPartialRounds; ++r) {
      if (int(threadIdx.x) + r * kBlock < G) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = is_max[k] ? fmax(v[k], lp.t[r][k]) : v[k] + lp.t[r][k];
      }
    }
  } else {
    for (int g = threadIdx.x; g < G; g += kBlock) {
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const double t = part[g * NV + k];
        v[k] = is_max[k] ? fmax(v[k], t) : v[k] + t;
      }
    }
  }
  block_reduce<NV>(v, is_max, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = lds[k];
  __syncthreads();
}

template <int NV>
__device__ __forceinline__ void reduce_partials_all(const double* __restrict__ part, int G,
                                                    const bool (&is_max)[NV], double (&out)[NV],
                                                    double* lds) {
  reduce_loaded<NV>(load_partials<NV>(part, G, is_max), part, G, is_max, out, lds);
}

// This block's problem, its blocks [b0, b0 + Gp) and its contiguous range of
// 256-slot tiles [t0, t1).  Blocks are dealt to the XCDs round-robin, so for a
// single problem block b is mapped to chunk (b % 8) * (G / 8) + b / 8: each XCD
// then sweeps one contiguous eighth of the Morton order and the neighbour octs
// it gathers are mostly in its own L2.
struct BlockPlan {
  int prob, b0, Gp, t0, t1;
};

__device__ __forceinline__ BlockPlan block_plan(const SweepPlan& P, int b) {
  BlockPlan bp;
  int T0, nt;
  if (P.blk0) {
    bp.prob = P.blk_prob[b];
    bp.b0 = P.blk0[bp.prob];
    bp.Gp = P.blk0[bp.prob + 1] - bp.b0;
    T0 = P.tile0[bp.prob];
    nt = P.tile0[bp.prob + 1] - T0;
  } else {
    bp.prob = 0;
    bp.b0 = 0;
    bp.Gp = P.G;
    T0 = 0;
    nt = P.n_tiles;
  }
  const int lb = b - bp.b0;
  const int c = (!P.blk0 && bp.Gp % 8 == 0) ? (lb % 8) * (bp.Gp / 8) + lb / 8 : lb;
  bp.t0 = T0 + int((int64_t(nt) * c) / bp.Gp);
  bp.t1 = T0 + int((int64_t(nt) * (c + 1)) / bp.Gp);
  return bp;
}

// Blocks of problem `prob` (for the one-block-per-problem finishers).
__device__ __forceinline__ void problem_blocks(const SweepPlan& P, int prob, int& b0, int& Gp) {
  b0 = P.blk0 ? P.blk0[prob] : 0;
  Gp = P.blk0 ? P.blk0[prob + 1] - b0 : P.G;
}


// Grid-wide barrier of a cooperative launch (all blocks resident), in two levels
// over the XCDs.  Every XCD has its own L2 and blocks of one XCD see each other's
// stores there once they have completed; another XCD sees them only after that L2
// has been written back (agent-scope release) and its own copies invalidated
// (agent-scope acquire).  So a block waits until its own stores have completed and
// arrives at its XCD's word; the last arrival of an XCD writes back that L2 once
// for all its blocks and arrives at the global word; the last XCD publishes the
// barrier number there; each XCD's last arrival, once it sees it, publishes it on
// its XCD's word, where that XCD's other blocks wait; every block then acquires.
// Blocks learn their XCD from the hardware register that names it, and the first
// barrier of a launch (a flat one: every block writes back and arrives at one
// word) also counts each XCD's blocks.  Arrival words only ever grow; barrier
// number `epoch` is complete on a word when it reaches epoch times its arrivals.
// Every wait is bounded: after spin_limit polls the block reports failure instead
// of waiting forever.  All words live in `bar` (kBarWords, the first kBarAbort
// zeroed before the launch).
struct GridSync {
  unsigned* bar;
  unsigned n_blocks;
  unsigned spin_limit;
  unsigned epoch = 0;    // barriers this block has passed
  unsigned xcd = 0;      // thread 0: this block's XCD
  unsigned xcd_size = 0; // thread 0: resident blocks of that XCD
  unsigned n_xcd = 0;    // thread 0: XCDs with resident blocks
};

__device__ __forceinline__ unsigned this_xcd() {
  // HW_REG_XCC_ID: bits [3:0] hold the XCD the wave runs on
  return __builtin_amdgcn_s_getreg((15 << 11) | 20) & unsigned(kMaxXcd - 1);
}

__device__ __forceinline__ bool spin_until(unsigned* w, unsigned target, unsigned spin_limit) {
  unsigned polls = 0;
  while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(2);
    if (++polls > spin_limit) return false;
  }
  return true;
}

__device__ __forceinline__ bool grid_barrier(GridSync& gs) {
  __shared__ int ok;
  ++gs.epoch;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed (they are in its XCD's L2)
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned* bar = gs.bar;
    int good = 1;
    if (gs.epoch == 1) {
      // flat: count this XCD's blocks, write back, arrive at one word
      gs.xcd = this_xcd();
      __hip_atomic_fetch_add(bar + kBarXcdCount + 64 * gs.xcd, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned old =
          __hip_atomic_fetch_add(bar + kBarFirstArrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (old + 1u == gs.n_blocks) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(bar + kBarFirstRelease, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        good = spin_until(bar + kBarFirstRelease, 1u, gs.spin_limit);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      unsigned n = 0;
      for (int x = 0; x < kMaxXcd; ++x)
        n += __hip_atomic_load(bar + kBarXcdCount + 64 * x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0u;
      gs.n_xcd = n;
      gs.xcd_size = __hip_atomic_load(bar + kBarXcdCount + 64 * gs.xcd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned e = gs.epoch - 1;  // numbering of the two-level barriers
      const unsigned old =
          __hip_atomic_fetch_add(bar + kBarXcdArrive + 64 * gs.xcd, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (old + 1u == e * gs.xcd_size) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this XCD's stores, written back once
        const unsigned o2 = __hip_atomic_fetch_add(bar + kBarArrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (o2 + 1u == e * gs.n_xcd) {
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
          __hip_atomic_store(bar + kBarRelease, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          good = spin_until(bar + kBarRelease, e, gs.spin_limit);
        }
        __hip_atomic_store(bar + kBarXcdRelease + 64 * gs.xcd, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        good = spin_until(bar + kBarXcdRelease + 64 * gs.xcd, e, gs.spin_limit);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// Couplings of slot ii to other levels in the composite system of all levels: its
// out-of-oct faces that look at a coarser leaf, and the four finer cells on each
// face shared with a refined same-level neighbour (their coefficients are stored
// at the finer cells, so both rows of a pair read the same value).  Returns the
// sum of coefficient x get(neighbour), to be subtracted from the row.
template <typename T, class Get>
__device__ __forceinline__ T interface_terms(int ii, const DevLevel& L, int n, Get get) {
  const int pos = ii & 7, o = ii >> 3;
  T s = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T cf = T(L.cif[size_t(a) * n + ii]);
    if (cf != T(0)) {
      const int my = (pos >> a) & 1;
      s += cf * get(L.cnb[o * 6 + 2 * a + my]);
    }
  }
  const unsigned m = L.c2f[ii];
  if (m) {
    for (int d = 0; d < 6; ++d) {
      if (!((m >> d) & 1)) continue;
      const int a = d >> 1, side = d & 1;
      const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
      const int co = L.child[same_level_nb(L.nbr, ii, d)];
      const int fb = side ? 0 : 1;  // the finer cells on the side that faces ii
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int f = (co << 3) | (fb << a) | ((k & 1) << t0) | ((k >> 1) << t1);
        s += T(L.cif[size_t(a) * n + f]) * get(f);
      }
    }
  }
  return s;
}

// The 7-point operator at slot ii applied to a vector whose value at ii is pi
// and at other slots is get(j).  T is the storage and arithmetic type.
template <typename T, class Get>
__device__ __forceinline__ T apply_stencil(int ii, const int32_t* __restrict__ nbr,
                                           const T* __restrict__ Cp, int n, T di, T pi, Get get) {
  const int pos = ii & 7, o = ii >> 3;
  T acc = di * pi;
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    const int bit = 1 << axis;
    const T* __restrict__ Ca = Cp + size_t(axis) * n;
    const T c_own = Ca[ii];
    const T p_sib = __shfl_xor(pi, bit, 64);
    const T c_sib = __shfl_xor(c_own, bit, 64);
    const int my = (pos >> axis) & 1;
    acc -= (my ? c_sib : c_own) * p_sib;
    const int nb = nbr[o * 6 + 2 * axis + my];
    if (nb >= 0) {
      const int j = (nb << 3) | (pos ^ bit);
      const T c_out = my ? c_own : Ca[j];
      if (c_out != T(0)) acc -= c_out * get(j);
    }
  }
  return acc;
}

// The same operator with stored or formed face coefficients; `scale` is the
// problem's coef_scale.
template <typename T, class Get>
__device__ __forceinline__ T apply_stencil(int ii, const int32_t* __restrict__ nbr, const FaceCoefs<T>& A,
                                           T scale, int n, T di, T pi, Get get) {
  if (A.Cp) return apply_stencil<T>(ii, nbr, A.Cp, n, di, pi, get);
  const int pos = ii & 7, o = ii >> 3;
  const T Ki = A.K[ii];
  const unsigned m = A.mask[ii];
  const T th = T(A.theta);
  T acc = di * pi;
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    const int bit = 1 << axis;
    const T K_sib = __shfl_xor(Ki, bit, 64);
    const T p_sib = __shfl_xor(pi, bit, 64);
    const int my = (pos >> axis) & 1;
    const T c_in = ((m >> (2 * axis + 1 - my)) & 1u) ? face_coef(Ki, K_sib, scale, th) : T(0);
    acc -= c_in * p_sib;
    const int nb = nbr[o * 6 + 2 * axis + my];
    if (nb >= 0 && ((m >> (2 * axis + my)) & 1u)) {
      const int j = (nb << 3) | (pos ^ bit);
      const T c_out = face_coef(Ki, A.K[j], scale, th);
      if (c_out != T(0)) acc -= c_out * get(j);
    }
  }
  return acc;
}

// The Jacobi-scaled operator at slot ii (diagonal 1) applied to a vector whose value
// at ii is vi and at other slots is get(j); `scale` is the problem's coef_scale.
template <typename T, class Get>
__device__ __forceinline__ T apply_scaled(int ii, const int32_t* __restrict__ nbr, const ScaledOp<T>& A, T scale,
                                          int n, T vi, Get get) {
  const int pos = ii & 7, o = ii >> 3;
  T acc = vi;
  if (A.Ch) {
#pragma unroll
    for (int axis = 0; axis < 3; ++axis) {
      const int bit = 1 << axis;
      const T* __restrict__ Ca = A.Ch + size_t(axis) * n;
      const T c_own = Ca[ii];
      const T v_sib = __shfl_xor(vi, bit, 64);
      const T c_sib = __shfl_xor(c_own, bit, 64);
      const int my = (pos >> axis) & 1;
      acc -= (my ? c_sib : c_own) * v_sib;
      const int nb = nbr[o * 6 + 2 * axis + my];
      if (nb >= 0) {
        const int j = (nb << 3) | (pos ^ bit);
        const T c_out = my ? c_own : Ca[j];
        if (c_out != T(0)) acc -= c_out * get(j);
      }
    }
    return acc;
  }
  const T Ki = A.K[ii], rsi = A.rs[ii];
  const unsigned m = A.mask[ii];
  const T th = T(A.theta);
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    const int bit = 1 << axis;
    const T K_sib = __shfl_xor(Ki, bit, 64);
    const T rs_sib = __shfl_xor(rsi, bit, 64);
    const T v_sib = __shfl_xor(vi, bit, 64);
    const int my = (pos >> axis) & 1;
    const T c_in = ((m >> (2 * axis + 1 - my)) & 1u) ? scaled_face(Ki, K_sib, rsi, rs_sib, scale, th) : T(0);
    acc -= c_in * v_sib;
    const int nb = nbr[o * 6 + 2 * axis + my];
    if (nb >= 0 && ((m >> (2 * axis + my)) & 1u)) {
      const int j = (nb << 3) | (pos ^ bit);
      const T c_out = scaled_face(Ki, A.K[j], rsi, A.rs[j], scale, th);
      if (c_out != T(0)) acc -= c_out * get(j);
    }
  }
  return acc;
}

}  // namespace dev
}  // namespace amrfld
