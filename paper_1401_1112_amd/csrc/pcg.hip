// Jacobi-preconditioned conjugate gradient on one level (Sect. 3.3.4), run as CG
// on the Jacobi-scaled system A^ = S A S (S = diag(1 / sqrt(diag A)), unknown
// S^-1 x, right-hand side S b) with the recurrences of Chronopoulos and Gear: one
// fused sweep per iteration updates p, s = A^ p, x and r and applies the operator
// to the new r, and the two dot products it needs, (r, r) and (A^ r, r), are
// reduced together at the head of the next sweep.  In exact arithmetic the
// iterates are those of Jacobi PCG on A x = b.  Also the FP64 iterative-refinement
// sweeps of the mixed-precision form.
//
// Reductions without atomics: every sweep runs G blocks, each block sweeps a
// contiguous range of 256-slot tiles and writes one partial per reduced
// quantity.  The NEXT sweep reduces all G partials at its head, in the same
// fixed order in every block, and derives alpha, beta and the stopping
// decision itself; the kernel boundary makes the partials visible.  Runs are
// therefore bitwise reproducible.  Scalars that a sweep writes and later
// sweeps read are double-buffered by iteration parity, and so are the partials:
// the sweep of iteration it writes region it & 1 (4 per block: (r^, r^),
// (w^, r^), ||r||^2, max relative change) and reads region (it - 1) & 1.  The
// other kernels (refinement sweep, true residual, post-solve) use [0, 4G) at
// times when no iteration sweep runs.
#include <hip/hip_ext.h>

#include <algorithm>

#include "common.h"

namespace amrfld {

// At most max_tiles tiles per block: the iteration sweep stages the block's whole
// range of the new residual in LDS (16 tiles = 32 KB in FP64, 32 tiles in FP32).  A
// level with more than max_blocks * max_tiles tiles gets a whole multiple of
// max_blocks, so that the blocks of a persistent launch of max_blocks blocks each
// sweep the same number of equal ranges.
int sweep_blocks(int n_tiles, int max_blocks, int max_tiles) {
  const int B = std::max(1, max_blocks);
  const int64_t per = int64_t(B) * std::max(1, max_tiles);
  if (n_tiles <= B) return std::max(1, n_tiles);
  const int64_t rounds = (int64_t(n_tiles) + per - 1) / per;
  return int(rounds * B);
}

namespace {

using dev::apply_scaled;
using dev::apply_stencil;
using dev::block_plan;
using dev::block_read_flag;
using dev::block_reduce;
using dev::BlockPlan;
using dev::grid_barrier;
using dev::problem_blocks;
using dev::reduce_partials_all;
using dev::scaled_face;

constexpr int kLds = (kBlock / 64) * 4 + 4;

template <typename T>
__device__ __forceinline__ T rel_change(T x, T dx) {
  const T ax = fabs(x);
  return ax > T(0) ? fabs(dx) / ax : fabs(dx);
}

// The partials of the iteration sweep of iteration `it` (and of the start, it = 0).
__device__ __forceinline__ double* part_of(double* part, const SweepPlan& P, int it) {
  return part + size_t(it & 1) * 4 * size_t(P.G);
}
__device__ __forceinline__ const double* part_of(const double* part, const SweepPlan& P, int it) {
  return part + size_t(it & 1) * 4 * size_t(P.G);
}

// Stopping test of Sect. 3.3.4 for iterate it_done from its sweep's reduced
// partials: ||r|| <= thresh AND (optionally) the largest relative change < tol.
struct StopTest {
  double rn, linf;
  bool fin, conv, stop;
};

__device__ __forceinline__ StopTest stop_test(const PcgScalars* sc, const double (&red)[4], int it_done) {
  StopTest s;
  s.rn = sqrt(red[2]);
  s.linf = red[3];
  s.fin = isfinite(s.rn) && isfinite(red[0]) && isfinite(red[1]);
  s.conv = s.fin && ((s.rn <= sc->thresh && (!sc->linf_test || s.linf < sc->tol)) || s.rn == 0.0);
  s.stop = !s.fin || s.conv || it_done >= sc->max_iter;
  return s;
}

// Marks a problem stopped.  The done counter (which ends the persistent loops) is
// only advanced at the heads of the iteration sweeps, so that every block reads
// the same count right after a grid barrier.
__device__ __forceinline__ void mark_done(PcgScalars* sc, const SweepPlan& P, bool count = true) {
  sc->done = 1;
  if (count && P.done_count && !sc->counted) {
    sc->counted = 1;
    atomicAdd(P.done_count, 1u);
  }
}

__device__ __forceinline__ void record_stop(PcgScalars* sc, const StopTest& s, int it_done, const SweepPlan& P) {
  sc->rnorm = s.rn;
  sc->linf = s.linf;
  sc->iter = it_done;
  if (s.stop) {
    sc->converged = s.conv ? 1 : 0;
    sc->nonfinite = s.fin ? 0 : 1;
    mark_done(sc, P);
  }
}

template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], const bool (&mx)[NV], double* dst, double* lds,
                                               int vb) {
  block_reduce<NV>(v, mx, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) dst[vb * NV + k] = v[k];
  }
}

// Start, sweep 1: r^_0 = rs (b - A x0) with the unscaled operator, p^ = 0, s^_{-1} = 0.
template <typename T>
__device__ __forceinline__ void body_cg_init_r(int vb, DevLevel L, SweepPlan P, const FaceCoefs<T>& A,
                                               const T* __restrict__ diag, const T* __restrict__ b,
                                               const T* __restrict__ x, const T* __restrict__ rs, CgVecs<T> v) {
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  const T scale = dev::coef_scale(A, L, bp.prob);
  for (int t = bp.t0; t < bp.t1; ++t) {
    const int i = t * kBlock + int(threadIdx.x);
    const bool valid = i < n;
    const int ii = valid ? i : n - 1;
    T ax = apply_stencil<T>(ii, L.nbr, A, scale, n, diag[ii], x[ii], [&](int j) { return x[j]; });
    if (L.cif) ax -= dev::interface_terms<T>(ii, L, n, [&](int j) { return x[j]; });
    if (valid) {
      v.r[0][i] = rs[i] * (b[i] - ax);
      v.p[i] = T(0);
      v.s[0][i] = T(0);
    }
  }
}

// Start, sweep 2: w^_0 = A^ r^_0; partials (r^, r^), (w^, r^), ||r_0||^2 and ||b||^2
// (over the unknowns only: identity rows hold b = E, which is no part of the system).
template <typename T>
__device__ __forceinline__ void body_cg_init_w(int vb, DevLevel L, SweepPlan P, const ScaledOp<T>& Ah,
                                               const T* __restrict__ b, CgVecs<T> v, double* part) {
  __shared__ double lds[kLds];
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  const T scale = dev::coef_scale(Ah, L, bp.prob);
  const T* __restrict__ r = v.r[0];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t = bp.t0; t < bp.t1; ++t) {
    const int i = t * kBlock + int(threadIdx.x);
    const bool valid = i < n;
    const int ii = valid ? i : n - 1;
    const T ri = r[ii];
    const T wi = apply_scaled<T>(ii, L.nbr, Ah, scale, n, ri, [&](int j) { return r[j]; });
    if (valid) {
      v.w[0][i] = wi;
      acc[0] += double(ri) * double(ri);
      acc[1] += double(wi) * double(ri);
      const double ru = double(ri) / double(Ah.rs[i]);
      acc[2] += ru * ru;
      if (L.child[i] == -1) acc[3] += double(b[i]) * double(b[i]);
    }
  }
  const bool mx[4] = {false, false, false, false};
  write_partials<4>(acc, mx, part_of(part, P, 0), lds, vb);
}

// Operand values at slots outside a block's range, from the values loaded there
// (the block computes the same values for its own range into LDS, in the same
// arithmetic, so both agree bitwise).
// The new scaled residual of an iteration sweep from the previous r^, w^ and s^
// (read buffers, which no block writes during the sweep).
template <typename T>
struct HaloIterate {
  const T* __restrict__ r;
  const T* __restrict__ w;
  const T* __restrict__ s;
  T ta, tb;
  struct V {
    T r, w, s;
  };
  __device__ __forceinline__ V load(int j) const { return V{r[j], w[j], s[j]}; }
  __device__ __forceinline__ T value(const V& g) const { return fma(-ta, fma(tb, g.s, g.w), g.r); }
};
// Values of an array written by an earlier kernel.
template <typename T>
struct HaloPlain {
  const T* __restrict__ v;
  struct V {
    T v;
  };
  __device__ __forceinline__ V load(int j) const { return V{v[j]}; }
  __device__ __forceinline__ T value(const V& g) const { return g.v; }
};
// The scaled FP32 residual of an inner start, rs r32.
struct HaloScaledResidual {
  const float* __restrict__ r32;
  const float* __restrict__ rs;
  struct V {
    float r, q;
  };
  __device__ __forceinline__ V load(int j) const { return V{r32[j], rs[j]}; }
  __device__ __forceinline__ float value(const V& g) const { return g.q * g.r; }
};
// The scaled FP64 iterate of a refinement sweep, (x + d) / rs (d may be null).
struct HaloScaledIterate {
  const double* __restrict__ x;
  const float* __restrict__ d;
  const double* __restrict__ rs;
  struct V {
    double x, q;
    float d;
  };
  __device__ __forceinline__ V load(int j) const { return V{x[j], rs[j], d ? d[j] : 0.0f}; }
  __device__ __forceinline__ double value(const V& g) const { return (g.x + double(g.d)) / g.q; }
};

// The scaled iterate x / rs of a start sweep.
template <typename T>
struct HaloScaledIterateT {
  const T* __restrict__ x;
  const T* __restrict__ rs;
  struct V {
    T x, q;
  };
  __device__ __forceinline__ V load(int j) const { return V{x[j], rs[j]}; }
  __device__ __forceinline__ T value(const V& g) const { return g.x / g.q; }
};

// Phase 2 of a staged sweep: out(i, (A^ v)_i, v_i) for every slot of the block's
// range, where the block has staged v over its range in LDS (rl).  In-oct neighbours
// come by cross-lane shuffle, out-of-oct neighbours inside the range from LDS, the
// rest from halo.  Lanes that need no gather read the range's first slot (one line,
// in cache) instead of their own, whose lines the first phase read long enough ago
// to have left L2.
template <typename T, int U2, bool kFormed, class Halo, class Out>
__device__ __forceinline__ void staged_operator(const DevLevel& L, const ScaledOp<T>& Ah, T scale, int s0, int s1,
                                                int t0, int t1, const T* rl, const Halo& halo, Out out) {
  const int n = L.n_slots;
  const T th = T(Ah.theta);
  for (int tb0 = t0; tb0 < t1; tb0 += U2) {
    int ii[U2], nbv[U2][3];
    unsigned mk[U2];
    T own[U2][3], rsi[U2];
    bool valid[U2];
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const int i = (tb0 + u) * kBlock + int(threadIdx.x);
      valid[u] = (tb0 + u < t1) && i < n;
      ii[u] = valid[u] ? i : s1 - 1;
      const int pos = ii[u] & 7, o = ii[u] >> 3;
      if constexpr (!kFormed) {
#pragma unroll
        for (int a = 0; a < 3; ++a) own[u][a] = Ah.Ch[size_t(a) * n + ii[u]];
        mk[u] = 0x3fu;
        rsi[u] = T(1);
      } else {
        own[u][0] = Ah.K[ii[u]];
        own[u][1] = own[u][2] = T(0);
        mk[u] = Ah.mask[ii[u]];
        rsi[u] = Ah.rs[ii[u]];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) nbv[u][a] = L.nbr[o * 6 + 2 * a + ((pos >> a) & 1)];
    }
    // gathers: the out-of-oct coefficient (stored: of a -face, at the neighbour;
    // formed: the neighbour's K and rs) and the halo inputs of neighbours outside
    // the range
    int jv[U2][3];
    T cj[U2][3], kj[U2][3];
    typename Halo::V hv[U2][3];
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const int pos = ii[u] & 7;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int my = (pos >> a) & 1;
        const int nb = nbv[u][a];
        const bool cpl = nb >= 0 && ((mk[u] >> (2 * a + my)) & 1u);
        const int j = cpl ? ((nb << 3) | (pos ^ (1 << a))) : ii[u];
        jv[u][a] = cpl ? j : -1;
        const bool inr = j >= s0 && j < s1;
        const int jo = inr ? s0 : j;
        if constexpr (!kFormed) {
          cj[u][a] = Ah.Ch[size_t(a) * n + (my ? ii[u] : j)];
          kj[u][a] = T(0);
        } else {
          cj[u][a] = Ah.K[j];
          kj[u][a] = Ah.rs[j];
        }
        hv[u][a] = halo.load(jo);
      }
    }
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const int pos = ii[u] & 7;
      const T vi = valid[u] ? rl[ii[u] - s0] : T(0);
      T acc = vi;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int bit = 1 << a;
        const int my = (pos >> a) & 1;
        const T v_sib = __shfl_xor(vi, bit, 64);
        T c_in;
        if constexpr (!kFormed) {
          const T c_sib = __shfl_xor(own[u][a], bit, 64);
          c_in = my ? c_sib : own[u][a];
        } else {
          const T K_sib = __shfl_xor(own[u][0], bit, 64);
          const T rs_sib = __shfl_xor(rsi[u], bit, 64);
          c_in = ((mk[u] >> (2 * a + 1 - my)) & 1u) ? scaled_face(own[u][0], K_sib, rsi[u], rs_sib, scale, th) : T(0);
        }
        acc -= c_in * v_sib;
        const int j = jv[u][a];
        if (j >= 0) {
          T c_out;
          if constexpr (!kFormed) c_out = my ? own[u][a] : cj[u][a];
          else c_out = scaled_face(own[u][0], cj[u][a], rsi[u], kj[u][a], scale, th);
          const T vn = (j >= s0 && j < s1) ? rl[j - s0] : halo.value(hv[u][a]);
          acc -= c_out * vn;
        }
      }
      if (valid[u]) out(ii[u], acc, vi);
    }
  }
}

template <typename T, int U2, class Halo, class Out>
__device__ __forceinline__ void staged_operator(const DevLevel& L, const ScaledOp<T>& Ah, T scale, int s0, int s1,
                                                int t0, int t1, const T* rl, const Halo& halo, Out out) {
  if (Ah.Ch) staged_operator<T, U2, false>(L, Ah, scale, s0, s1, t0, t1, rl, halo, out);
  else staged_operator<T, U2, true>(L, Ah, scale, s0, s1, t0, t1, rl, halo, out);
}

// Slots per thread of the streaming phase and tiles per trip of the operator phase
// of the sweeps (twice these in FP32 measured slower).
template <typename T>
constexpr int kStreamUnroll = 4;
template <typename T>
constexpr int kOperatorUnroll = 2;

// Start, sweep 1, staged: r^_0 = rs b - A^ x^_0 with x^_0 = x0 / rs in LDS (the same
// residual as rs (b - A x0), A applied as S^-1 A^ S^-1), p^ = 0, s^_{-1} = 0.
template <typename T>
__device__ __forceinline__ void body_cg_start_r(int vb, DevLevel L, SweepPlan P, const ScaledOp<T>& Ah,
                                                const T* __restrict__ b, const T* __restrict__ x, CgVecs<T> v) {
  extern __shared__ unsigned char dyn_lds[];
  T* rl = reinterpret_cast<T*>(dyn_lds);
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  const int s0 = bp.t0 * kBlock, s1 = min(bp.t1 * kBlock, n);
  const T* __restrict__ rs = Ah.rs;
  for (int i = s0 + int(threadIdx.x); i < s1; i += kBlock) rl[i - s0] = x[i] / rs[i];
  __syncthreads();
  const T scale = dev::coef_scale(Ah, L, bp.prob);
  staged_operator<T, kOperatorUnroll<T>>(L, Ah, scale, s0, s1, bp.t0, bp.t1, rl, HaloScaledIterateT<T>{x, rs},
                                         [&](int i, T ax, T) {
                                           v.r[0][i] = rs[i] * b[i] - ax;
                                           v.p[i] = T(0);
                                           v.s[0][i] = T(0);
                                         });
}

// Start, sweep 2, staged: w^_0 = A^ r^_0 with r^_0 staged in LDS; partials (r^, r^),
// (w^, r^), ||r_0||^2 and ||b||^2 (over the unknowns only: identity rows hold b = E,
// which is no part of the system).
template <typename T>
__device__ __forceinline__ void body_cg_start_w(int vb, DevLevel L, SweepPlan P, const ScaledOp<T>& Ah,
                                                const T* __restrict__ b, CgVecs<T> v, double* part) {
  __shared__ double lds[kLds];
  extern __shared__ unsigned char dyn_lds[];
  T* rl = reinterpret_cast<T*>(dyn_lds);
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  const int s0 = bp.t0 * kBlock, s1 = min(bp.t1 * kBlock, n);
  const T* __restrict__ r = v.r[0];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = s0 + int(threadIdx.x); i < s1; i += kBlock) {
    const T ri = r[i];
    rl[i - s0] = ri;
    acc[0] += double(ri) * double(ri);
    const double ru = double(ri) / double(Ah.rs[i]);
    acc[2] += ru * ru;
    if (L.child[i] == -1) acc[3] += double(b[i]) * double(b[i]);
  }
  __syncthreads();
  const T scale = dev::coef_scale(Ah, L, bp.prob);
  T* __restrict__ w = v.w[0];
  double dl = 0.0;
  staged_operator<T, kOperatorUnroll<T>>(L, Ah, scale, s0, s1, bp.t0, bp.t1, rl, HaloPlain<T>{r},
                                         [&](int i, T wi, T ri) {
                                           w[i] = wi;
                                           dl += double(wi) * double(ri);
                                         });
  acc[1] = dl;
  const bool mx[4] = {false, false, false, false};
  write_partials<4>(acc, mx, part_of(part, P, 0), lds, vb);
}

// The FP64 true residual norm of a solve without couplings to other levels, staged:
// x^ = x / rs in LDS, r = b - (A^ x^) / rs; one partial ||r||^2 per block.
__device__ __forceinline__ void body_true_residual_staged(int vb, DevLevel L, SweepPlan P,
                                                          const ScaledOp<double>& Ah,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ x, double* part) {
  __shared__ double lds[kLds];
  extern __shared__ unsigned char dyn_lds[];
  double* rl = reinterpret_cast<double*>(dyn_lds);
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  const int s0 = bp.t0 * kBlock, s1 = min(bp.t1 * kBlock, n);
  const double* __restrict__ rs = Ah.rs;
  for (int i = s0 + int(threadIdx.x); i < s1; i += kBlock) rl[i - s0] = x[i] / rs[i];
  __syncthreads();
  const double scale = dev::coef_scale(Ah, L, bp.prob);
  double v[1] = {0.0};
  staged_operator<double, kOperatorUnroll<double>>(L, Ah, scale, s0, s1, bp.t0, bp.t1, rl,
                                                   HaloScaledIterateT<double>{x, rs}, [&](int i, double ax, double) {
                                                     const double ri = b[i] - ax / rs[i];
                                                     v[0] += ri * ri;
                                                   });
  const bool mx[1] = {false};
  write_partials<1>(v, mx, part, lds, vb);
}

// Inner start of the mixed form: d = 0 (the inner solve's iterate, a correction of
// the FP64 x), r^ = rs r32 (the FP64 residual, rounded and scaled), w^ = A^ r^;
// partials (r^, r^), (w^, r^), ||r32||^2 twice.  A fresh start (inner cont = 0)
// clears p^ and s^; a continued one (the residual replaced after a refinement
// sweep, the search direction kept) moves s^ of the last iteration into buffer 0.
__device__ __forceinline__ void body_inner_init(int vb, DevLevel L, SweepPlan P, const ScaledOp<float>& Ah,
                                                const float* __restrict__ r32, float* __restrict__ d,
                                                CgVecs<float> v, const PcgScalars* outer,
                                                const PcgScalars* inner, double* part) {
  __shared__ double lds[kLds];
  extern __shared__ unsigned char dyn_lds[];
  float* rl = reinterpret_cast<float*>(dyn_lds);
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  if (outer[bp.prob].done) return;  // set by an earlier kernel (or before a grid barrier)
  const int cont = inner[bp.prob].cont;
  const int s0 = bp.t0 * kBlock, s1 = min(bp.t1 * kBlock, n);
  const float* __restrict__ rs = Ah.rs;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = s0 + int(threadIdx.x); i < s1; i += kBlock) {
    const float ri = rs[i] * r32[i];
    rl[i - s0] = ri;
    v.r[0][i] = ri;
    d[i] = 0.0f;
    if (cont == 0) {
      v.p[i] = 0.0f;
      v.s[0][i] = 0.0f;
    } else if (cont == 2) {
      v.s[0][i] = v.s[1][i];
    }
    acc[0] += double(ri) * double(ri);
    const double rr = double(r32[i]) * double(r32[i]);
    acc[2] += rr;
    acc[3] += rr;
  }
  __syncthreads();
  const float scale = dev::coef_scale(Ah, L, bp.prob);
  float* __restrict__ w = v.w[0];
  double dl = 0.0;
  staged_operator<float, kOperatorUnroll<float>>(L, Ah, scale, s0, s1, bp.t0, bp.t1, rl,
                                                 HaloScaledResidual{r32, rs}, [&](int i, float wi, float ri) {
                                                   w[i] = wi;
                                                   dl += double(wi) * double(ri);
                                                 });
  acc[1] = dl;
  const bool mx[4] = {false, false, false, false};
  write_partials<4>(acc, mx, part_of(part, P, 0), lds, vb);
}

// The iteration sweep of iteration `it`: it advances every problem of the plan from
// iterate it - 1 to iterate it.  Head: the previous sweep's partials give the
// stopping test on iterate it - 1 and the recurrences
//   beta_j = gamma_j / gamma_{j-1},  alpha_j = gamma_j / (delta_j - beta_j gamma_j / alpha_{j-1})
// (j = it - 1; for it = 1 the start's partials give ||r_0||, the threshold, the
// absolute floor and alpha_0 = gamma_0 / delta_0, beta_0 = 0, unless the record
// continues an inner solve, whose previous scalars sit at index 1).  Then two phases over
// the block's contiguous slot range: (1) p^ = r^ + beta p^, s^ = w^ + beta s^,
// x += alpha rs p^, r^ -= alpha s^, the new r^ also into LDS; (2) w^ = A^ r^.
template <typename T>
__device__ __forceinline__ void body_cg_sweep(int vb, DevLevel L, SweepPlan P, int it, const ScaledOp<T>& Ah,
                                              CgVecs<T> v, T* __restrict__ x, PcgScalars* scs, double* part) {
  __shared__ double lds[kLds];
  extern __shared__ unsigned char dyn_lds[];
  T* rl = reinterpret_cast<T*>(dyn_lds);
  const BlockPlan bp = block_plan(P, vb);
  PcgScalars* sc = scs + bp.prob;
  const int j = it - 1;
  // the previous sweep's partials are loaded together with the stop flag (the
  // problem's first block may set it during this sweep); a stopped problem's sweep
  // returns before it loads anything else
  const bool mxh[4] = {false, false, false, it > 1};
  const double* part_prev = part_of(part, P, j) + 4 * bp.b0;
  const dev::LoadedPartials<4> lp = dev::load_partials<4>(part_prev, bp.Gp, mxh);
  if (block_read_flag(&sc->done)) {
    if (vb == bp.b0 && threadIdx.x == 0) mark_done(sc, P);
    return;
  }
  const int n = L.n_slots;
  const int t0 = bp.t0, t1 = bp.t1;
  const int s0 = t0 * kBlock;
  const int s1 = min(t1 * kBlock, n);
  const int ob = j & 1, nb = it & 1;
  const T* __restrict__ r_o = v.r[ob];
  const T* __restrict__ w_o = v.w[ob];
  const T* __restrict__ s_o = v.s[ob];
  T* __restrict__ r_n = v.r[nb];
  T* __restrict__ s_n = v.s[nb];
  T* __restrict__ p = v.p;
  const T* __restrict__ rs = Ah.rs;
  // phase 1 loads: U1 slots per thread and trip, the first batch issued before the
  // head reduction (it does not depend on alpha or beta) and each next batch before
  // the current one is used
  constexpr int U1 = kStreamUnroll<T>;
  T pv[U1], sv[U1], wv[U1], xv[U1], rv[U1], qv[U1];
  auto load1 = [&](int base) {
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int i = min(base + u * kBlock, s1 - 1);
      pv[u] = p[i];
      sv[u] = s_o[i];
      wv[u] = w_o[i];
      xv[u] = x[i];
      rv[u] = r_o[i];
      qv[u] = rs[i];
    }
  };
  int base = s0 + int(threadIdx.x);
  load1(min(base, s1 - 1));
  double red[4];
  dev::reduce_loaded<4>(lp, part_prev, bp.Gp, mxh, red, lds);
  if (P.extra_part) {  // composite system: the (w^, r^) part of the couplings to other levels
    double pe[1];
    const bool mx1[1] = {false};
    reduce_partials_all<1>(P.extra_part, P.n_extra, mx1, pe, lds);
    red[1] += pe[0];
  }
  const bool lead = vb == bp.b0 && threadIdx.x == 0;
  double alpha, beta;
  if (it == 1 && !sc->cont) {
    const double r0 = sqrt(red[2]), bn = sqrt(red[3]);
    const double floor_b = sc->abs_floor * bn;
    const bool fin = isfinite(red[0]) && isfinite(red[1]) && isfinite(r0) && isfinite(bn);
    // ||r_0|| <= abs_floor ||b||: x_0 is returned after 0 iterations
    const bool at_floor = fin && r0 <= floor_b;
    alpha = red[0] / red[1];
    beta = 0.0;
    if (lead) {
      sc->rnorm0 = r0;
      sc->rnorm = r0;
      sc->bnorm = bn;
      sc->thresh = fmax(sc->tol * r0, floor_b);
      sc->iter = 0;
      sc->linf = 0.0;
      sc->nonfinite = fin ? 0 : 1;
      sc->converged = at_floor ? 1 : 0;
      sc->gam[0] = red[0];
      sc->alpha[0] = alpha;
      if (!fin || at_floor) mark_done(sc, P);
    }
    if (!fin || at_floor) return;
  } else {
    // (it = 1 of a continued inner solve: the previous iteration's scalars at index 1)
    const StopTest st = stop_test(sc, red, j);
    if (lead) record_stop(sc, st, j, P);
    if (st.stop) return;
    beta = red[0] / sc->gam[(j - 1) & 1];
    alpha = red[0] / (red[1] - beta * red[0] / sc->alpha[(j - 1) & 1]);
    if (lead) {
      sc->gam[j & 1] = red[0];
      sc->alpha[j & 1] = alpha;
    }
  }
  if (!isfinite(alpha) || !isfinite(beta)) {
    if (lead) {
      sc->nonfinite = 1;
      sc->iter = j;
      mark_done(sc, P);
    }
    return;
  }
  const T ta = T(alpha), tb = T(beta);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // (r^, r^), (w^, r^), ||r||^2, max relative change
  for (; base < s1; base += U1 * kBlock) {
    T pn[U1], sn[U1], xn[U1], rn[U1];
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      pn[u] = fma(tb, pv[u], rv[u]);
      sn[u] = fma(tb, sv[u], wv[u]);
      const T dx = qv[u] * (ta * pn[u]);
      xn[u] = xv[u] + dx;
      rn[u] = fma(-ta, sn[u], rv[u]);
      if (base + u * kBlock < s1) {
        acc[3] = fmax(acc[3], double(rel_change(xv[u], dx)));
        acc[0] += double(rn[u]) * double(rn[u]);
        const double ru = double(rn[u]) / double(qv[u]);
        acc[2] += ru * ru;
      }
    }
    if (base + U1 * kBlock < s1) load1(base + U1 * kBlock);
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int i = base + u * kBlock;
      if (i < s1) {
        rl[i - s0] = rn[u];
        p[i] = pn[u];
        s_n[i] = sn[u];
        x[i] = xn[u];
        r_n[i] = rn[u];
      }
    }
  }
  __syncthreads();
  const T scale = dev::coef_scale(Ah, L, bp.prob);
  T* __restrict__ w_n = v.w[nb];
  double dl = 0.0;
  staged_operator<T, kOperatorUnroll<T>>(L, Ah, scale, s0, s1, t0, t1, rl, HaloIterate<T>{r_o, w_o, s_o, ta, tb},
                                         [&](int i, T wi, T ri) {
                                           w_n[i] = wi;
                                           dl += double(wi) * double(ri);
                                         });
  acc[1] = dl;
  const bool mx[4] = {false, false, false, true};
  write_partials<4>(acc, mx, part_of(part, P, it), lds, vb);
}

// Applies the stopping test to iterate it_last from its sweep's partials (the test
// the next sweep would make) so that the host sees convergence.
__device__ __forceinline__ void body_check(int prob, SweepPlan P, int it_last, PcgScalars* scs, const double* part) {
  __shared__ double lds[kLds];
  int b0, Gp;
  problem_blocks(P, prob, b0, Gp);
  PcgScalars* sc = scs + prob;
  if (sc->done) return;
  double red[4];
  const bool mx[4] = {false, false, false, true};
  reduce_partials_all<4>(part_of(part, P, it_last) + 4 * b0, Gp, mx, red, lds);
  const StopTest st = stop_test(sc, red, it_last);
  if (threadIdx.x == 0) record_stop(sc, st, it_last, P);
}

__device__ __forceinline__ void body_true_residual(int vb, DevLevel L, SweepPlan P, const FaceCoefs<double>& A,
                                                          const double* __restrict__ diag,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ x, double* part) {
  __shared__ double lds[kLds];
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  const double scale = dev::coef_scale(A, L, bp.prob);
  double v[1] = {0.0};
  for (int t = bp.t0; t < bp.t1; ++t) {
    const int i = t * kBlock + int(threadIdx.x);
    const bool valid = i < n;
    const int ii = valid ? i : n - 1;
    double ax = apply_stencil<double>(ii, L.nbr, A, scale, n, diag[ii], x[ii], [&](int j) { return x[j]; });
    if (L.cif) ax -= dev::interface_terms<double>(ii, L, n, [&](int j) { return x[j]; });
    if (valid) {
      const double ri = b[i] - ax;
      v[0] += ri * ri;
    }
  }
  const bool mx[1] = {false};
  write_partials<1>(v, mx, part, lds, vb);
}

// T update of the coupling term (linearised emission) and smallest leaf energy.
__device__ __forceinline__ void body_post_solve(int vb, DevLevel L, SweepPlan P, const double* __restrict__ E,
                                                       const double* __restrict__ rho, CouplingParams cp,
                                                       double dt, double* __restrict__ T_out, double* part) {
  __shared__ double lds[kLds];
  const BlockPlan bp = block_plan(P, vb);
  double v[1] = {-DBL_MAX};
  for (int t = bp.t0; t < bp.t1; ++t) {
    const int i = t * kBlock + int(threadIdx.x);
    if (i < L.n_slots && L.child[i] == -1) {
      const double e = E[i];
      v[0] = fmax(v[0], -e);
      if (cp.T) {
        const double T = cp.T[i], r = rho[i];
        const double eta = cp.kappa_P * r * cp.c_light * dt;
        const double bT = 4.0 * cp.a_rad * T * T * T;
        const double den = r * cp.c_v + eta * bT;
        T_out[i] = T + eta * (e - cp.a_rad * (T * T * T * T)) / den;
      }
    }
  }
  const bool mx[1] = {true};
  write_partials<1>(v, mx, part, lds, vb);
}

// kind 0: true residual norm; kind 1: smallest leaf energy.
__device__ __forceinline__ void body_finish(int prob, SweepPlan P, int kind, const double* part, PcgScalars* scs) {
  __shared__ double lds[kLds];
  int b0, Gp;
  problem_blocks(P, prob, b0, Gp);
  PcgScalars* sc = scs + prob;
  double v[1];
  const bool mx[1] = {kind == 1};
  reduce_partials_all<1>(part + b0, Gp, mx, v, lds);
  if (threadIdx.x == 0) {
    if (kind == 0) sc->true_rnorm = sqrt(v[0]);
    else sc->min_E = -v[0];
  }
}

// Refinement sweep of the mixed form: x_new = x_old + d (d null on the first), the
// FP64 residual r = b - A x_new with A applied as S^-1 A^ S^-1 (the FP64 scaled
// operator: x^ = x_new / rs staged in LDS, r = b - (A^ x^) / rs), r32 = (float) r;
// partials ||r||^2, ||b||^2 (over the unknowns) and the largest relative change of
// the last inner iteration, |dx| / |x_new - dx| with dx = rs32 (alpha p^) as that
// iteration formed it (alpha of the inner record).
__device__ __forceinline__ void body_ir_sweep(int vb, DevLevel L, SweepPlan P, const ScaledOp<double>& Ah,
                                              const double* __restrict__ b, const double* __restrict__ x_old,
                                              const float* __restrict__ d, const float* __restrict__ p32,
                                              const float* __restrict__ rs32, double* __restrict__ x_new,
                                              float* __restrict__ r32, const PcgScalars* outer,
                                              const PcgScalars* inner, double* part) {
  __shared__ double lds[kLds];
  extern __shared__ unsigned char dyn_lds[];
  double* rl = reinterpret_cast<double*>(dyn_lds);
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  const int s0 = bp.t0 * kBlock, s1 = min(bp.t1 * kBlock, n);
  if (outer[bp.prob].done) {  // converged problem: carry its iterate into the new buffer
    for (int i = s0 + int(threadIdx.x); i < s1; i += kBlock) x_new[i] = x_old[i];
    return;
  }
  // the last inner iteration (none on the first sweep or after an empty inner solve)
  const int jl = d ? inner[bp.prob].iter : 0;
  const float a_last = jl >= 1 ? float(inner[bp.prob].alpha[(jl - 1) & 1]) : 0.0f;
  const double* __restrict__ rs = Ah.rs;
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = s0 + int(threadIdx.x); i < s1; i += kBlock) {
    const double xn = d ? x_old[i] + double(d[i]) : x_old[i];
    x_new[i] = xn;
    rl[i - s0] = xn / rs[i];
    if (jl >= 1) {
      const double dx = double(rs32[i] * (a_last * p32[i]));
      v[2] = fmax(v[2], rel_change(xn - dx, dx));
    }
  }
  __syncthreads();
  const double scale = dev::coef_scale(Ah, L, bp.prob);
  staged_operator<double, kOperatorUnroll<double>>(L, Ah, scale, s0, s1, bp.t0, bp.t1, rl,
                                                   HaloScaledIterate{x_old, d, rs}, [&](int i, double ax, double) {
                                                     const double ri = b[i] - ax / rs[i];
                                                     r32[i] = float(ri);
                                                     v[0] += ri * ri;
                                                     if (L.child[i] == -1) v[1] += b[i] * b[i];
                                                   });
  const bool mx[3] = {false, false, true};
  write_partials<3>(v, mx, part + P.G, lds, vb);
}

// One block per problem: the outer stopping test, then the inner scalars.  A
// problem done in an earlier sweep keeps its state and its inner solve is off.
// Every decision of the refinement loop is made here, on the device: the FP64
// stopping test (Sect. 3.3.4 on the true residual, the relative change being that
// of the last inner iteration), the cap of max_outer refinement sweeps and the cap
// of the outer record's max_iter inner iterations in all (both end the loop
// unconverged).  The inner solve that just ended is added to the outer record's
// count first.  After the first sweep the inner CG is continued, not restarted: its
// residual is replaced by the new FP64 one and its search direction kept (residual
// replacement), and it runs until its residual has fallen by inner_tol from there.
// outer_done (or nullptr) counts the problems whose loop has ended, for the
// persistent launch.
__device__ __forceinline__ void body_ir_finish(int prob, SweepPlan P, int first, double inner_tol, int max_outer,
                                               PcgScalars* outs, PcgScalars* ins, const double* part,
                                               unsigned* outer_done) {
  __shared__ double lds[kLds];
  int b0, Gp;
  problem_blocks(P, prob, b0, Gp);
  PcgScalars* out = outs + prob;
  PcgScalars* in = ins + prob;
  if (out->done) {
    if (threadIdx.x == 0) {
      in->done = 1;
      in->iter = 0;
      in->counted = 0;
    }
    return;
  }
  double v[3];
  const bool mx[3] = {false, false, true};
  reduce_partials_all<3>(part + P.G + 3 * b0, Gp, mx, v, lds);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(v[0]), bn = sqrt(v[1]), linf = v[2];
  const bool fin = isfinite(rn) && isfinite(bn);
  bool conv;
  if (first) {
    const double floor_b = out->abs_floor * bn;
    out->rnorm0 = rn;
    out->bnorm = bn;
    out->thresh = fmax(out->tol * rn, floor_b);
    out->iter = 0;
    out->linf = 0.0;
    out->inner_total = 0;
    conv = fin && rn <= floor_b;
  } else {
    out->inner_total += max(1, in->iter);
    out->iter += 1;
    out->linf = linf;
    conv = fin && ((rn <= out->thresh && (!out->linf_test || linf < out->tol)) || rn == 0.0);
  }
  const int budget = out->max_iter - out->inner_total;
  const bool stop = !fin || conv || out->iter >= max_outer || budget <= 0;
  out->rnorm = rn;
  out->nonfinite = fin ? 0 : 1;
  out->converged = conv ? 1 : 0;
  out->done = stop ? 1 : 0;
  if (stop && outer_done) atomicAdd(outer_done, 1u);
  // the inner solve A d = r stops at a reduction inner_tol of its own residual
  in->tol = inner_tol;
  in->abs_floor = 0.0;
  in->max_iter = max(1, budget);
  in->linf_test = 0;
  in->done = out->done;
  in->converged = 0;
  in->nonfinite = 0;
  if (first) {
    in->cont = 0;
  } else {
    // the scalars of the last iteration j - 1 (j = iter) to index 1, where the
    // continued solve's first sweep (j = 0 of its own count) reads them
    const int jl = in->iter;
    if (jl >= 1 && ((jl - 1) & 1) == 0) {
      in->gam[1] = in->gam[0];
      in->alpha[1] = in->alpha[0];
    }
    in->cont = 1 + (jl & 1);
    in->rnorm0 = rn;
    in->thresh = inner_tol * rn;
  }
  in->iter = 0;
  in->counted = 0;
}

// ------------------------------------------------------------ kernels
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_start_r(DevLevel L, SweepPlan P, ScaledOp<T> Ah,
                                                       const T* __restrict__ b, const T* __restrict__ x,
                                                       CgVecs<T> v) {
  body_cg_start_r<T>(int(blockIdx.x), L, P, Ah, b, x, v);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_start_w(DevLevel L, SweepPlan P, ScaledOp<T> Ah,
                                                       const T* __restrict__ b, CgVecs<T> v, double* part) {
  body_cg_start_w<T>(int(blockIdx.x), L, P, Ah, b, v, part);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_init_r(DevLevel L, SweepPlan P, FaceCoefs<T> A,
                                                      const T* __restrict__ diag, const T* __restrict__ b,
                                                      const T* __restrict__ x, const T* __restrict__ rs,
                                                      CgVecs<T> v) {
  body_cg_init_r<T>(int(blockIdx.x), L, P, A, diag, b, x, rs, v);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_init_w(DevLevel L, SweepPlan P, ScaledOp<T> Ah,
                                                      const T* __restrict__ b, CgVecs<T> v, double* part) {
  body_cg_init_w<T>(int(blockIdx.x), L, P, Ah, b, v, part);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_sweep(DevLevel L, SweepPlan P, int it, ScaledOp<T> Ah, CgVecs<T> v,
                                                     T* __restrict__ x, PcgScalars* scs, double* part) {
  body_cg_sweep<T>(int(blockIdx.x), L, P, it, Ah, v, x, scs, part);
}

// Couplings of the composite system to other levels, one thread per listed row:
// w[i] -= sum_e val_e r[col_e] with the sweep's new r^; the row's share of (w^, r^)
// goes to this kernel's block partials (fixed order, no atomics).
__global__ __launch_bounds__(kBlock) void k_interface(DevLevel L, const double* __restrict__ r,
                                                      double* __restrict__ w, const PcgScalars* sc,
                                                      double* __restrict__ part_if) {
  __shared__ double lds[kLds];
  if (sc->done) return;  // uniform: set by a previous kernel
  const int t = int(blockIdx.x) * kBlock + int(threadIdx.x);
  double v[1] = {0.0};
  if (t < L.n_if_rows) {
    const int i = L.if_row[t];
    const int e0 = L.if_ptr[t], e1 = L.if_ptr[t + 1];
    double acc = 0.0;
#pragma unroll 4
    for (int e = e0; e < e1; ++e) acc += L.if_val[e] * r[L.if_col[e]];
    w[i] -= acc;
    v[0] = -r[i] * acc;
  }
  const bool mx[1] = {false};
  write_partials<1>(v, mx, part_if, lds, int(blockIdx.x));
}

__global__ __launch_bounds__(kBlock) void k_true_residual(DevLevel L, SweepPlan P, FaceCoefs<double> A,
                                                          const double* __restrict__ diag,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ x, double* part) {
  body_true_residual(int(blockIdx.x), L, P, A, diag, b, x, part);
}

__global__ __launch_bounds__(kBlock) void k_true_residual_staged(DevLevel L, SweepPlan P, ScaledOp<double> Ah,
                                                                 const double* __restrict__ b,
                                                                 const double* __restrict__ x, double* part) {
  body_true_residual_staged(int(blockIdx.x), L, P, Ah, b, x, part);
}

__global__ __launch_bounds__(kBlock) void k_post_solve(DevLevel L, SweepPlan P, const double* __restrict__ E,
                                                       const double* __restrict__ rho, CouplingParams cp,
                                                       double dt, double* __restrict__ T_out, double* part) {
  body_post_solve(int(blockIdx.x), L, P, E, rho, cp, dt, T_out, part);
}

__global__ __launch_bounds__(kBlock) void k_ir_sweep(DevLevel L, SweepPlan P, ScaledOp<double> Ah,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x_old,
                                                     const float* __restrict__ d, const float* __restrict__ p32,
                                                     const float* __restrict__ rs32, double* __restrict__ x_new,
                                                     float* __restrict__ r32, const PcgScalars* outer,
                                                     const PcgScalars* inner, double* part) {
  body_ir_sweep(int(blockIdx.x), L, P, Ah, b, x_old, d, p32, rs32, x_new, r32, outer, inner, part);
}

__global__ __launch_bounds__(kBlock) void k_inner_init(DevLevel L, SweepPlan P, ScaledOp<float> Ah,
                                                       const float* __restrict__ r32, float* __restrict__ d,
                                                       CgVecs<float> v, const PcgScalars* outer,
                                                       const PcgScalars* inner, double* part) {
  body_inner_init(int(blockIdx.x), L, P, Ah, r32, d, v, outer, inner, part);
}

__global__ __launch_bounds__(kBlock) void k_check(SweepPlan P, int it_last, PcgScalars* scs, const double* part) {
  body_check(int(blockIdx.x), P, it_last, scs, part);
}

__global__ __launch_bounds__(kBlock) void k_finish(SweepPlan P, int kind, const double* part, PcgScalars* scs) {
  body_finish(int(blockIdx.x), P, kind, part, scs);
}

__global__ __launch_bounds__(kBlock) void k_ir_finish(SweepPlan P, int first, double inner_tol, int max_outer,
                                                      PcgScalars* outs, PcgScalars* ins, const double* part) {
  body_ir_finish(int(blockIdx.x), P, first, inner_tol, max_outer, outs, ins, part, nullptr);
}

// All CG iterations of every problem of the plan in one cooperative launch: the G
// virtual blocks of each iteration sweep are dealt round-robin to the resident
// blocks, with a grid barrier after each sweep.  The loop ends once every problem
// has stopped (read right after the barrier, the stops being counted at the sweep
// heads), and in any case after max_iter + 1 sweeps.  A barrier that times out sets
// the abort flag and the block returns; the others then time out at their next
// barrier, so the launch always ends.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_persistent(DevLevel L, SweepPlan P, int max_iter, ScaledOp<T> Ah,
                                                           CgVecs<T> v, T* x, PcgScalars* scs, double* part,
                                                           unsigned* bar, unsigned spin_limit) {
  __shared__ unsigned n_done;
  const unsigned nb = gridDim.x;
  dev::GridSync gs{bar, nb, spin_limit};
  for (int it = 1; it <= max_iter + 1; ++it) {
    for (int vb = int(blockIdx.x); vb < P.G; vb += int(nb)) body_cg_sweep<T>(vb, L, P, it, Ah, v, x, scs, part);
    if (!grid_barrier(gs)) {
      if (threadIdx.x == 0) __hip_atomic_store(bar + kBarAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if (threadIdx.x == 0) n_done = __hip_atomic_load(P.done_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (n_done >= unsigned(P.n_prob)) break;
  }
}

// The whole mixed-precision solve of every problem of the plans in one cooperative
// launch: rounds of (FP64 refinement sweep, outer stopping test, inner start, FP32
// inner iteration sweeps) with a grid barrier after each phase, the same bodies in
// the same order and with the same plans (P for the FP64 sweeps, P32 for the FP32
// ones) as the host-driven launches, so the results are the same bits.
// Every decision is made on the device (body_ir_finish); the loop ends once every
// problem's refinement has stopped (a count read right after the barrier that
// follows the outer test) and in any case after max_outer + 1 refinement sweeps; an
// inner solve ends once every problem's inner CG stopped, and in any case after
// inner_cap + 1 sweeps.  A barrier that times out sets the abort flag and the
// block returns (the others time out in turn).
__global__ __launch_bounds__(kBlock) void k_mixed_persistent(DevLevel L, SweepPlan P, SweepPlan P32, MixedArgs M) {
  __shared__ unsigned n_done;
  const unsigned nb = gridDim.x;
  dev::GridSync gs{M.bar, nb, M.spin_limit};
  unsigned* inner_done = P32.done_count;
  unsigned* outer_done = M.bar + kBarOuterDone;
  double* x_cur = M.x;
  double* x_nxt = M.x_alt;
  auto sync = [&]() -> bool {
    if (grid_barrier(gs)) return true;
    if (threadIdx.x == 0) __hip_atomic_store(M.bar + kBarAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  };
  auto read_count = [&](unsigned* w) {
    if (threadIdx.x == 0) n_done = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    return n_done;
  };
  for (int outer = 0; outer <= M.max_outer; ++outer) {
    for (int vb = int(blockIdx.x); vb < P.G; vb += int(nb))
      body_ir_sweep(vb, L, P, M.Ah, M.b, x_cur, outer == 0 ? nullptr : M.d32, M.v32.p, M.Ah32.rs, x_nxt, M.r32,
                    M.outer, M.inner, M.part);
    if (!sync()) return;
    double* t = x_cur;
    x_cur = x_nxt;
    x_nxt = t;
    for (int q = int(blockIdx.x); q < P.n_prob; q += int(nb))
      body_ir_finish(q, P, outer == 0 ? 1 : 0, M.inner_tol, M.max_outer, M.outer, M.inner, M.part, outer_done);
    // the inner stop count restarts for this round's inner solves (no block reads it
    // again before the barrier below)
    if (blockIdx.x == 0 && threadIdx.x == 0)
      __hip_atomic_store(inner_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!sync()) return;
    if (read_count(outer_done) >= unsigned(P.n_prob)) break;
    for (int vb = int(blockIdx.x); vb < P32.G; vb += int(nb))
      body_inner_init(vb, L, P32, M.Ah32, M.r32, M.d32, M.v32, M.outer, M.inner, M.part);
    if (!sync()) return;
    for (int it = 1; it <= M.inner_cap + 1; ++it) {
      for (int vb = int(blockIdx.x); vb < P32.G; vb += int(nb))
        body_cg_sweep<float>(vb, L, P32, it, M.Ah32, M.v32, M.d32, M.inner, M.part);
      if (!sync()) return;
      // stops are counted only at the sweep heads (see k_pcg_persistent)
      if (read_count(inner_done) >= unsigned(P32.n_prob)) break;
    }
  }
  // the last refinement sweep wrote x_cur: make it the caller's iterate
  if (x_cur != M.x) {
    for (int i = int(blockIdx.x) * kBlock + int(threadIdx.x); i < L.n_slots; i += int(nb) * kBlock)
      M.x[i] = x_cur[i];
  }
}

__global__ __launch_bounds__(kBlock) void k_init_scalars(PcgScalars* sc, int n, double tol, double abs_floor,
                                                         int max_iter, int linf_test) {
  const int i = int(blockIdx.x * kBlock + threadIdx.x);
  if (i >= n) return;
  PcgScalars z{};
  z.tol = tol;
  z.abs_floor = abs_floor;
  z.max_iter = max_iter;
  z.linf_test = linf_test;
  sc[i] = z;
}

__global__ __launch_bounds__(kBlock) void k_copy_scalars(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                                                         int n_words, int to_host) {
  const int i = int(blockIdx.x * kBlock + threadIdx.x);
  if (i < n_words) dst[i] = src[i];
  if (to_host) __threadfence_system();
}

__global__ __launch_bounds__(kBlock) void k_zero_u32(unsigned* p, int n) {
  const int i = int(blockIdx.x * kBlock + threadIdx.x);
  if (i < n) p[i] = 0u;
}

// Scaled interface coefficients of the composite system, one thread per listed row.
__global__ __launch_bounds__(kBlock) void k_interface_values(DevLevel L, const double* __restrict__ cif,
                                                             const double* __restrict__ rs,
                                                             double* __restrict__ val) {
  const int t = int(blockIdx.x) * kBlock + int(threadIdx.x);
  if (t >= L.n_if_rows) return;
  const int i = L.if_row[t];
  for (int e = L.if_ptr[t]; e < L.if_ptr[t + 1]; ++e) val[e] = cif[L.if_src[e]] * (rs[i] * rs[L.if_col[e]]);
}

}  // namespace

// ------------------------------------------------------------ launchers
template <typename T>
void launch_cg_start(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<T>& Ah, const T* b,
                     const T* x, const CgVecs<T>& v, double* part) {
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(T);
  hipLaunchKernelGGL(k_cg_start_r<T>, dim3(P.G), dim3(kBlock), lds, s, L, P, Ah, b, x, v);
  hipLaunchKernelGGL(k_cg_start_w<T>, dim3(P.G), dim3(kBlock), lds, s, L, P, Ah, b, v, part);
}

template <typename T>
void launch_cg_init_r(hipStream_t s, const DevLevel& L, const SweepPlan& P, const FaceCoefs<T>& A, const T* diag,
                      const T* b, const T* x, const T* rs, const CgVecs<T>& v) {
  hipLaunchKernelGGL(k_cg_init_r<T>, dim3(P.G), dim3(kBlock), 0, s, L, P, A, diag, b, x, rs, v);
}

template <typename T>
void launch_cg_init_w(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<T>& Ah, const T* b,
                      const CgVecs<T>& v, double* part) {
  hipLaunchKernelGGL(k_cg_init_w<T>, dim3(P.G), dim3(kBlock), 0, s, L, P, Ah, b, v, part);
}

template <typename T>
void launch_cg_sweep(hipStream_t s, const DevLevel& L, const SweepPlan& P, int it, const ScaledOp<T>& Ah,
                     const CgVecs<T>& v, T* x, PcgScalars* sc, double* part, hipEvent_t t0, hipEvent_t t1) {
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(T);
  if (t0)
    hipExtLaunchKernelGGL(k_cg_sweep<T>, dim3(P.G), dim3(kBlock), uint32_t(lds), s, t0, t1, 0u, L, P, it, Ah, v, x,
                          sc, part);
  else
    hipLaunchKernelGGL(k_cg_sweep<T>, dim3(P.G), dim3(kBlock), lds, s, L, P, it, Ah, v, x, sc, part);
}

int interface_blocks(const DevLevel& L) { return std::max(1, (L.n_if_rows + kBlock - 1) / kBlock); }

void launch_interface_values(hipStream_t s, const DevLevel& L, int n_entries, const double* cif, const double* rs,
                             double* val) {
  if (n_entries <= 0 || L.n_if_rows <= 0) return;
  hipLaunchKernelGGL(k_interface_values, dim3(interface_blocks(L)), dim3(kBlock), 0, s, L, cif, rs, val);
}

void launch_interface(hipStream_t s, const DevLevel& L, const double* r, double* w, const PcgScalars* sc,
                      double* part_if) {
  hipLaunchKernelGGL(k_interface, dim3(interface_blocks(L)), dim3(kBlock), 0, s, L, r, w, sc, part_if);
}

void launch_check(hipStream_t s, const SweepPlan& P, int it_last, PcgScalars* sc, const double* part) {
  hipLaunchKernelGGL(k_check, dim3(P.n_prob), dim3(kBlock), 0, s, P, it_last, sc, part);
}

void launch_true_residual(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<double>& Ah,
                          const double* b, const double* x, PcgScalars* sc, double* part) {
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(double);
  hipLaunchKernelGGL(k_true_residual_staged, dim3(P.G), dim3(kBlock), lds, s, L, P, Ah, b, x, part);
  hipLaunchKernelGGL(k_finish, dim3(P.n_prob), dim3(kBlock), 0, s, P, 0, part, sc);
}

void launch_true_residual(hipStream_t s, const DevLevel& L, const SweepPlan& P, const FaceCoefs<double>& A,
                          const double* diag, const double* b, const double* x, PcgScalars* sc, double* part) {
  hipLaunchKernelGGL(k_true_residual, dim3(P.G), dim3(kBlock), 0, s, L, P, A, diag, b, x, part);
  hipLaunchKernelGGL(k_finish, dim3(P.n_prob), dim3(kBlock), 0, s, P, 0, part, sc);
}

void launch_post_solve(hipStream_t s, const DevLevel& L, const SweepPlan& P, const double* E, const double* rho,
                       const CouplingParams& cp, double dt, double* T_out, PcgScalars* sc, double* part) {
  hipLaunchKernelGGL(k_post_solve, dim3(P.G), dim3(kBlock), 0, s, L, P, E, rho, cp, dt, T_out, part);
  hipLaunchKernelGGL(k_finish, dim3(P.n_prob), dim3(kBlock), 0, s, P, 1, part, sc);
}

void launch_ir_sweep(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<double>& Ah,
                     const double* b, const double* x_old, const float* d, const float* p32, const float* rs32,
                     double* x_new, float* r32, const PcgScalars* outer, const PcgScalars* inner, double* part) {
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(double);
  hipLaunchKernelGGL(k_ir_sweep, dim3(P.G), dim3(kBlock), lds, s, L, P, Ah, b, x_old, d, p32, rs32, x_new, r32,
                     outer, inner, part);
}

void launch_ir_finish(hipStream_t s, const SweepPlan& P, int first, double inner_tol, int max_outer,
                      PcgScalars* outer, PcgScalars* inner, const double* part) {
  hipLaunchKernelGGL(k_ir_finish, dim3(P.n_prob), dim3(kBlock), 0, s, P, first, inner_tol, max_outer, outer,
                     inner, part);
}

void launch_inner_init(hipStream_t s, const DevLevel& L, const SweepPlan& P, const ScaledOp<float>& Ah,
                       const float* r32, float* d, const CgVecs<float>& v, const PcgScalars* outer,
                       const PcgScalars* inner, double* part) {
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(float);
  hipLaunchKernelGGL(k_inner_init, dim3(P.G), dim3(kBlock), lds, s, L, P, Ah, r32, d, v, outer, inner, part);
}

void launch_init_scalars(hipStream_t s, PcgScalars* sc, int n, double tol, double abs_floor, int max_iter,
                         int linf_test) {
  hipLaunchKernelGGL(k_init_scalars, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, sc, n, tol, abs_floor,
                     max_iter, linf_test);
}

void launch_copy_scalars(hipStream_t s, const PcgScalars* src, PcgScalars* dst, int count, bool to_host) {
  static_assert(sizeof(PcgScalars) % sizeof(uint64_t) == 0, "scalar records are whole words");
  const int n_words = count * int(sizeof(PcgScalars) / sizeof(uint64_t));
  if (n_words <= 0) return;
  hipLaunchKernelGGL(k_copy_scalars, dim3((n_words + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     reinterpret_cast<const uint64_t*>(src), reinterpret_cast<uint64_t*>(dst), n_words,
                     to_host ? 1 : 0);
}

void launch_zero_u32(hipStream_t s, unsigned* p, int n) {
  hipLaunchKernelGGL(k_zero_u32, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, p, n);
}

// Resident blocks of a cooperative kernel with the iteration sweep's LDS for this
// plan on this device (0 if unknown or not supported).
int resident_blocks(const void* kernel, size_t lds, int per_cu_cap) {
  int dev = 0, cus = 0, per_cu = 0, coop = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, lds) != hipSuccess) return 0;
  if (per_cu_cap > 0) per_cu = std::min(per_cu, per_cu_cap);
  return per_cu * cus;
}

template <typename T>
int persistent_blocks(const SweepPlan& P, int per_cu_cap) {
  const int res = resident_blocks(reinterpret_cast<const void*>(&k_pcg_persistent<T>),
                                  size_t(P.tpb_max) * kBlock * sizeof(T), per_cu_cap);
  return res > 0 ? std::min(P.G, res) : 0;
}

template int persistent_blocks<double>(const SweepPlan&, int);
template int persistent_blocks<float>(const SweepPlan&, int);

template <typename T>
hipError_t launch_pcg_persistent(hipStream_t s, const DevLevel& L, const SweepPlan& P, int max_iter,
                                 const ScaledOp<T>& Ah, const CgVecs<T>& v, T* x, PcgScalars* sc, double* part,
                                 unsigned* bar, int per_cu_cap) {
  const int grid = persistent_blocks<T>(P, per_cu_cap);
  if (grid <= 0) return hipErrorNotSupported;
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(T);
  // bounded barrier wait: ~2^26 polls of ~0.1 us, far above the longest sweep
  unsigned spin_limit = 1u << 26;
  DevLevel Lv = L;
  SweepPlan Pv = P;
  ScaledOp<T> Av = Ah;
  CgVecs<T> vv = v;
  void* args[] = {&Lv, &Pv, &max_iter, &Av, &vv, &x, &sc, &part, &bar, &spin_limit};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_pcg_persistent<T>), dim3(grid), dim3(kBlock),
                                    args, unsigned(lds), s);
}

// The refinement sweeps stage FP64 values over P's ranges, the inner sweeps FP32
// ones over P32's.
size_t mixed_persistent_lds(const SweepPlan& P, const SweepPlan& P32) {
  return std::max(size_t(P.tpb_max) * sizeof(double), size_t(P32.tpb_max) * sizeof(float)) * kBlock;
}

int mixed_persistent_blocks(const SweepPlan& P, const SweepPlan& P32, int per_cu_cap) {
  const int res = resident_blocks(reinterpret_cast<const void*>(&k_mixed_persistent),
                                  mixed_persistent_lds(P, P32), per_cu_cap);
  return res > 0 ? std::min(std::max(P.G, P32.G), res) : 0;
}

hipError_t launch_mixed_persistent(hipStream_t s, const DevLevel& L, const SweepPlan& P, const SweepPlan& P32,
                                   const MixedArgs& M, int per_cu_cap) {
  const int grid = mixed_persistent_blocks(P, P32, per_cu_cap);
  if (grid <= 0) return hipErrorNotSupported;
  const size_t lds = mixed_persistent_lds(P, P32);
  DevLevel Lv = L;
  SweepPlan Pv = P;
  SweepPlan P32v = P32;
  MixedArgs Mv = M;
  void* args[] = {&Lv, &Pv, &P32v, &Mv};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_mixed_persistent), dim3(grid), dim3(kBlock),
                                    args, unsigned(lds), s);
}

template hipError_t launch_pcg_persistent<double>(hipStream_t, const DevLevel&, const SweepPlan&, int,
                                                  const ScaledOp<double>&, const CgVecs<double>&, double*,
                                                  PcgScalars*, double*, unsigned*, int);
template hipError_t launch_pcg_persistent<float>(hipStream_t, const DevLevel&, const SweepPlan&, int,
                                                 const ScaledOp<float>&, const CgVecs<float>&, float*, PcgScalars*,
                                                 double*, unsigned*, int);
template void launch_cg_start<double>(hipStream_t, const DevLevel&, const SweepPlan&, const ScaledOp<double>&,
                                      const double*, const double*, const CgVecs<double>&, double*);
template void launch_cg_init_r<double>(hipStream_t, const DevLevel&, const SweepPlan&, const FaceCoefs<double>&,
                                       const double*, const double*, const double*, const double*,
                                       const CgVecs<double>&);
template void launch_cg_init_w<double>(hipStream_t, const DevLevel&, const SweepPlan&, const ScaledOp<double>&,
                                       const double*, const CgVecs<double>&, double*);
template void launch_cg_sweep<double>(hipStream_t, const DevLevel&, const SweepPlan&, int, const ScaledOp<double>&,
                                      const CgVecs<double>&, double*, PcgScalars*, double*, hipEvent_t, hipEvent_t);
template void launch_cg_sweep<float>(hipStream_t, const DevLevel&, const SweepPlan&, int, const ScaledOp<float>&,
                                     const CgVecs<float>&, float*, PcgScalars*, double*, hipEvent_t, hipEvent_t);

}  // namespace amrfld
