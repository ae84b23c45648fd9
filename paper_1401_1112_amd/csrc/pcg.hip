// Jacobi-preconditioned conjugate gradient on one level (Sect. 3.3.4) as two
// fused sweeps per iteration, plus the FP64 iterative-refinement sweeps of the
// mixed-precision form.
//
// Reductions without atomics: every sweep runs G blocks, each block sweeps a
// contiguous range of 256-slot tiles and writes one partial per reduced
// quantity.  The NEXT sweep reduces all G partials at its head, in the same
// fixed order in every block, and derives alpha, beta and the stopping
// decision itself; the kernel boundary makes the partials visible.  Runs are
// therefore bitwise reproducible.  Scalars that a sweep writes and later
// sweeps read are double-buffered by iteration parity.
//
// Partial buffer: [0, G) operator-sweep partial (p, q); [G, 4G) update-sweep
// partials (r, z), ||r||^2, max relative change (also used by the start sweeps).
#include <hip/hip_ext.h>

#include <algorithm>

#include "common.h"

namespace amrfld {

// At most kMaxTilesPerBlock tiles per block: the operator sweep stages the
// block's whole range of the new p in LDS (16 tiles = 32 KB in FP64).  A level
// with more than max_blocks * 16 tiles gets a whole multiple of max_blocks, so
// that the blocks of a persistent launch of max_blocks blocks each sweep the
// same number of equal ranges.
int sweep_blocks(int n_tiles, int max_blocks) {
  const int B = std::max(1, max_blocks);
  if (n_tiles <= B) return std::max(1, n_tiles);
  const int64_t rounds = (int64_t(n_tiles) + int64_t(B) * kMaxTilesPerBlock - 1) / (int64_t(B) * kMaxTilesPerBlock);
  return int(rounds * B);
}

namespace {

using dev::apply_stencil;
using dev::block_plan;
using dev::block_read_flag;
using dev::block_reduce;
using dev::BlockPlan;
using dev::grid_barrier;
using dev::problem_blocks;
using dev::reduce_partials_all;

constexpr int kLds = (kBlock / 64) * 3 + 4;

template <typename T>
__device__ __forceinline__ T rel_change(T x, T dx) {
  const T ax = fabs(x);
  return ax > T(0) ? fabs(dx) / ax : fabs(dx);
}

// Stopping test of Sect. 3.3.4 for the iterate completed by the previous update
// sweep: ||r|| <= thresh AND (optionally) the largest relative change < tol.
struct StopTest {
  double rz, rn, linf;
  bool fin, conv, stop;
};

// partB: the problem's update-sweep partials (3 per block, Gp blocks).
__device__ __forceinline__ StopTest stop_test(const PcgScalars* sc, const double* partB, int Gp, int it_done,
                                              double* lds) {
  double v[3];
  const bool mx[3] = {false, false, true};
  reduce_partials_all<3>(partB, Gp, mx, v, lds);
  StopTest s;
  s.rz = v[0];
  s.rn = sqrt(v[1]);
  s.linf = v[2];
  s.fin = isfinite(s.rn) && isfinite(s.rz);
  s.conv = s.fin && ((s.rn <= sc->thresh && (!sc->linf_test || s.linf < sc->tol)) || s.rn == 0.0);
  s.stop = !s.fin || s.conv || it_done >= sc->max_iter;
  return s;
}

// Marks a problem stopped.  The done counter (which ends the persistent sweep)
// is only advanced from the start sweeps, the operator sweep and the check, so
// that every block reads the same count right after a grid barrier; a stop
// found in the update sweep is counted by the next operator sweep.
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

// r0 = b - A x0, p = 0; partials (r, r / d), ||r||^2, ||b||^2.
template <typename T>
__device__ __forceinline__ void body_pcg_init(int vb, DevLevel L, SweepPlan P, const FaceCoefs<T>& A,
                                                     const T* __restrict__ diag, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ r,
                                                     T* __restrict__ p_clear, double* part) {
  __shared__ double lds[kLds];
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  const T scale = dev::coef_scale(A, L, bp.prob);
  double v[3] = {0.0, 0.0, 0.0};
  for (int t = bp.t0; t < bp.t1; ++t) {
    const int i = t * kBlock + int(threadIdx.x);
    const bool valid = i < n;
    const int ii = valid ? i : n - 1;
    const T di = diag[ii];
    T ax = apply_stencil<T>(ii, L.nbr, A, scale, n, di, x[ii], [&](int j) { return x[j]; });
    if (L.cif) ax -= dev::interface_terms<T>(ii, L, n, [&](int j) { return x[j]; });
    if (valid) {
      const T ri = b[i] - ax;
      r[i] = ri;
      p_clear[i] = T(0);
      const double rd = double(ri);
      v[0] += rd * double(ri / di);
      v[1] += rd * rd;
      // ||b|| over the unknowns only: identity rows (refined and padding slots) hold
      // b = E there, which is no part of the system
      if (L.child[i] == -1) v[2] += double(b[i]) * double(b[i]);
    }
  }
  const bool mx[3] = {false, false, false};
  write_partials<3>(v, mx, part + P.G, lds, vb);
}

// One block per problem.  A problem already marked done (the inner solve of a
// converged problem in the batched refinement) is left as it is.
__device__ __forceinline__ void body_init_finish(int prob, SweepPlan P, const double* part, PcgScalars* scs) {
  __shared__ double lds[kLds];
  int b0, Gp;
  problem_blocks(P, prob, b0, Gp);
  PcgScalars* sc = scs + prob;
  if (sc->done) return;
  double v[3];
  const bool mx[3] = {false, false, false};
  reduce_partials_all<3>(part + P.G + 3 * b0, Gp, mx, v, lds);
  if (threadIdx.x == 0) {
    const double r0 = sqrt(v[1]), bn = sqrt(v[2]);
    const double floor_b = sc->abs_floor * bn;
    sc->rho[0] = v[0];
    sc->rho[1] = v[0];
    sc->rnorm0 = r0;
    sc->rnorm = r0;
    sc->bnorm = bn;
    sc->thresh = fmax(sc->tol * r0, floor_b);
    sc->iter = 0;
    sc->linf = 0.0;
    const bool fin = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
    sc->nonfinite = fin ? 0 : 1;
    // ||r_0|| <= abs_floor ||b||: x_0 is returned after 0 iterations
    sc->converged = (fin && r0 <= floor_b) ? 1 : 0;
    if (!fin || r0 <= floor_b) mark_done(sc, P);
  }
}

// Phase 2 of the operator sweep with face coefficients formed from K: as the
// stored form below, but each slot reads its K and face mask, takes its sibling's
// K by shuffle and gathers K of the out-of-oct neighbours it is coupled to.
template <typename T, int U2>
__device__ __forceinline__ void operator_formed(const DevLevel& L, const FaceCoefs<T>& A, T scale, bool first, T tb,
                                                int s0, int s1, int t0, int t1, const T* pl,
                                                const T* __restrict__ diag, const T* __restrict__ r,
                                                const T* __restrict__ p_old, T* __restrict__ q, double& pq) {
  const int n = L.n_slots;
  const T th = T(A.theta);
  const T* __restrict__ K = A.K;
  for (int tb0 = t0; tb0 < t1; tb0 += U2) {
    int ii[U2], nbv[U2][3];
    unsigned mk[U2];
    T dg[U2], kown[U2];
    bool valid[U2];
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const int i = (tb0 + u) * kBlock + int(threadIdx.x);
      valid[u] = (tb0 + u < t1) && i < n;
      ii[u] = valid[u] ? i : s1 - 1;
      const int pos = ii[u] & 7, o = ii[u] >> 3;
      dg[u] = diag[ii[u]];
      kown[u] = K[ii[u]];
      mk[u] = A.mask[ii[u]];
#pragma unroll
      for (int a = 0; a < 3; ++a) nbv[u][a] = L.nbr[o * 6 + 2 * a + ((pos >> a) & 1)];
    }
    // gathers: K of the coupled out-of-oct neighbours, and the inputs of p at
    // neighbours outside the block's range (lanes that need none read their own)
    int jv[U2][3];
    T kj[U2][3], rj[U2][3], dj[U2][3], pj[U2][3];
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const int pos = ii[u] & 7;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int nb = nbv[u][a];
        const bool cpl = nb >= 0 && ((mk[u] >> (2 * a + ((pos >> a) & 1))) & 1u);
        const int j = cpl ? ((nb << 3) | (pos ^ (1 << a))) : ii[u];
        jv[u][a] = cpl ? j : -1;
        const int jo = (j >= s0 && j < s1) ? s0 : j;  // as in the stored form below
        kj[u][a] = K[j];
        rj[u][a] = r[jo];
        dj[u][a] = diag[jo];
        pj[u][a] = p_old[jo];
      }
    }
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const int pos = ii[u] & 7;
      const T pi = valid[u] ? pl[ii[u] - s0] : T(0);
      const T Ki = kown[u];
      T acc = dg[u] * pi;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int bit = 1 << a;
        const T p_sib = __shfl_xor(pi, bit, 64);
        const T K_sib = __shfl_xor(Ki, bit, 64);
        const int my = (pos >> a) & 1;
        const T c_in = ((mk[u] >> (2 * a + 1 - my)) & 1u) ? dev::face_coef(Ki, K_sib, scale, th) : T(0);
        acc -= c_in * p_sib;
        const int j = jv[u][a];
        if (j >= 0) {
          const T c_out = dev::face_coef(Ki, kj[u][a], scale, th);
          T pn;
          if (j >= s0 && j < s1) {
            pn = pl[j - s0];
          } else {
            const T z = rj[u][a] / dj[u][a];
            pn = first ? z : fma(tb, pj[u][a], z);
          }
          acc -= c_out * pn;
        }
      }
      if (valid[u]) {
        q[ii[u]] = acc;
        pq += double(pi) * double(acc);
      }
    }
  }
}

// Operator sweep of iteration `it`: p_it = z + beta p_{it-1} with z = r / d formed
// on the fly (p_1 = z), q = A p_it, partial (p, q).
//
// Two phases over the block's contiguous slot range: (1) p_it of every slot of
// the range into LDS (and to p_new); (2) the operator, with in-oct neighbours by
// cross-lane shuffle, out-of-oct neighbours inside the range from LDS, and the
// rest recomputed from r, d and p_{it-1} in global memory (the two p buffers
// alternate, so p_{it-1} is never overwritten during the sweep).
template <typename T>
__device__ __forceinline__ void body_pass_a(int vb, DevLevel L, SweepPlan P, int it,
                                                   const FaceCoefs<T>& A, const T* __restrict__ diag,
                                                   const T* __restrict__ r, const T* __restrict__ p_old,
                                                   T* __restrict__ p_new, T* __restrict__ q,
                                                   PcgScalars* scs, double* part) {
  __shared__ double lds[kLds];
  extern __shared__ unsigned char dyn_lds[];
  T* pl = reinterpret_cast<T*>(dyn_lds);
  const BlockPlan bp = block_plan(P, vb);
  PcgScalars* sc = scs + bp.prob;
  // the problem's first block may set `done` during this sweep
  if (block_read_flag(&sc->done)) {
    if (vb == bp.b0 && threadIdx.x == 0) mark_done(sc, P);
    return;
  }
  const bool first = it == 1;
  const int n = L.n_slots;
  const int t0 = bp.t0, t1 = bp.t1;
  const int s0 = t0 * kBlock;
  const int s1 = min(t1 * kBlock, n);
  // phase 1 loads: U1 slots per thread and trip, the first batch issued before
  // the head reduction (it does not depend on beta) and each next batch before
  // the current one is used
  constexpr int U1 = 4;
  T rv[U1], dv[U1], pv[U1];
  auto load1 = [&](int base) {
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int i = min(base + u * kBlock, s1 - 1);
      rv[u] = r[i];
      dv[u] = diag[i];
      pv[u] = p_old[i];
    }
  };
  int base = s0 + int(threadIdx.x);
  load1(min(base, s1 - 1));
  double beta = 0.0;
  if (!first) {
    const StopTest s = stop_test(sc, part + P.G + 3 * bp.b0, bp.Gp, it - 1, lds);
    if (vb == bp.b0 && threadIdx.x == 0) {
      record_stop(sc, s, it - 1, P);
      if (!s.stop) sc->rho[it & 1] = s.rz;
    }
    if (s.stop) return;
    beta = s.rz / sc->rho[(it - 1) & 1];
  }
  const T tb = T(beta);
  for (; base < s1; base += U1 * kBlock) {
    T pi[U1];
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const T z = rv[u] / dv[u];
      pi[u] = first ? z : fma(tb, pv[u], z);
    }
    if (base + U1 * kBlock < s1) load1(base + U1 * kBlock);
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int i = base + u * kBlock;
      if (i < s1) {
        pl[i - s0] = pi[u];
        p_new[i] = pi[u];
      }
    }
  }
  __syncthreads();
  // phase 2: the operator, U2 tiles per trip
  constexpr int U2 = 2;
  double v[1] = {0.0};
  if (!A.Cp) {  // coefficients formed from K
    operator_formed<T, U2>(L, A, dev::coef_scale(A, L, bp.prob), first, tb, s0, s1, t0, t1, pl, diag, r, p_old, q,
                           v[0]);
    const bool mx[1] = {false};
    write_partials<1>(v, mx, part, lds, vb);
    return;
  }
  const T* __restrict__ Cp = A.Cp;
  for (int tb0 = t0; tb0 < t1; tb0 += U2) {
    int ii[U2], nbv[U2][3];
    T dg[U2], cown[U2][3];
    bool valid[U2];
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const int i = (tb0 + u) * kBlock + int(threadIdx.x);
      valid[u] = (tb0 + u < t1) && i < n;
      ii[u] = valid[u] ? i : s1 - 1;
      const int pos = ii[u] & 7, o = ii[u] >> 3;
      dg[u] = diag[ii[u]];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cown[u][a] = Cp[size_t(a) * n + ii[u]];
        nbv[u][a] = L.nbr[o * 6 + 2 * a + ((pos >> a) & 1)];
      }
    }
    // gathers of the out-of-oct neighbours: coefficient of a -face, and the
    // inputs of p at neighbours outside the block's range
    int jv[U2][3];
    T cj[U2][3], rj[U2][3], dj[U2][3], pj[U2][3];
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const int pos = ii[u] & 7;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int nb = nbv[u][a];
        const int j = nb >= 0 ? ((nb << 3) | (pos ^ (1 << a))) : ii[u];
        jv[u][a] = j;
        const bool inr = j >= s0 && j < s1;
        // no gather needed inside the range: those lanes read the range's first slot
        // (one line, cached) rather than their own, whose lines the first phase read
        // long enough ago to have left L2
        const int jo = inr ? s0 : j;
        // the coefficient of a -face lives at the neighbour; cells on the + side of
        // their oct use their own (already loaded) coefficient instead
        const int jc = ((pos >> a) & 1) ? ii[u] : j;
        cj[u][a] = Cp[size_t(a) * n + jc];
        rj[u][a] = r[jo];
        dj[u][a] = diag[jo];
        pj[u][a] = p_old[jo];
      }
    }
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const int pos = ii[u] & 7;
      const T pi = valid[u] ? pl[ii[u] - s0] : T(0);
      T acc = dg[u] * pi;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int bit = 1 << a;
        const T c_own = cown[u][a];
        const T p_sib = __shfl_xor(pi, bit, 64);
        const T c_sib = __shfl_xor(c_own, bit, 64);
        const int my = (pos >> a) & 1;
        acc -= (my ? c_sib : c_own) * p_sib;
        if (nbv[u][a] >= 0) {
          const int j = jv[u][a];
          const T c_out = my ? c_own : cj[u][a];
          T pn;
          if (j >= s0 && j < s1) {
            pn = pl[j - s0];
          } else {
            const T z = rj[u][a] / dj[u][a];
            pn = first ? z : fma(tb, pj[u][a], z);
          }
          acc -= c_out * pn;
        }
      }
      if (valid[u]) {
        q[ii[u]] = acc;
        v[0] += double(pi) * double(acc);
      }
    }
  }
  const bool mx[1] = {false};
  write_partials<1>(v, mx, part, lds, vb);
}

// Update sweep of iteration `it`: alpha = rho / (p, q); x += alpha p; r -= alpha q;
// partials (r, z), ||r||^2 and max |alpha p| / |x|.
template <typename T>
__device__ __forceinline__ void body_pass_b(int vb, DevLevel L, SweepPlan P, int it,
                                                   const T* __restrict__ diag, const T* __restrict__ p,
                                                   const T* __restrict__ q, T* __restrict__ x,
                                                   T* __restrict__ r, PcgScalars* scs, double* part) {
  __shared__ double lds[kLds];
  const BlockPlan bp = block_plan(P, vb);
  PcgScalars* sc = scs + bp.prob;
  if (block_read_flag(&sc->done)) return;
  const int n = L.n_slots;
  const int t0 = bp.t0, t1 = bp.t1;
  const int s1 = min(t1 * kBlock, n);
  // U slots per thread and trip; the first batch is loaded before the head
  // reduction (it does not depend on alpha), each next one before the current is used
  constexpr int U = 4;
  T xv[U], pv[U], rv[U], qv[U], dv[U];
  auto load = [&](int base) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = min(base + u * kBlock, s1 - 1);
      xv[u] = x[i];
      pv[u] = p[i];
      rv[u] = r[i];
      qv[u] = q[i];
      dv[u] = diag[i];
    }
  };
  int base = t0 * kBlock + int(threadIdx.x);
  load(min(base, s1 - 1));
  double pq[1];
  const bool mx1[1] = {false};
  reduce_partials_all<1>(part + bp.b0, bp.Gp, mx1, pq, lds);
  if (P.extra_part) {  // couplings to other levels, summed after the operator sweep's partials
    double pe[1];
    reduce_partials_all<1>(P.extra_part, P.n_extra, mx1, pe, lds);
    pq[0] += pe[0];
  }
  const double alpha = sc->rho[it & 1] / pq[0];
  if (!isfinite(alpha)) {
    if (vb == bp.b0 && threadIdx.x == 0) {
      sc->nonfinite = 1;
      sc->iter = it - 1;
      mark_done(sc, P, false);
    }
    return;
  }
  const T ta = T(alpha);
  double v[3] = {0.0, 0.0, 0.0};
  for (; base < s1; base += U * kBlock) {
    T xn[U], rn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T dx = ta * pv[u];
      xn[u] = xv[u] + dx;
      rn[u] = rv[u] - ta * qv[u];
      if (base + u * kBlock < s1) {
        v[2] = fmax(v[2], double(rel_change(xv[u], dx)));
        const T z = rn[u] / dv[u];
        v[0] += double(rn[u]) * double(z);
        v[1] += double(rn[u]) * double(rn[u]);
      }
    }
    if (base + U * kBlock < s1) load(base + U * kBlock);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * kBlock;
      if (i < s1) {
        x[i] = xn[u];
        r[i] = rn[u];
      }
    }
  }
  const bool mx[3] = {false, false, true};
  write_partials<3>(v, mx, part + P.G, lds, vb);
}

// Applies the stopping test after the update sweep of iteration it_last (the
// test the next operator sweep would make) so that the host sees convergence.
__device__ __forceinline__ void body_check(int prob, SweepPlan P, int it_last, PcgScalars* scs, const double* part) {
  __shared__ double lds[kLds];
  int b0, Gp;
  problem_blocks(P, prob, b0, Gp);
  PcgScalars* sc = scs + prob;
  if (sc->done) return;
  const StopTest s = stop_test(sc, part + P.G + 3 * b0, Gp, it_last, lds);
  if (threadIdx.x == 0) record_stop(sc, s, it_last, P);
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

// ------------------------------------------------------------ mixed precision
__device__ __forceinline__ void body_ir_sweep(int vb, DevLevel L, SweepPlan P, const FaceCoefs<double>& A,
                                                     const double* __restrict__ diag,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x_old,
                                                     const float* __restrict__ d, double* __restrict__ x_new,
                                                     float* __restrict__ r32, const PcgScalars* outer,
                                                     double* part) {
  __shared__ double lds[kLds];
  const int n = L.n_slots;
  const BlockPlan bp = block_plan(P, vb);
  if (outer[bp.prob].done) {  // converged problem: carry its iterate into the new buffer
    for (int i = bp.t0 * kBlock + int(threadIdx.x); i < min(bp.t1 * kBlock, n); i += kBlock) x_new[i] = x_old[i];
    return;
  }
  auto xv = [&](int j) -> double { return d ? x_old[j] + double(d[j]) : x_old[j]; };
  const double scale = dev::coef_scale(A, L, bp.prob);
  double v[3] = {0.0, 0.0, 0.0};
  for (int t = bp.t0; t < bp.t1; ++t) {
    const int i = t * kBlock + int(threadIdx.x);
    const bool valid = i < n;
    const int ii = valid ? i : n - 1;
    const double xi = xv(ii);
    const double ax = apply_stencil<double>(ii, L.nbr, A, scale, n, diag[ii], xi, xv);
    if (valid) {
      const double ri = b[i] - ax;
      x_new[i] = xi;
      r32[i] = float(ri);
      v[0] += ri * ri;
      if (L.child[i] == -1) v[1] += b[i] * b[i];  // ||b|| over the unknowns only
      if (d) v[2] = fmax(v[2], rel_change(x_old[i], double(d[i])));
    }
  }
  const bool mx[3] = {false, false, true};
  write_partials<3>(v, mx, part + P.G, lds, vb);
}

// One block per problem: the outer stopping test, then the inner scalars.  A
// problem done in an earlier sweep keeps its state and its inner solve is off.
// Every decision of the refinement loop is made here, on the device: the FP64
// stopping test (Sect. 3.3.4 on the true residual), the cap of max_outer refinement
// sweeps and the cap of the outer record's max_iter inner iterations in all (both
// end the loop unconverged).  The inner solve that just ended is added to the
// outer record's count first.  outer_done (or nullptr) counts the problems whose
// loop has ended, for the persistent launch.
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
  in->iter = 0;
  in->counted = 0;
}

__device__ __forceinline__ void body_inner_init(int vb, DevLevel L, SweepPlan P, const float* __restrict__ diag32,
                                                       const float* __restrict__ r32, float* __restrict__ d,
                                                       float* __restrict__ p_clear, const PcgScalars* outer,
                                                       double* part) {
  __shared__ double lds[kLds];
  const BlockPlan bp = block_plan(P, vb);
  if (outer[bp.prob].done) return;
  double v[3] = {0.0, 0.0, 0.0};
  for (int t = bp.t0; t < bp.t1; ++t) {
    const int i = t * kBlock + int(threadIdx.x);
    if (i < L.n_slots) {
      d[i] = 0.0f;
      p_clear[i] = 0.0f;
      const float ri = r32[i];
      const double rd = double(ri);
      v[0] += rd * double(ri / diag32[i]);
      v[1] += rd * rd;
      v[2] += rd * rd;
    }
  }
  const bool mx[3] = {false, false, false};
  write_partials<3>(v, mx, part + P.G, lds, vb);
}

// ------------------------------------------------------------ kernels
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_init(DevLevel L, SweepPlan P, FaceCoefs<T> A,
                                                     const T* __restrict__ diag, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ r,
                                                     T* __restrict__ p_clear, double* part) {
  body_pcg_init<T>(int(blockIdx.x), L, P, A, diag, b, x, r, p_clear, part);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pass_a(DevLevel L, SweepPlan P, int it,
                                                   FaceCoefs<T> A, const T* __restrict__ diag,
                                                   const T* __restrict__ r, const T* __restrict__ p_old,
                                                   T* __restrict__ p_new, T* __restrict__ q,
                                                   PcgScalars* scs, double* part) {
  body_pass_a<T>(int(blockIdx.x), L, P, it, A, diag, r, p_old, p_new, q, scs, part);
}

// Couplings of the composite system to other levels, one thread per listed row:
// q[i] -= sum_e cif[src_e] p[col_e] with the new p of the operator sweep; the row's
// share of (p, q) goes to this kernel's block partials (fixed order, no atomics).
__global__ __launch_bounds__(kBlock) void k_interface(DevLevel L, const double* __restrict__ p,
                                                      double* __restrict__ q, const PcgScalars* sc,
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
    for (int e = e0; e < e1; ++e) acc += L.if_val[e] * p[L.if_col[e]];
    q[i] -= acc;
    v[0] = -p[i] * acc;
  }
  const bool mx[1] = {false};
  write_partials<1>(v, mx, part_if, lds, int(blockIdx.x));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pass_b(DevLevel L, SweepPlan P, int it,
                                                   const T* __restrict__ diag, const T* __restrict__ p,
                                                   const T* __restrict__ q, T* __restrict__ x,
                                                   T* __restrict__ r, PcgScalars* scs, double* part) {
  body_pass_b<T>(int(blockIdx.x), L, P, it, diag, p, q, x, r, scs, part);
}

__global__ __launch_bounds__(kBlock) void k_true_residual(DevLevel L, SweepPlan P, FaceCoefs<double> A,
                                                          const double* __restrict__ diag,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ x, double* part) {
  body_true_residual(int(blockIdx.x), L, P, A, diag, b, x, part);
}

__global__ __launch_bounds__(kBlock) void k_post_solve(DevLevel L, SweepPlan P, const double* __restrict__ E,
                                                       const double* __restrict__ rho, CouplingParams cp,
                                                       double dt, double* __restrict__ T_out, double* part) {
  body_post_solve(int(blockIdx.x), L, P, E, rho, cp, dt, T_out, part);
}

__global__ __launch_bounds__(kBlock) void k_ir_sweep(DevLevel L, SweepPlan P, FaceCoefs<double> A,
                                                     const double* __restrict__ diag,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x_old,
                                                     const float* __restrict__ d, double* __restrict__ x_new,
                                                     float* __restrict__ r32, const PcgScalars* outer,
                                                     double* part) {
  body_ir_sweep(int(blockIdx.x), L, P, A, diag, b, x_old, d, x_new, r32, outer, part);
}

__global__ __launch_bounds__(kBlock) void k_inner_init(DevLevel L, SweepPlan P, const float* __restrict__ diag32,
                                                       const float* __restrict__ r32, float* __restrict__ d,
                                                       float* __restrict__ p_clear, const PcgScalars* outer,
                                                       double* part) {
  body_inner_init(int(blockIdx.x), L, P, diag32, r32, d, p_clear, outer, part);
}

__global__ __launch_bounds__(kBlock) void k_init_finish(SweepPlan P, const double* part, PcgScalars* scs) {
  body_init_finish(int(blockIdx.x), P, part, scs);
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

// All PCG iterations of every problem of the plan in one cooperative launch: the
// G virtual blocks of each sweep are dealt round-robin to the resident blocks,
// with a grid barrier after each sweep.  The loop ends once every problem has
// stopped (read right after the barrier that follows the operator sweep, where
// the stopping tests are made), and in any case after max_iter + 1 operator
// sweeps.  A barrier that times out sets *abort and the block returns; the
// others then time out at their next barrier, so the launch always ends.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_persistent(DevLevel L, SweepPlan P, int max_iter, FaceCoefs<T> A,
                                                           const T* diag, T* x, T* r, T* p0, T* p1, T* q,
                                                           PcgScalars* scs, double* part, unsigned* bar,
                                                           unsigned spin_limit) {
  __shared__ unsigned n_done;
  const unsigned nb = gridDim.x;
  dev::GridSync gs{bar, nb, spin_limit};
  for (int it = 1; it <= max_iter + 1; ++it) {
    T* pn = (it & 1) ? p1 : p0;
    const T* po = (it & 1) ? p0 : p1;
    for (int vb = int(blockIdx.x); vb < P.G; vb += int(nb))
      body_pass_a<T>(vb, L, P, it, A, diag, r, po, pn, q, scs, part);
    if (!grid_barrier(gs)) {
      if (threadIdx.x == 0) __hip_atomic_store(bar + kBarAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    // stops are counted only in the operator sweep, so the count is the same for
    // every block between this barrier and the next
    if (threadIdx.x == 0) n_done = __hip_atomic_load(P.done_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (n_done >= unsigned(P.n_prob)) break;
    for (int vb = int(blockIdx.x); vb < P.G; vb += int(nb))
      body_pass_b<T>(vb, L, P, it, diag, pn, q, x, r, scs, part);
    if (!grid_barrier(gs)) {
      if (threadIdx.x == 0) __hip_atomic_store(bar + kBarAbort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
  }
}

// The whole mixed-precision solve of every problem of the plan in one cooperative
// launch: rounds of (FP64 refinement sweep, outer stopping test, inner start, inner
// scalars, FP32 inner PCG iterations) with a grid barrier after each phase, the
// same bodies in the same order as the host-driven launches, so the results are
// the same bits.  Every decision is made on the device (body_ir_finish); the loop
// ends once every problem's refinement has stopped (a count read right after the
// barrier that follows the outer test) and in any case after max_outer + 1
// refinement sweeps; an inner solve ends once every problem's inner PCG stopped,
// and in any case after inner_cap + 1 operator sweeps.  A barrier that times out
// sets the abort flag and the block returns (the others time out in turn).
__global__ __launch_bounds__(kBlock) void k_mixed_persistent(DevLevel L, SweepPlan P, MixedArgs M) {
  __shared__ unsigned n_done;
  const unsigned nb = gridDim.x;
  dev::GridSync gs{M.bar, nb, M.spin_limit};
  unsigned* inner_done = P.done_count;
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
      body_ir_sweep(vb, L, P, M.A, M.diag, M.b, x_cur, outer == 0 ? nullptr : M.d32, x_nxt, M.r32, M.outer,
                    M.part);
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
    for (int vb = int(blockIdx.x); vb < P.G; vb += int(nb))
      body_inner_init(vb, L, P, M.diag32, M.r32, M.d32, M.p32[0], M.outer, M.part);
    if (!sync()) return;
    for (int q = int(blockIdx.x); q < P.n_prob; q += int(nb)) body_init_finish(q, P, M.part, M.inner);
    if (!sync()) return;
    for (int it = 1; it <= M.inner_cap + 1; ++it) {
      float* pn = M.p32[it & 1];
      const float* po = M.p32[(it & 1) ^ 1];
      for (int vb = int(blockIdx.x); vb < P.G; vb += int(nb))
        body_pass_a<float>(vb, L, P, it, M.A32, M.diag32, M.r32, po, pn, M.q32, M.inner, M.part);
      if (!sync()) return;
      // stops are counted only in the operator sweep (see k_pcg_persistent)
      if (read_count(inner_done) >= unsigned(P.n_prob)) break;
      for (int vb = int(blockIdx.x); vb < P.G; vb += int(nb))
        body_pass_b<float>(vb, L, P, it, M.diag32, pn, M.q32, M.d32, M.r32, M.inner, M.part);
      if (!sync()) return;
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

}  // namespace

// ------------------------------------------------------------ launchers
template <typename T>
void launch_pcg_init(hipStream_t s, const DevLevel& L, const SweepPlan& P, const FaceCoefs<T>& A, const T* diag,
                     const T* b, const T* x, T* r, T* p_clear, double* part) {
  hipLaunchKernelGGL(k_pcg_init<T>, dim3(P.G), dim3(kBlock), 0, s, L, P, A, diag, b, x, r, p_clear, part);
}

void launch_init_finish(hipStream_t s, const SweepPlan& P, const double* part, PcgScalars* sc) {
  hipLaunchKernelGGL(k_init_finish, dim3(P.n_prob), dim3(kBlock), 0, s, P, part, sc);
}

template <typename T>
void launch_pass_a(hipStream_t s, const DevLevel& L, const SweepPlan& P, int it, const FaceCoefs<T>& A, const T* diag,
                   const T* r, const T* p_old, T* p_new, T* q, PcgScalars* sc, double* part, hipEvent_t t0,
                   hipEvent_t t1) {
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(T);
  if (t0)
    hipExtLaunchKernelGGL(k_pass_a<T>, dim3(P.G), dim3(kBlock), uint32_t(lds), s, t0, t1, 0u, L, P, it, A, diag,
                          r, p_old, p_new, q, sc, part);
  else
    hipLaunchKernelGGL(k_pass_a<T>, dim3(P.G), dim3(kBlock), lds, s, L, P, it, A, diag, r, p_old, p_new, q, sc,
                       part);
}

template <typename T>
void launch_pass_b(hipStream_t s, const DevLevel& L, const SweepPlan& P, int it, const T* diag, const T* p,
                   const T* q, T* x, T* r, PcgScalars* sc, double* part, hipEvent_t t0, hipEvent_t t1) {
  if (t0)
    hipExtLaunchKernelGGL(k_pass_b<T>, dim3(P.G), dim3(kBlock), 0u, s, t0, t1, 0u, L, P, it, diag, p, q, x, r, sc,
                          part);
  else
    hipLaunchKernelGGL(k_pass_b<T>, dim3(P.G), dim3(kBlock), 0, s, L, P, it, diag, p, q, x, r, sc, part);
}

__global__ __launch_bounds__(kBlock) void k_interface_values(int n, const int32_t* __restrict__ src,
                                                             const double* __restrict__ cif,
                                                             double* __restrict__ val) {
  const int e = int(blockIdx.x) * kBlock + int(threadIdx.x);
  if (e < n) val[e] = cif[src[e]];
}

int interface_blocks(const DevLevel& L) { return std::max(1, (L.n_if_rows + kBlock - 1) / kBlock); }

void launch_interface_values(hipStream_t s, int n_entries, const int32_t* src, const double* cif, double* val) {
  if (n_entries <= 0) return;
  hipLaunchKernelGGL(k_interface_values, dim3((n_entries + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n_entries,
                     src, cif, val);
}

void launch_interface(hipStream_t s, const DevLevel& L, const double* p, double* q, const PcgScalars* sc,
                      double* part_if) {
  hipLaunchKernelGGL(k_interface, dim3(interface_blocks(L)), dim3(kBlock), 0, s, L, p, q, sc, part_if);
}

void launch_check(hipStream_t s, const SweepPlan& P, int it_last, PcgScalars* sc, const double* part) {
  hipLaunchKernelGGL(k_check, dim3(P.n_prob), dim3(kBlock), 0, s, P, it_last, sc, part);
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

void launch_ir_sweep(hipStream_t s, const DevLevel& L, const SweepPlan& P, const FaceCoefs<double>& A, const double* diag,
                     const double* b, const double* x_old, const float* d, double* x_new, float* r32,
                     const PcgScalars* outer, double* part) {
  hipLaunchKernelGGL(k_ir_sweep, dim3(P.G), dim3(kBlock), 0, s, L, P, A, diag, b, x_old, d, x_new, r32, outer,
                     part);
}

void launch_ir_finish(hipStream_t s, const SweepPlan& P, int first, double inner_tol, int max_outer,
                      PcgScalars* outer, PcgScalars* inner, const double* part) {
  hipLaunchKernelGGL(k_ir_finish, dim3(P.n_prob), dim3(kBlock), 0, s, P, first, inner_tol, max_outer, outer,
                     inner, part);
}

void launch_inner_init(hipStream_t s, const DevLevel& L, const SweepPlan& P, const float* diag32,
                       const float* r32, float* d, float* p_clear, const PcgScalars* outer, double* part) {
  hipLaunchKernelGGL(k_inner_init, dim3(P.G), dim3(kBlock), 0, s, L, P, diag32, r32, d, p_clear, outer, part);
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

// Resident blocks of the persistent sweep on this device (0 if unknown).
template <typename T>
int resident_blocks(const SweepPlan& P, int per_cu_cap) {
  int dev = 0, cus = 0, per_cu = 0, coop = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(T);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_pcg_persistent<T>),
                                                   kBlock, lds) != hipSuccess)
    return 0;
  if (per_cu_cap > 0) per_cu = std::min(per_cu, per_cu_cap);
  return per_cu * cus;
}

template <typename T>
int persistent_blocks(const SweepPlan& P, int per_cu_cap) {
  const int res = resident_blocks<T>(P, per_cu_cap);
  return res > 0 ? std::min(P.G, res) : 0;
}

template int persistent_blocks<double>(const SweepPlan&, int);
template int persistent_blocks<float>(const SweepPlan&, int);

template <typename T>
hipError_t launch_pcg_persistent(hipStream_t s, const DevLevel& L, const SweepPlan& P, int max_iter,
                                 const FaceCoefs<T>& A,
                                 const T* diag, T* x, T* r, T* const* p, T* q, PcgScalars* sc, double* part,
                                 unsigned* bar, int per_cu_cap) {
  const int res = resident_blocks<T>(P, per_cu_cap);
  if (res <= 0) return hipErrorNotSupported;
  const int grid = std::min(P.G, res);
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(T);
  // bounded barrier wait: ~2^26 polls of ~0.1 us, far above the longest sweep
  unsigned spin_limit = 1u << 26;
  DevLevel Lv = L;
  SweepPlan Pv = P;
  T* p0 = p[0];
  T* p1 = p[1];
  FaceCoefs<T> Av = A;
  void* args[] = {&Lv, &Pv, &max_iter, &Av, (void*)&diag, &x, &r, &p0, &p1, &q, &sc, &part, &bar,
                  &spin_limit};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_pcg_persistent<T>), dim3(grid), dim3(kBlock),
                                    args, unsigned(lds), s);
}

int mixed_persistent_blocks(const SweepPlan& P, int per_cu_cap) {
  int dev = 0, cus = 0, per_cu = 0, coop = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(float);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_mixed_persistent),
                                                   kBlock, lds) != hipSuccess)
    return 0;
  if (per_cu_cap > 0) per_cu = std::min(per_cu, per_cu_cap);
  return std::min(P.G, per_cu * cus);
}

hipError_t launch_mixed_persistent(hipStream_t s, const DevLevel& L, const SweepPlan& P, const MixedArgs& M,
                                   int per_cu_cap) {
  const int grid = mixed_persistent_blocks(P, per_cu_cap);
  if (grid <= 0) return hipErrorNotSupported;
  const size_t lds = size_t(P.tpb_max) * kBlock * sizeof(float);
  DevLevel Lv = L;
  SweepPlan Pv = P;
  MixedArgs Mv = M;
  void* args[] = {&Lv, &Pv, &Mv};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_mixed_persistent), dim3(grid), dim3(kBlock),
                                    args, unsigned(lds), s);
}

template hipError_t launch_pcg_persistent<double>(hipStream_t, const DevLevel&, const SweepPlan&, int,
                                                  const FaceCoefs<double>&, const double*, double*, double*, double* const*,
                                                  double*, PcgScalars*, double*, unsigned*, int);
template hipError_t launch_pcg_persistent<float>(hipStream_t, const DevLevel&, const SweepPlan&, int,
                                                 const FaceCoefs<float>&, const float*, float*, float*, float* const*,
                                                 float*, PcgScalars*, double*, unsigned*, int);

template void launch_pcg_init<double>(hipStream_t, const DevLevel&, const SweepPlan&, const FaceCoefs<double>&,
                                      const double*, const double*, const double*, double*, double*,
                                      double*);
template void launch_pass_a<double>(hipStream_t, const DevLevel&, const SweepPlan&, int, const FaceCoefs<double>&,
                                    const double*, const double*, const double*, double*, double*,
                                    PcgScalars*, double*, hipEvent_t, hipEvent_t);
template void launch_pass_b<double>(hipStream_t, const DevLevel&, const SweepPlan&, int, const double*,
                                    const double*, const double*, double*, double*, PcgScalars*, double*,
                                    hipEvent_t, hipEvent_t);
template void launch_pass_a<float>(hipStream_t, const DevLevel&, const SweepPlan&, int, const FaceCoefs<float>&,
                                   const float*, const float*, const float*, float*, float*, PcgScalars*,
                                   double*, hipEvent_t, hipEvent_t);
template void launch_pass_b<float>(hipStream_t, const DevLevel&, const SweepPlan&, int, const float*,
                                   const float*, const float*, float*, float*, PcgScalars*, double*,
                                   hipEvent_t, hipEvent_t);

}  // namespace amrfld
