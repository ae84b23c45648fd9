// HIP kernels (gfx950) of the level solve: cell diffusivity, face coefficients
// and right-hand side, Jacobi-PCG sweeps with fused reductions, flux register,
// restriction.
//
// Layout: a level's cells are "slots", 8 per oct, octs in Morton order, x
// fastest inside an oct, so slot i lives in oct i >> 3 at position i & 7 and
// its in-oct face neighbour along axis a is slot i ^ (1 << a).  A 64-wide
// wavefront therefore holds 8 whole octs and in-oct neighbours are exchanged
// with cross-lane shuffles; the three faces of a cell that leave its oct go
// through the per-oct neighbour table.
//
// The operator is stored symmetric: Cp[a][i] is the coefficient of the face
// between slot i and its +a neighbour when both are leaves of this level and
// zero otherwise; the -a face of slot i is Cp[a] of the -a neighbour.  Refined
// slots carry an identity row (diag 1, all coefficients 0, r = 0), so the sweeps
// run over every slot without branching on the cell type.
#include "device.h"

#include <cfloat>

namespace amrfld {

int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

namespace {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int same_level_nb(const int32_t* __restrict__ nbr, int i, int dir) {
  const int pos = i & 7, axis = dir >> 1, side = dir & 1, bit = 1 << axis;
  if (((pos >> axis) & 1) != side) return i ^ bit;
  const int n = nbr[(i >> 3) * 6 + dir];
  return n < 0 ? -1 : ((n << 3) | (pos ^ bit));
}

__device__ __forceinline__ double harmonic(double a, double b) {
  const double s = a + b;
  return s != 0.0 ? (2.0 * a * b) / s : 0.0;
}

// Sums over the block (thread 0 gets the result).
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

// Writes this block's partials and reports whether it is the last block to
// arrive.  In the last block, on return, every thread sees all partials.
template <int NV>
__device__ __forceinline__ bool publish_partials(const double (&v)[NV], double* partials,
                                                 unsigned* counter) {
  __shared__ bool last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) partials[blockIdx.x * NV + k] = v[k];
    __threadfence();
    const unsigned t = atomicAdd(counter, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// Fixed-order reduction of all blocks' partials, run by the last block.
template <int NV>
__device__ __forceinline__ void reduce_partials(double (&v)[NV], const bool (&is_max)[NV],
                                                const double* partials, double* lds) {
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = is_max[k] ? -DBL_MAX : 0.0;
  for (int b = threadIdx.x; b < int(gridDim.x); b += kBlock) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double t = partials[b * NV + k];
      v[k] = is_max[k] ? fmax(v[k], t) : v[k] + t;
    }
  }
  block_reduce<NV>(v, is_max, lds);
}

// The 7-point operator applied at slot i to a vector whose values at other
// slots are produced by get(j).  pi is the value at slot i.
template <class Get>
__device__ __forceinline__ double apply_stencil(int i, int ii, const int32_t* __restrict__ nbr,
                                                const double* __restrict__ Cp, int n, double di,
                                                double pi, Get get) {
  const int pos = ii & 7, o = ii >> 3;
  double acc = di * pi;
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    const int bit = 1 << axis;
    const double* __restrict__ Ca = Cp + size_t(axis) * n;
    const double c_own = Ca[ii];
    const double p_sib = __shfl_xor(pi, bit, 64);
    const double c_sib = __shfl_xor(c_own, bit, 64);
    const int my = (pos >> axis) & 1;
    acc -= (my ? c_sib : c_own) * p_sib;
    const int nb = nbr[o * 6 + 2 * axis + my];
    if (nb >= 0) {
      const int j = (nb << 3) | (pos ^ bit);
      const double c_out = my ? c_own : Ca[j];
      if (c_out != 0.0) acc -= c_out * get(j);
    }
  }
  (void)i;
  return acc;
}

// ----------------------------------------------------------- setup kernels
__global__ __launch_bounds__(kBlock) void k_cell_K(DevLevel L, const double* __restrict__ E,
                                                   const double* __restrict__ rho,
                                                   const double* __restrict__ Ec, CellKParams kp,
                                                   double* __restrict__ K) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.n_slots) return;
  if (kp.kmode == 0) {
    K[i] = kp.K_const;
    return;
  }
  const double Ei = E[i];
  double g2 = 0.0;
#pragma unroll
  for (int axis = 0; axis < 3; ++axis) {
    double v[2], h[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int dir = 2 * axis + side;
      const int j = same_level_nb(L.nbr, i, dir);
      if (j >= 0) {
        v[side] = E[j];
        h[side] = L.dx;
      } else {
        const int c = L.cnb[(i >> 3) * 6 + dir];
        if (c >= 0) {
          v[side] = Ec[c];
          h[side] = 1.5 * L.dx;
        } else {
          v[side] = Ei;
          h[side] = L.dx;
        }
      }
    }
    const double g = (v[1] - v[0]) / (h[0] + h[1]);
    g2 += g * g;
  }
  const double rk = rho[i] * kp.kappa_R;
  const double R = sqrt(g2) / (rk * Ei);
  const double lam = (2.0 + R) / (6.0 + 3.0 * R + R * R);
  K[i] = kp.c_light * lam / rk;
}

__global__ __launch_bounds__(kBlock) void k_assemble(
    DevLevel L, const double* __restrict__ K, const double* __restrict__ Kc,
    const double* __restrict__ E, const double* __restrict__ Ec, const double* __restrict__ rho,
    const double* __restrict__ reg, double coef, double w, CouplingParams cp, double dt,
    double* __restrict__ Cp, double* __restrict__ diag, double* __restrict__ b) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int n = L.n_slots;
  if (i >= n) return;
  if (L.child[i] >= 0) {  // refined slot: identity row, r stays 0
    Cp[i] = 0.0;
    Cp[size_t(n) + i] = 0.0;
    Cp[2 * size_t(n) + i] = 0.0;
    diag[i] = 1.0;
    b[i] = E[i];
    return;
  }
  const double Ki = K[i];
  double d = 1.0, bb = E[i];
  double cplus[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int dir = 0; dir < 6; ++dir) {
    const int j = same_level_nb(L.nbr, i, dir);
    if (j >= 0) {
      const double C = harmonic(Ki, K[j]) * coef;
      if (L.child[j] >= 0) {  // coarse-to-fine face: D / N / R (Sect. 3.2)
        const double Fin = reg ? -reg[size_t(dir) * n + i] / L.vol : 0.0;
        d += w * C;
        bb += w * C * E[j] + (1.0 - w) * Fin;
      } else {
        d += C;
        if (dir & 1) cplus[dir >> 1] = C;
      }
    } else {
      const int c = L.cnb[(i >> 3) * 6 + dir];
      if (c >= 0) {  // fine-to-coarse face: Dirichlet, centre distance 3 dx / 2
        const double C = (2.0 / 3.0) * harmonic(Ki, Kc[c]) * coef;
        d += C;
        bb += C * Ec[c];
      }
    }
  }
  if (cp.T) {  // linearised coupling term kappa_P rho c (a T^4 - E)
    const double T = cp.T[i], r = rho[i];
    const double eta = cp.kappa_P * r * cp.c_light * dt;
    const double bT = 4.0 * cp.a_rad * T * T * T;
    const double den = r * cp.c_v + eta * bT;
    const double f = eta * bT / den;
    d += eta * (1.0 - f);
    bb += eta * (1.0 - f) * cp.a_rad * (T * T * T * T);
  }
  Cp[i] = cplus[0];
  Cp[size_t(n) + i] = cplus[1];
  Cp[2 * size_t(n) + i] = cplus[2];
  diag[i] = d;
  b[i] = bb;
}

// -------------------------------------------------------------- PCG sweeps
// r0 = b - A x0, z0 = r0 / d; partial sums of (r, z), ||r||^2, ||b||^2.
__global__ __launch_bounds__(kBlock) void k_pcg_init(DevLevel L, const double* __restrict__ Cp,
                                                     const double* __restrict__ diag,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ r,
                                                     double* __restrict__ p_clear,
                                                     PcgScalars* sc, double* partials) {
  __shared__ double lds[(kBlock / 64) * 3];
  const int n = L.n_slots;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  const double xi = x[ii], di = diag[ii];
  const double ax = apply_stencil(i, ii, L.nbr, Cp, n, di, xi, [&](int j) { return x[j]; });
  double v[3] = {0.0, 0.0, 0.0};
  if (valid) {
    const double ri = b[i] - ax;
    r[i] = ri;
    p_clear[i] = 0.0;
    const double z = ri / di;
    const double bi = b[i];
    v[0] = ri * z;
    v[1] = ri * ri;
    v[2] = bi * bi;
  }
  const bool is_max[3] = {false, false, false};
  block_reduce<3>(v, is_max, lds);
  if (!publish_partials<3>(v, partials, &sc->cnt[0])) return;
  reduce_partials<3>(v, is_max, partials, lds);
  if (threadIdx.x == 0) {
    const double r0 = sqrt(v[1]), bn = sqrt(v[2]);
    sc->rho = v[0];
    sc->rnorm0 = r0;
    sc->rnorm = r0;
    sc->bnorm = bn;
    const double floor_b = sc->abs_floor * bn;
    sc->thresh = fmax(sc->tol * r0, floor_b);
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->iter = 0;
    sc->linf = 0.0;
    const bool fin = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
    sc->nonfinite = fin ? 0 : 1;
    // already converged: ||r_0|| <= abs_floor ||b|| returns x_0 after 0 iterations
    sc->converged = (fin && r0 <= floor_b) ? 1 : 0;
    sc->done = (!fin || r0 <= floor_b) ? 1 : 0;
    sc->cnt[0] = 0;
  }
}

// Pass A of iteration j: p_j = z_j + beta p_{j-1} (z = r / d formed on the fly;
// p_1 = z_0), q = A p_j, partial (p_j, q).  Neighbour values of p_j outside the
// oct are recomputed from r, d and p_{j-1} (the two p buffers alternate).
__global__ __launch_bounds__(kBlock) void k_pass_a(DevLevel L, const double* __restrict__ Cp,
                                                   const double* __restrict__ diag,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ p_old,
                                                   double* __restrict__ p_new,
                                                   double* __restrict__ q, PcgScalars* sc,
                                                   double* partials) {
  if (sc->done) return;
  __shared__ double lds[kBlock / 64];
  const bool first = sc->iter == 0;
  const double beta = sc->beta;
  const int n = L.n_slots;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  auto pval = [&](int j) {
    const double z = r[j] / diag[j];
    return first ? z : fma(beta, p_old[j], z);
  };
  const double di = diag[ii];
  const double pi = pval(ii);
  const double qi = apply_stencil(i, ii, L.nbr, Cp, n, di, pi, pval);
  double v[1] = {0.0};
  if (valid) {
    p_new[i] = pi;
    q[i] = qi;
    v[0] = pi * qi;
  }
  const bool is_max[1] = {false};
  block_reduce<1>(v, is_max, lds);
  if (!publish_partials<1>(v, partials, &sc->cnt[1])) return;
  reduce_partials<1>(v, is_max, partials, lds);
  if (threadIdx.x == 0) {
    const double pq = v[0];
    sc->alpha = sc->rho / pq;
    if (!isfinite(sc->alpha)) {
      sc->nonfinite = 1;
      sc->done = 1;
    }
    sc->cnt[1] = 0;
  }
}

// Pass B: x += alpha p, r -= alpha q; partial (r, z), ||r||^2 and the largest
// relative change |alpha p| / |x|; the last block applies the stopping test.
__global__ __launch_bounds__(kBlock) void k_pass_b(DevLevel L, const double* __restrict__ diag,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ q,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   PcgScalars* sc, double* partials) {
  if (sc->done) return;
  __shared__ double lds[(kBlock / 64) * 3];
  const double alpha = sc->alpha;
  const int n = L.n_slots;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double v[3] = {0.0, 0.0, 0.0};
  if (i < n) {
    const double xi = x[i];
    const double dx = alpha * p[i];
    const double ax = fabs(xi);
    v[2] = ax > 0.0 ? fabs(dx) / ax : fabs(dx);
    x[i] = xi + dx;
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    const double z = ri / diag[i];
    v[0] = ri * z;
    v[1] = ri * ri;
  }
  const bool is_max[3] = {false, false, true};
  block_reduce<3>(v, is_max, lds);
  if (!publish_partials<3>(v, partials, &sc->cnt[2])) return;
  reduce_partials<3>(v, is_max, partials, lds);
  if (threadIdx.x == 0) {
    const double rn = sqrt(v[1]);
    const int it = sc->iter + 1;
    sc->iter = it;
    sc->rnorm = rn;
    sc->linf = v[2];
    const bool conv = (rn <= sc->thresh && (!sc->linf_test || v[2] < sc->tol)) || rn == 0.0;
    if (!isfinite(rn) || !isfinite(v[0])) {
      sc->nonfinite = 1;
      sc->done = 1;
    } else if (conv) {
      sc->converged = 1;
      sc->done = 1;
    } else if (it >= sc->max_iter) {
      sc->done = 1;
    } else {
      sc->beta = v[0] / sc->rho;
      sc->rho = v[0];
    }
    sc->cnt[2] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_true_residual(DevLevel L, const double* __restrict__ Cp,
                                                          const double* __restrict__ diag,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ x,
                                                          PcgScalars* sc, double* partials) {
  __shared__ double lds[kBlock / 64];
  const int n = L.n_slots;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  const double ax = apply_stencil(i, ii, L.nbr, Cp, n, diag[ii], x[ii], [&](int j) { return x[j]; });
  double v[1] = {0.0};
  if (valid) {
    const double ri = b[i] - ax;
    v[0] = ri * ri;
  }
  const bool is_max[1] = {false};
  block_reduce<1>(v, is_max, lds);
  if (!publish_partials<1>(v, partials, &sc->cnt[3])) return;
  reduce_partials<1>(v, is_max, partials, lds);
  if (threadIdx.x == 0) {
    sc->true_rnorm = sqrt(v[0]);
    sc->cnt[3] = 0;
  }
}

// T update of the coupling term and smallest leaf energy.
__global__ __launch_bounds__(kBlock) void k_post_solve(DevLevel L, const double* __restrict__ E,
                                                       const double* __restrict__ rho,
                                                       CouplingParams cp, double dt,
                                                       double* __restrict__ T_out, PcgScalars* sc,
                                                       double* partials) {
  __shared__ double lds[kBlock / 64];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double v[1] = {-DBL_MAX};
  if (i < L.n_slots && L.child[i] < 0) {
    const double e = E[i];
    v[0] = -e;
    if (cp.T) {
      const double T = cp.T[i], r = rho[i];
      const double eta = cp.kappa_P * r * cp.c_light * dt;
      const double bT = 4.0 * cp.a_rad * T * T * T;
      const double den = r * cp.c_v + eta * bT;
      T_out[i] = T + eta * (e - cp.a_rad * (T * T * T * T)) / den;
    }
  }
  const bool is_max[1] = {true};
  block_reduce<1>(v, is_max, lds);
  if (!publish_partials<1>(v, partials, &sc->cnt[3])) return;
  reduce_partials<1>(v, is_max, partials, lds);
  if (threadIdx.x == 0) {
    sc->min_E = -v[0];
    sc->cnt[3] = 0;
  }
}

// One thread per (fine oct, direction): the four cells of that oct face that
// see a coarser leaf add their energy gain V C (E_c - E_i) (eq. mean_flux with
// dt inside C) to the register of that coarse cell, on its face looking back.
__global__ __launch_bounds__(kBlock) void k_flux_register(DevLevel F, const double* __restrict__ Kf,
                                                          const double* __restrict__ Kc,
                                                          const double* __restrict__ Ef,
                                                          const double* __restrict__ Ec,
                                                          double coef, double* __restrict__ reg_c,
                                                          int n_slots_c) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= F.n_oct * 6) return;
  const int o = t / 6, dir = t % 6;
  if (F.nbr[o * 6 + dir] >= 0) return;
  const int c = F.cnb[o * 6 + dir];
  if (c < 0) return;
  const int axis = dir >> 1, side = dir & 1;
  double sum = 0.0;
  for (int pos = 0; pos < 8; ++pos) {
    if (((pos >> axis) & 1) != side) continue;
    const int i = (o << 3) | pos;
    if (F.child[i] >= 0) continue;
    const double C = (2.0 / 3.0) * harmonic(Kf[i], Kc[c]) * coef;
    sum += F.vol * C * (Ec[c] - Ef[i]);
  }
  const size_t k = size_t(dir ^ 1) * n_slots_c + c;
  reg_c[k] += sum;
}

__global__ __launch_bounds__(kBlock) void k_restrict(DevLevel F, const double* __restrict__ Ef,
                                                     double* __restrict__ Ec) {
  const int o = blockIdx.x * kBlock + threadIdx.x;
  if (o >= F.n_oct) return;
  const double* e = Ef + size_t(o) * 8;
  const double s = ((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]));
  Ec[F.parent[o]] = s * 0.125;
}

__global__ __launch_bounds__(kBlock) void k_fill(double* p, int64_t n, double v) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

// ------------------------------------------------------------ launchers
void launch_cell_K(hipStream_t s, const DevLevel& L, const double* E, const double* rho,
                   const double* E_coarse, const CellKParams& kp, double* K) {
  hipLaunchKernelGGL(k_cell_K, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, E, rho, E_coarse,
                     kp, K);
}

void launch_assemble(hipStream_t s, const DevLevel& L, const double* K, const double* K_coarse,
                     const double* E, const double* E_coarse, const double* rho, const double* reg,
                     double dt, double w, const CouplingParams& cp, double* Cp, double* diag,
                     double* b) {
  const double coef = dt / (L.dx * L.dx);
  hipLaunchKernelGGL(k_assemble, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, K, K_coarse, E,
                     E_coarse, rho, reg, coef, w, cp, dt, Cp, diag, b);
}

void launch_pcg_init(hipStream_t s, const DevLevel& L, const double* Cp, const double* diag,
                     const double* b, const double* x, double* r, double* p_clear,
                     PcgScalars* sc, double* partials) {
  hipLaunchKernelGGL(k_pcg_init, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, Cp, diag, b, x, r,
                     p_clear, sc, partials);
}

void launch_pass_a(hipStream_t s, const DevLevel& L, const double* Cp, const double* diag,
                   const double* r, const double* p_old, double* p_new, double* q, PcgScalars* sc,
                   double* partials) {
  hipLaunchKernelGGL(k_pass_a, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, Cp, diag, r, p_old,
                     p_new, q, sc, partials);
}

void launch_pass_b(hipStream_t s, const DevLevel& L, const double* diag, const double* p,
                   const double* q, double* x, double* r, PcgScalars* sc, double* partials) {
  hipLaunchKernelGGL(k_pass_b, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, diag, p, q, x, r,
                     sc, partials);
}

void launch_true_residual(hipStream_t s, const DevLevel& L, const double* Cp, const double* diag,
                          const double* b, const double* x, PcgScalars* sc, double* partials) {
  hipLaunchKernelGGL(k_true_residual, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, Cp, diag, b,
                     x, sc, partials);
}

void launch_post_solve(hipStream_t s, const DevLevel& L, const double* E, const double* rho,
                       const CouplingParams& cp, double dt, double* T_out, PcgScalars* sc,
                       double* partials) {
  hipLaunchKernelGGL(k_post_solve, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, E, rho, cp, dt,
                     T_out, sc, partials);
}

void launch_flux_register(hipStream_t s, const DevLevel& F, const double* K_f, const double* K_c,
                          const double* E_f, const double* E_c, double dt, double* reg_c,
                          int n_slots_c) {
  const double coef = dt / (F.dx * F.dx);
  hipLaunchKernelGGL(k_flux_register, dim3(grid_for(int64_t(F.n_oct) * 6)), dim3(kBlock), 0, s, F,
                     K_f, K_c, E_f, E_c, coef, reg_c, n_slots_c);
}

void launch_restrict(hipStream_t s, const DevLevel& F, const double* E_f, double* E_c) {
  hipLaunchKernelGGL(k_restrict, dim3(grid_for(F.n_oct)), dim3(kBlock), 0, s, F, E_f, E_c);
}

void launch_fill(hipStream_t s, double* p, int64_t n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
}

}  // namespace amrfld
