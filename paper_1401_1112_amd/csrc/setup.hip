// Setup kernels of a level solve (once per solve): cell diffusivity, face
// coefficients with the interface rows, right-hand side; and the level-coupling
// kernels: flux register and restriction.
#include "common.h"

namespace amrfld {

int grid_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

namespace {

using dev::harmonic;
using dev::same_level_nb;

// Diffusivity of an energy held at a box face: the cell law at that value with no
// gradient there (flux limiter at R = 0, 1/3 for both limiters).
__device__ inline double held_K(int kmode, double K_const, double K_exp, double kappa_R, double c_light,
                                double rho, double v) {
  if (kmode == 0) return K_const;
  if (kmode == 3) return K_const * pow(v, K_exp);
  return c_light / (3.0 * rho * kappa_R);
}

// ----------------------------------------------------------- setup kernels
__global__ __launch_bounds__(kBlock) void k_cell_K(DevLevel L, const double* __restrict__ E,
                                                   const double* __restrict__ rho,
                                                   const double* __restrict__ Ec, CellKParams kp,
                                                   OuterBC ob, double* __restrict__ K) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.n_slots) return;
  if (L.child[i] == -2) {  // padding slot of a batch
    K[i] = 0.0;
    return;
  }
  const PatchParams* pp = L.pp ? &L.pp[L.oct_prob[i >> 3]] : nullptr;
  const int kmode = pp ? pp->kmode : kp.kmode;
  if (kmode == 0) {
    K[i] = pp ? pp->K_const : kp.K_const;
    return;
  }
  if (kmode == 3) {  // power law (nonlinear equilibrium test, Sect. 4.2); levels only
    K[i] = kp.K_const * pow(E[i], kp.K_exp);
    return;
  }
  const double dx = pp ? pp->dx : L.dx;
  const double kappa_R = pp ? pp->kappa_R : kp.kappa_R;
  const double c_light = pp ? pp->c_light : kp.c_light;
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
        h[side] = dx;
      } else {
        const int c = L.cnb[(i >> 3) * 6 + dir];
        if (c >= 0) {
          v[side] = Ec[c];
          h[side] = 1.5 * dx;
        } else if (!pp && ((ob.mask >> dir) & 1u)) {  // value held at the box face
          v[side] = ob.val[dir];
          h[side] = 0.5 * dx;
        } else {
          v[side] = Ei;
          h[side] = dx;
        }
      }
    }
    const double g = (v[1] - v[0]) / (h[0] + h[1]);
    g2 += g * g;
  }
  const double rk = rho[i] * kappa_R;
  const double R = sqrt(g2) / (rk * Ei);
  double lam;
  if (kmode == 2) {  // Minerbo limiter
    lam = R <= 1.5 ? 2.0 / (3.0 + sqrt(9.0 + 12.0 * R * R)) : 1.0 / (1.0 + R + sqrt(1.0 + 2.0 * R));
  } else {  // Levermore-Pomraning limiter
    lam = (2.0 + R) / (6.0 + 3.0 * R + R * R);
  }
  K[i] = c_light * lam / rk;
}

// Theta-weighted step from the backward-Euler system (A1, b1): the right-hand side
// loses (1 - theta) (A1 - I) E^n (same-level fluxes at the old time; the ghost
// values are the same at both times), then ...
__global__ __launch_bounds__(kBlock) void k_theta_rhs(DevLevel L, FaceCoefs<double> A1,
                                                      const double* __restrict__ diag,
                                                      const double* __restrict__ E, double theta,
                                                      double* __restrict__ b) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  // every lane of a wave takes part in the operator's shuffles
  const int ii = i < L.n_slots ? i : L.n_slots - 1;
  const double ax = dev::apply_stencil<double>(ii, L.nbr, A1, A1.scale, L.n_slots, diag[ii], E[ii],
                                               [&](int j) { return E[j]; });
  if (i >= L.n_slots || L.child[i] != -1) return;
  b[i] -= (1.0 - theta) * (ax - E[i]);
}

// ... the matrix becomes I + theta (A1 - I) (identity rows stay identity rows).
__global__ __launch_bounds__(kBlock) void k_theta_scale(int n, double theta, double* __restrict__ Cp,
                                                        double* __restrict__ diag) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) Cp[size_t(a) * n + i] *= theta;
  diag[i] = 1.0 + theta * (diag[i] - 1.0);
}

__global__ __launch_bounds__(kBlock) void k_assemble(
    DevLevel L, const double* __restrict__ K, const double* __restrict__ Kc,
    const double* __restrict__ E, const double* __restrict__ Ec, const double* __restrict__ rho,
    const double* __restrict__ reg, double coef, double w, double alpha, CouplingParams cp, CellKParams kp,
    OuterBC ob, double dt, double* __restrict__ Cp, uint8_t* __restrict__ mask, double* __restrict__ diag,
    double* __restrict__ b) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int n = L.n_slots;
  if (i >= n) return;
  if (L.child[i] != -1) {  // refined or padding slot: identity row, r stays 0
    Cp[i] = 0.0;
    Cp[size_t(n) + i] = 0.0;
    Cp[2 * size_t(n) + i] = 0.0;
    mask[i] = 0;
    diag[i] = 1.0;
    b[i] = E[i];
    return;
  }
  const PatchParams* pp = L.pp ? &L.pp[L.oct_prob[i >> 3]] : nullptr;
  if (pp) coef = pp->coef;
  const double Ki = K[i];
  double d = 1.0, bb = E[i];
  double cplus[3] = {0.0, 0.0, 0.0};
  unsigned m = 0;
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
        m |= 1u << dir;
        if (dir & 1) cplus[dir >> 1] = C;
      }
    } else {
      const int c = L.cnb[(i >> 3) * 6 + dir];
      if (c >= 0) {  // fine-to-coarse face: Dirichlet, centre distance 3 dx / 2
        const double C = (2.0 / 3.0) * harmonic(Ki, Kc[c]) * coef;
        d += C;
        bb += C * Ec[c];
      } else if (pp) {  // patch boundary: D / N / R with a given ghost and inflow
        const int m = pp->mode[dir];
        const double wf = m == 0 ? 1.0 : m == 1 ? 0.0 : alpha;
        const double C = Ki * coef;  // ghost cell with the cell's own diffusivity
        d += wf * C;
        bb += wf * C * pp->ghost[dir] + (1.0 - wf) * pp->flux[dir];
      } else if ((ob.mask >> dir) & 1u) {  // Dirichlet value held at the box face, dx / 2 away
        const double v = ob.val[dir];
        const double C = 2.0 * harmonic(Ki, held_K(kp.kmode, kp.K_const, kp.K_exp, kp.kappa_R, kp.c_light,
                                                   rho[i], v)) * coef;
        d += C;
        bb += C * v;
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
  mask[i] = uint8_t(m);
  diag[i] = d;
  b[i] = bb;
}

// Composite system (unique time step): rows of every level's leaves multiplied by
// the cell volume.  Same-level faces C = A = K_f dt / dx^2; a face towards a coarser
// leaf C = (2/3) A; a face shared with a refined same-level neighbour couples to its
// four finer cells, each with 2^(3-ndim) A / 3 = A / 3 (K_f with that finer cell).
// The coefficient of a fine-to-coarse pair is stored once, at the finer cell
// (V_f (2/3) A_f, equal to V_c A_c / 3), and read by both rows.
__global__ __launch_bounds__(kBlock) void k_assemble_composite(
    DevLevel L, const double* __restrict__ K, const double* __restrict__ E, const double* __restrict__ rho,
    CouplingParams cp, OuterBC ob, double dt, double* __restrict__ Cp, double* __restrict__ cif,
    uint8_t* __restrict__ c2f, double* __restrict__ diag, double* __restrict__ b) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int n = L.n_slots;
  if (i >= n) return;
  if (L.child[i] != -1) {  // refined or padding slot: identity row, r stays 0
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Cp[size_t(a) * n + i] = 0.0;
      cif[size_t(a) * n + i] = 0.0;
    }
    c2f[i] = 0;
    diag[i] = 1.0;
    b[i] = E[i];
    return;
  }
  const PatchParams& P = L.pp[L.oct_prob[i >> 3]];
  const double coef = P.coef, V = P.vol, Ki = K[i];
  double d = 1.0, bb = E[i];
  double cplus[3] = {0.0, 0.0, 0.0}, cf[3] = {0.0, 0.0, 0.0};
  unsigned mask = 0;
  for (int dir = 0; dir < 6; ++dir) {
    const int a = dir >> 1, side = dir & 1;
    const int j = same_level_nb(L.nbr, i, dir);
    if (j >= 0) {
      const int co = L.child[j];
      if (co >= 0) {  // refined neighbour: its four finer cells on the shared face
        mask |= 1u << dir;
        const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
        const int fb = side ? 0 : 1;
        for (int k = 0; k < 4; ++k) {
          const int f = (co << 3) | (fb << a) | ((k & 1) << t0) | ((k >> 1) << t1);
          d += harmonic(Ki, K[f]) * coef / 3.0;
        }
      } else {
        const double C = harmonic(Ki, K[j]) * coef;
        d += C;
        if (side) cplus[a] = V * C;
      }
    } else {
      const int c = L.cnb[(i >> 3) * 6 + dir];
      if (c >= 0) {  // coarser leaf, centre distance 3 dx / 2
        const double C = (2.0 / 3.0) * harmonic(Ki, K[c]) * coef;
        d += C;
        cf[a] = V * C;
      } else if ((ob.mask >> dir) & 1u) {  // Dirichlet value held at the box face, dx / 2 away
        const double v = ob.val[dir];
        const double C = 2.0 * harmonic(Ki, held_K(P.kmode, P.K_const, P.K_exp, P.kappa_R, P.c_light, rho[i], v)) *
                         coef;
        d += C;
        bb += C * v;
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
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Cp[size_t(a) * n + i] = cplus[a];
    cif[size_t(a) * n + i] = cf[a];
  }
  c2f[i] = uint8_t(mask);
  diag[i] = V * d;
  b[i] = V * bb;
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

// Two doubles per thread, consecutive threads on consecutive pairs.
__global__ __launch_bounds__(kBlock) void k_copy_f64(double* __restrict__ dst, const double* __restrict__ src,
                                                     int64_t n) {
  const int64_t i = 2 * (int64_t(blockIdx.x) * kBlock + threadIdx.x);
  if (i + 1 < n) {
    const double a = src[i], b = src[i + 1];
    dst[i] = a;
    dst[i + 1] = b;
  } else if (i < n) {
    dst[i] = src[i];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* p, int64_t n, T v) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// FP32 copies of the operator for the inner solve of the mixed-precision form.
// Jacobi scaling of an assembled operator (Sect. 3.3.4's diagonal preconditioner as
// a symmetric scaling): rs = 1 / sqrt(diag) and Ch[a][i] = Cp[a][i] rs_i rs_j for the
// +a neighbour j, computed with the expression the sweeps use for formed
// coefficients, so both forms give the same bits.  Identity rows: diag 1, Ch 0.
__global__ __launch_bounds__(kBlock) void k_jacobi_scale(DevLevel L, const double* __restrict__ Cp,
                                                         const double* __restrict__ diag, double* __restrict__ rs,
                                                         double* __restrict__ Ch) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int n = L.n_slots;
  if (i >= n) return;
  const double rsi = 1.0 / sqrt(diag[i]);
  rs[i] = rsi;
  if (!Cp) return;
  const int pos = i & 7, o = i >> 3;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double c = Cp[size_t(a) * n + i];
    double ch = 0.0;
    if (c != 0.0) {
      const int bit = 1 << a;
      int j = -1;
      if (((pos >> a) & 1) == 0) {
        j = i ^ bit;
      } else {
        const int nb = L.nbr[o * 6 + 2 * a + 1];
        if (nb >= 0) j = (nb << 3) | (pos ^ bit);
      }
      if (j >= 0) ch = c * (rsi * (1.0 / sqrt(diag[j])));
    }
    Ch[size_t(a) * n + i] = ch;
  }
}

__global__ __launch_bounds__(kBlock) void k_to_f32(int64_t n, const double* __restrict__ Ch,
                                                   const double* __restrict__ K,
                                                   const double* __restrict__ rs,
                                                   float* __restrict__ Ch32, float* __restrict__ K32,
                                                   float* __restrict__ rs32) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  if (Ch) {
    Ch32[i] = float(Ch[i]);
    Ch32[n + i] = float(Ch[n + i]);
    Ch32[2 * n + i] = float(Ch[2 * n + i]);
  }
  if (K) K32[i] = float(K[i]);
  rs32[i] = float(rs[i]);
}

__global__ __launch_bounds__(kBlock) void k_batch_gather(DevLevel L, const int32_t* __restrict__ idx,
                                                         const double* const* __restrict__ src, double pad,
                                                         double* __restrict__ dst) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.n_slots) return;
  const int k = idx[i];
  dst[i] = k >= 0 ? src[L.oct_prob[i >> 3]][k] : pad;
}

__global__ __launch_bounds__(kBlock) void k_batch_scatter(DevLevel L, const int32_t* __restrict__ idx,
                                                          const int64_t* __restrict__ out_off,
                                                          const double* __restrict__ src, double* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.n_slots) return;
  const int k = idx[i];
  if (k >= 0) out[out_off[L.oct_prob[i >> 3]] + k] = src[i];
}

}  // namespace

void launch_batch_gather(hipStream_t s, const DevLevel& L, const int32_t* idx, const double* const* src,
                         double pad, double* dst) {
  hipLaunchKernelGGL(k_batch_gather, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, idx, src, pad, dst);
}

void launch_batch_scatter(hipStream_t s, const DevLevel& L, const int32_t* idx, const int64_t* out_off,
                          const double* src, double* out) {
  hipLaunchKernelGGL(k_batch_scatter, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, idx, out_off, src, out);
}

void launch_cell_K(hipStream_t s, const DevLevel& L, const double* E, const double* rho,
                   const double* E_coarse, const CellKParams& kp, const OuterBC& ob, double* K) {
  hipLaunchKernelGGL(k_cell_K, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, E, rho, E_coarse,
                     kp, ob, K);
}

void launch_assemble(hipStream_t s, const DevLevel& L, const double* K, const double* K_coarse,
                     const double* E, const double* E_coarse, const double* rho, const double* reg,
                     double dt, double w, double alpha, const CouplingParams& cp, const CellKParams& kp,
                     const OuterBC& ob, double* Cp, uint8_t* mask, double* diag, double* b) {
  const double coef = dt / (L.dx * L.dx);
  hipLaunchKernelGGL(k_assemble, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, K, K_coarse, E,
                     E_coarse, rho, reg, coef, w, alpha, cp, kp, ob, dt, Cp, mask, diag, b);
}

void launch_assemble_composite(hipStream_t s, const DevLevel& C, const double* K, const double* E,
                               const double* rho, const CouplingParams& cp, const OuterBC& ob, double dt,
                               double* Cp, double* cif, uint8_t* c2f, double* diag, double* b) {
  hipLaunchKernelGGL(k_assemble_composite, dim3(grid_for(C.n_slots)), dim3(kBlock), 0, s, C, K, E, rho, cp, ob, dt,
                     Cp, cif, c2f, diag, b);
}

void launch_theta_step(hipStream_t s, const DevLevel& L, double theta, const double* E,
                       const FaceCoefs<double>& A1, double* Cp, double* diag, double* b) {
  hipLaunchKernelGGL(k_theta_rhs, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, A1, diag, E, theta, b);
  hipLaunchKernelGGL(k_theta_scale, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L.n_slots, theta, Cp, diag);
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

void launch_copy_f64(hipStream_t s, double* dst, const double* src, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy_f64, dim3(int((n + 2 * kBlock - 1) / (2 * kBlock))), dim3(kBlock), 0, s, dst, src, n);
}

void launch_fill(hipStream_t s, double* p, int64_t n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
}

void launch_fill_f32(hipStream_t s, float* p, int64_t n, float v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
}

void launch_jacobi_scale(hipStream_t s, const DevLevel& L, const double* Cp, const double* diag, double* rs,
                         double* Ch) {
  hipLaunchKernelGGL(k_jacobi_scale, dim3(grid_for(L.n_slots)), dim3(kBlock), 0, s, L, Cp, diag, rs, Ch);
}

void launch_to_f32(hipStream_t s, int64_t n, const double* Ch, const double* K, const double* rs, float* Ch32,
                   float* K32, float* rs32) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(kBlock), 0, s, n, Ch, K, rs, Ch32, K32, rs32);
}

}  // namespace amrfld
