// Discrete adjoint kernels (gradient of the salt-mass QoI with respect to theta).
//
// Each converged implicit-Euler step satisfies R^n(u^n, u^{n-1}; phi, K, u_in) = 0 and
// Q = Q(u^r).  With the Lagrangian Q + sum_n lam_n^T R^n (implicit-function theorem on
// the converged steps):
//   J_r^T lam_r = -dQ/du^r,    J_n^T lam_n = -(dR^{n+1}/du^n)^T lam_{n+1},
//   dQ/dtheta = sum_n lam_n^T dR^n/dtheta.
// R^{n+1} depends on u^n only through the storage terms in c^n (a diagonal coupling).
#pragma once

#include "henry_kernels.hpp"

namespace henry {

// rhs for the last step: -dQ/du, Q = sum_{x > Lx/2} c rho(c) V
__global__ void k_adj_rhs_final(Map m, Grid2 G, Phys P, const double* __restrict__ c, double* __restrict__ rhs) {
  int s, cell, sb, cb;
  if (!map_cell(m, G.ncell, s, cell, sb, cb)) return;
  const size_t N = (size_t)G.ncell * m.S, id = (size_t)cell * m.S + s;
  const int j = cell / G.nx, i = cell - j * G.nx;
  const double cP = c[id];
  rhs[id] = 0.0;
  rhs[N + id] = ((i + 0.5) * P.hx > P.qoi_xmin) ? -(P.rho0 + 2.0 * P.drho * cP) * P.vol : 0.0;
}

// rhs for step n-1: -(dR^n/dc^{n-1})^T lam_n, with dR^p/dc_old = -V phi drho / tau and
// dR^c/dc_old = -V phi (rho0 + 2 drho c_old) / tau
__global__ void k_adj_rhs_prev(Map m, Grid2 G, Phys P, const double* __restrict__ c_old,
                               const double* __restrict__ phi, const double* __restrict__ lam,
                               double* __restrict__ rhs) {
  int s, cell, sb, cb;
  if (!map_cell(m, G.ncell, s, cell, sb, cb)) return;
  const size_t N = (size_t)G.ncell * m.S, id = (size_t)cell * m.S + s;
  const double co = c_old[id], ph = phi[id];
  rhs[id] = 0.0;
  rhs[N + id] = (lam[id] * P.vol * ph * P.drho + lam[N + id] * P.vol * ph * (P.rho0 + 2.0 * P.drho * co)) / P.tau;
}

// Accumulate g_phi += lam^T dR/dphi, g_K += lam^T dR/dK for one step (gathered per cell),
// and per-sample partials of lam^T dR/du_in for the base inflow u_in, which enters the
// step as u_in * uin_fac (the recharge time factor at the end of the step).
__global__ void __launch_bounds__(256) k_adj_param(Map m, Grid2 G, Phys P, const double* __restrict__ p,
                                                   const double* __restrict__ c, const double* __restrict__ c_old,
                                                   const double* __restrict__ phi, const double* __restrict__ K,
                                                   const double* __restrict__ lam, double* __restrict__ gphi,
                                                   double* __restrict__ gK, double* __restrict__ part) {
  __shared__ double lds[256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  const int S = m.S;
  const size_t N = (size_t)G.ncell * S;
  double acc[1] = {0.0};
  for (int kk = 0; kk < m.CPT; ++kk) {
    const int cell = (cblk * m.CPT + kk) * m.CY + threadIdx.y;
    if (!sv || cell >= G.ncell) continue;
    const int j = cell / G.nx, i = cell - j * G.nx;
    const size_t id = (size_t)cell * S + s;
    const double pP = p[id], cP = c[id], phP = phi[id], KP = K[id], co = c_old[id];
    const double lp = lam[id], lc = lam[N + id];
    const double rP = P.rho0 + P.drho * cP, ro = P.rho0 + P.drho * co;
    double gph = (lp * P.vol * (rP - ro) + lc * P.vol * (rP * cP - ro * co)) / P.tau;
    double gk = 0.0;
    // interior faces: (L, H) canonical; P is L for east/north, H for west/south
    auto face = [&](bool north, size_t q, bool P_is_L) {
      const size_t iL = P_is_L ? id : q, iH = P_is_L ? q : id;
      const double pL = p[iL], pH = p[iH], cL = c[iL], cH = c[iH];
      const double KL = K[iL], KH = K[iH];
      const double d = north ? P.hy : P.hx, A = north ? P.hx : P.hy, w = A / d;
      const double Kf = 2.0 * KL * KH / (KL + KH);
      const double rf = 0.5 * ((P.rho0 + P.drho * cL) + (P.rho0 + P.drho * cH));
      const double grad = (pH - pL) / d + (north ? rf * P.g : 0.0);
      const double F = -(Kf / P.mu) * grad * rf * A;
      const double cup = F >= 0.0 ? cL : cH;
      const double dF_dKf = -(rf * A / P.mu) * grad;
      const double lpd = lam[iL] - lam[iH], lcd = lam[N + iL] - lam[N + iH];
      gph += lcd * (-0.5 * rf * P.Dm * (cH - cL) * w);
      const double KQ = P_is_L ? KH : KL;
      const double dKf_dKP = 2.0 * KQ * KQ / ((KL + KH) * (KL + KH));
      gk += (lpd * dF_dKf + lcd * cup * dF_dKf) * dKf_dKP;
      (void)F;
    };
    if (i > 0) face(false, id - S, false);
    if (i < G.nx - 1) face(false, id + S, true);
    if (j > 0) face(true, id - (size_t)G.nx * S, false);
    if (j < G.ny - 1) face(true, id + (size_t)G.nx * S, true);
    const double wb = P.hy / P.hx;
    if (i == 0) {
      gph += lc * 2.0 * rP * P.Dm * (cP - P.c_left) * wb;
      const double dF_duin = -(P.rho0 + P.drho * P.c_left) * P.uin_fac * P.hy;
      acc[0] += lp * dF_duin + lc * dF_duin * P.c_left;
    }
    if (i == G.nx - 1) {
      const double y = -P.Ly + (j + 0.5) * P.hy;
      const double u = -(KP / P.mu) * (-P.rho1 * P.g * y - pP) / (0.5 * P.hx);
      const bool inflow = u < 0.0;
      const double F = (inflow ? P.rho1 : rP) * u * P.hy;
      const double Gadv = F * (inflow ? 1.0 : cP);
      gk += (lp * F + lc * Gadv) / KP;
      if (P.right_dir) gph += lc * 2.0 * rP * P.Dm * (cP - 1.0) * wb;
    }
    gphi[id] += gph;
    gK[id] += gk;
  }
  block_sum_y<1>(acc, lds);
  if (threadIdx.y == 0 && sv) part[(size_t)cblk * S + s] = acc[0];
}

// out[s] += sum of partials (fixed order)
__global__ void __launch_bounds__(64 * FIN_Y) k_fin_accum(Map m, const double* __restrict__ part,
                                                          double* __restrict__ out) {
  __shared__ double lds[64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double a[1];
  reduce_partials<1>(m, part, s, a, lds);
  if (threadIdx.y == 0 && s < m.S) out[s] += a[0];
}

// Contract the per-cell sensitivities with dphi/dtheta_k and dK/dtheta_k: partials [12][ncb][S].
// KL model: phi depends on xi_1..4 (not where clipped), K on eta_1..8 through ln K.  The
// paper's model (section 4): phi = phi_hat C0 C1 C2 (eq. poro_2levels) depends on xi_1 =
// theta[0] and xi_2 = theta[1] (product rule), and K = kappa phi^3 / (1 - phi^2) (eq.
// e_perm_Kozeny_Carman) on phi, with dK/dphi = kappa phi^2 (3 - phi^2) / (1 - phi^2)^2.
__global__ void __launch_bounds__(256) k_adj_theta(Map m, Grid2 G, Phys P, KLModes kl, FieldParams fp,
                                                   const double* __restrict__ theta, const double* __restrict__ K,
                                                   const double* __restrict__ gphi, const double* __restrict__ gK,
                                                   double* __restrict__ part) {
  __shared__ double lds[12 * 256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int kk = 0; kk < m.CPT; ++kk) {
    const int cell = (cblk * m.CPT + kk) * m.CY + threadIdx.y;
    if (!sv || cell >= G.ncell) continue;
    const int j = cell / G.nx, i = cell - j * G.nx;
    const double x = (i + 0.5) * P.hx, y = -P.Ly + (j + 0.5) * P.hy;
    const size_t id = (size_t)cell * m.S + s;
    const double* th = theta + (size_t)s * 13;
    if (fp.model == 1) {
      const double xi1 = th[0], xi2 = th[1];
      const bool low = y < -0.8;
      const double c0 = low ? 1.2 * (1.0 + 0.2 * xi1) : 1.0;
      const double c1 = 1.0 + 0.15 * (xi2 * cospi(0.5 * x) - xi2 * sinpi(2.0 * y) + xi1 * cospi(2.0 * x));
      const double c2 = 1.0 + 0.2 * (xi1 * sinpi(64.0 * x) + xi2 * sinpi(32.0 * y));
      const double d0_1 = low ? 1.2 * 0.2 : 0.0;
      const double d1_1 = 0.15 * cospi(2.0 * x), d2_1 = 0.2 * sinpi(64.0 * x);
      const double d1_2 = 0.15 * (cospi(0.5 * x) - sinpi(2.0 * y)), d2_2 = 0.2 * sinpi(32.0 * y);
      const double ph = fp.phi_mean * c0 * c1 * c2, ph2 = ph * ph, om = 1.0 - ph2;
      const double dKdphi = fp.kappa_kc * ph2 * (3.0 - ph2) / (om * om);
      const double g = gphi[id] + gK[id] * dKdphi;
      acc[0] += g * fp.phi_mean * (d0_1 * c1 * c2 + c0 * d1_1 * c2 + c0 * c1 * d2_1);
      acc[1] += g * fp.phi_mean * (c0 * d1_2 * c2 + c0 * c1 * d2_2);
      continue;
    }
    double e[8];
    double sp = 0.0;
    for (int k = 0; k < kl.n; ++k) {
      e[k] = kl_1d(kl.wx[k], kl.oddx[k], kl.normx[k], x - kl.xc) * kl_1d(kl.wy[k], kl.oddy[k], kl.normy[k], y - kl.yc);
      if (k < fp.n_phi) sp += kl.sqrt_lam[k] * th[k] * e[k];
    }
    const double raw = fp.phi_mean * (1.0 + fp.phi_amp * sp);
    const bool inside = raw > fp.phi_min && raw < fp.phi_max;
    const double gp = gphi[id], gk = gK[id] * K[id];
    for (int k = 0; k < fp.n_phi; ++k)
      if (inside) acc[k] += gp * fp.phi_mean * fp.phi_amp * kl.sqrt_lam[k] * e[k];
    for (int k = 0; k < fp.n_logK; ++k) acc[4 + k] += gk * fp.logK_amp * kl.sqrt_lam[k] * e[k];
  }
  block_sum_y<12>(acc, lds);
  if (threadIdx.y == 0 && sv) {
#pragma unroll
    for (int k = 0; k < 12; ++k) part[((size_t)k * m.ncb + cblk) * m.S + s] = acc[k];
  }
}

__global__ void __launch_bounds__(64 * FIN_Y) k_fin_theta(Map m, const double* __restrict__ part,
                                                          const double* __restrict__ guin, double duin_dzeta,
                                                          double* __restrict__ out) {
  __shared__ double lds[4 * 64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  for (int k0 = 0; k0 < 12; k0 += 4) {
    double a[4];
    reduce_partials<4>(m, part + (size_t)k0 * m.ncb * m.S, s, a, lds);
    if (threadIdx.y == 0 && s < m.S) {
#pragma unroll
      for (int q = 0; q < 4; ++q) out[(size_t)s * 13 + k0 + q] = a[q];
    }
  }
  if (threadIdx.y == 0 && s < m.S) out[(size_t)s * 13 + 12] = guin[s] * duin_dzeta;
}

__global__ void k_zero_f64(size_t n, double* __restrict__ a) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] = 0.0;
}

// out = a x + b y (first guess of a transposed solve from earlier adjoint solutions)
__global__ void k_axpby(size_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ out) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = a * x[t] + b * y[t];
}

}  // namespace henry
