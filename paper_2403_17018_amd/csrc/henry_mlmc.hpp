// Small control kernels, the time-resolved QoIs (section 5) and the MLMC estimator kernels
// (section 3).
#pragma once

#include <hip/hip_runtime.h>

#include "henry_kernels.hpp"

namespace henry {

__global__ void k_zero_int(int* __restrict__ a, int n) {
  const int t = threadIdx.x;
  if (t < n) a[t] = 0;
}

__global__ void k_zero_i32(size_t n, int* __restrict__ a) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] = 0;
}

__global__ void k_check_finite(size_t n, const double* __restrict__ a, int* __restrict__ flag) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && !isfinite(a[t])) atomicOr(flag, 1);
}

// stats[s][1] += BiCGStab iterations of the last linear solve
__global__ void k_accum_its(int S, const double* __restrict__ sc, double* __restrict__ stats) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) stats[(size_t)s * 4 + 1] += sc[7 * S + s];
}

__global__ void k_mark_unconverged(int S, const int* __restrict__ ndone, int* __restrict__ status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S && !ndone[s] && status[s] == 0) status[s] = 1;
}

__global__ void k_count_nonzero(int S, const int* __restrict__ a, int* __restrict__ count) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S && a[s] != 0) atomicAdd(count, 1);
}

// Initial Newton guess by extrapolation in time: u <- u + gamma (u - u_prev), u_prev <- u
// (old u); gamma = 0 (first step) only records u.
__global__ void k_extrapolate(size_t n, double gamma, double* __restrict__ u, double* __restrict__ u_prev) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double un = u[t];
  if (gamma != 0.0) u[t] = un + gamma * (un - u_prev[t]);
  u_prev[t] = un;
}

// Polynomial extrapolation through the last order + 1 steps (order 0: u kept, the first
// step; 1: 2u - h1; 2: 3u - 3h1 + h2; 3: 4u - 6h1 + 4h2 - h3), h1..h3 the states of the
// previous steps (h3 may be NULL when order never exceeds 2); the history shifts by one.
__global__ void k_extrapolate_poly(size_t n, int order, double* __restrict__ u, double* __restrict__ h1,
                                   double* __restrict__ h2, double* __restrict__ h3) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double un = u[t];
  const double a = order > 0 ? h1[t] : un;
  const double b = order > 1 ? h2[t] : a;
  if (order == 3) u[t] = 4.0 * (un + b) - 6.0 * a - h3[t];
  else if (order == 2) u[t] = 3.0 * (un - a) + b;
  else if (order == 1) u[t] = 2.0 * un - a;
  if (h3) h3[t] = b;
  h2[t] = a;
  h1[t] = un;
}

// Indices of the samples with ndone[s] == 0, in increasing order.  One block: each thread
// owns a contiguous range of samples, counts its active ones, and an exclusive scan of the
// counts (in LDS) gives where its indices start.
constexpr int COMPACT_THREADS = 1024;
__global__ void __launch_bounds__(COMPACT_THREADS) k_compact_index(int S, const int* __restrict__ ndone,
                                                                   int* __restrict__ idx) {
  __shared__ int cnt[COMPACT_THREADS];
  const int t = threadIdx.x, T = blockDim.x;
  const int per = (S + T - 1) / T;
  const int s0 = min(S, t * per), s1 = min(S, s0 + per);
  int c = 0;
  for (int s = s0; s < s1; ++s) c += ndone[s] == 0;
  cnt[t] = c;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {   // inclusive scan (Hillis-Steele)
    const int v = t >= off ? cnt[t - off] : 0;
    __syncthreads();
    cnt[t] += v;
    __syncthreads();
  }
  int a = cnt[t] - c;
  for (int s = s0; s < s1; ++s)
    if (ndone[s] == 0) idx[a++] = s;
}

// dst[r][a] = src[r][idx[a]] for rows r of sample-fastest arrays ([rows][S] -> [rows][Sa])
__global__ void k_gather_cols(size_t rows, int S, int Sa, const int* __restrict__ idx, const double* __restrict__ src,
                              double* __restrict__ dst) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * Sa) return;
  const size_t r = t / Sa, a = t - r * Sa;
  dst[t] = src[r * S + idx[a]];
}

__global__ void k_scatter_cols(size_t rows, int S, int Sa, const int* __restrict__ idx, const double* __restrict__ src,
                               double* __restrict__ dst) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * Sa) return;
  const size_t r = t / Sa, a = t - r * Sa;
  dst[r * S + idx[a]] = src[t];
}

__global__ void k_gather_sample_info(int Sa, const int* __restrict__ idx, const int* __restrict__ status,
                                     const double* __restrict__ stats, const double* __restrict__ nhist,
                                     int* __restrict__ cstatus, double* __restrict__ cstats,
                                     double* __restrict__ cnhist) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= Sa) return;
  const int s = idx[a];
  cstatus[a] = status[s];
  for (int q = 0; q < 4; ++q) cstats[(size_t)a * 4 + q] = stats[(size_t)s * 4 + q];
  cnhist[2 * a] = nhist[2 * s];
  cnhist[2 * a + 1] = nhist[2 * s + 1];
}

__global__ void k_scatter_sample_info(int Sa, const int* __restrict__ idx, const int* __restrict__ cstatus,
                                      const double* __restrict__ cstats, const int* __restrict__ cndone,
                                      const double* __restrict__ cnhist, int* __restrict__ status,
                                      double* __restrict__ stats, int* __restrict__ ndone,
                                      double* __restrict__ nhist) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= Sa) return;
  const int s = idx[a];
  status[s] = cstatus[a];
  ndone[s] = cndone[a];
  for (int q = 0; q < 4; ++q) stats[(size_t)s * 4 + q] = cstats[(size_t)a * 4 + q];
  nhist[2 * s] = cnhist[2 * a];
  nhist[2 * s + 1] = cnhist[2 * a + 1];
}

// Time-resolved QoIs of the current state (section 5), per-sample partial sums
// [NSERIES][ncb][S]: 0: Q_S = sum c rho(c) |cell| (eq. integral_s); 1: Q_FW = area of the
// cells with c <= 0.012178 (eq. integral_fw); 2 + b: sum c rho(c) |cell n Delta_b| with
// Delta_b the square of half-width 0.1 around point b of eq. 12points (eq. integral_box).
// The cell-wise constant field is integrated exactly over each box.
constexpr int NSERIES = 17;
__global__ void __launch_bounds__(256) k_series(Map m, Grid2 G, Phys P, const double* __restrict__ c,
                                                double* __restrict__ part) {
  __shared__ double lds[NSERIES * 256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  double acc[NSERIES];
#pragma unroll
  for (int q = 0; q < NSERIES; ++q) acc[q] = 0.0;
  for (int kk = 0; kk < m.CPT; ++kk) {
    const int cell = (cblk * m.CPT + kk) * m.CY + threadIdx.y;
    if (!sv || cell >= G.ncell) continue;
    const int j = cell / G.nx, i = cell - j * G.nx;
    const double cP = c[(size_t)cell * m.S + s];
    const double mass = cP * (P.rho0 + P.drho * cP);
    acc[0] += mass * P.vol;
    acc[1] += cP <= 0.012178 ? P.vol : 0.0;
    const double x0 = i * P.hx, x1 = (i + 1) * P.hx;
    const double y0 = -P.Ly + j * P.hy, y1 = -P.Ly + (j + 1) * P.hy;
#pragma unroll
    for (int b = 0; b < 15; ++b) {
      const int col = b % 5, row = b / 5;
      const double bx = col == 0 ? 0.90 : col == 1 ? 1.15 : col == 2 ? 1.40 : col == 3 ? 1.65 : 1.90;
      const double by = row == 0 ? -0.95 : row == 1 ? -0.75 : -0.50;
      const double ox = fmax(0.0, fmin(x1, bx + 0.1) - fmax(x0, bx - 0.1));
      const double oy = fmax(0.0, fmin(y1, by + 0.1) - fmax(y0, by - 0.1));
      acc[2 + b] += mass * (oy * ox);
    }
  }
  block_sum_y<NSERIES>(acc, lds);
  if (threadIdx.y == 0 && sv) {
#pragma unroll
    for (int q = 0; q < NSERIES; ++q) part[((size_t)q * m.ncb + cblk) * m.S + s] = acc[q];
  }
}

// out[q][s] = sum of the partials (fixed order), q < NSERIES
__global__ void __launch_bounds__(64 * FIN_Y) k_fin_series(Map m, const double* __restrict__ part,
                                                           double* __restrict__ out) {
  __shared__ double lds[4 * 64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  for (int q0 = 0; q0 < 16; q0 += 4) {
    double a[4];
    reduce_partials<4>(m, part + (size_t)q0 * m.ncb * m.S, s, a, lds);
    if (threadIdx.y == 0 && s < m.S) {
#pragma unroll
      for (int q = 0; q < 4; ++q) out[(size_t)(q0 + q) * m.S + s] = a[q];
    }
  }
  double a[1];
  reduce_partials<1>(m, part + (size_t)16 * m.ncb * m.S, s, a, lds);
  if (threadIdx.y == 0 && s < m.S) out[(size_t)16 * m.S + s] = a[0];
}

// Fixed-order tree sum over 256 threads.
__device__ __forceinline__ double block_sum_256(double v, double* lds) {
  const int t = threadIdx.x;
  __syncthreads();
  lds[t] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) lds[t] += lds[t + w];
    __syncthreads();
  }
  return lds[0];
}

// Mean and unbiased variance of Y = g_fine - g_coarse (g_coarse may be NULL): out[0], out[1].
__global__ void __launch_bounds__(256) k_level_moments(int m, const double* __restrict__ gf,
                                                       const double* __restrict__ gc, double* __restrict__ out) {
  __shared__ double lds[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) a += gf[i] - (gc ? gc[i] : 0.0);
  const double mean = block_sum_256(a, lds) / m;
  double q = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    const double d = gf[i] - (gc ? gc[i] : 0.0) - mean;
    q += d * d;
  }
  const double ss = block_sum_256(q, lds);
  if (threadIdx.x == 0) {
    out[0] = mean;
    out[1] = m > 1 ? ss / (m - 1) : 0.0;
  }
}

// Per cell: mean and unbiased variance over m samples of a [cell][m] field.
__global__ void k_cell_moments(int ncell, int m, const double* __restrict__ f, double* __restrict__ mean,
                               double* __restrict__ var) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const double* v = f + (size_t)c * m;
  double a = 0.0;
  for (int s = 0; s < m; ++s) a += v[s];
  const double mu = a / m;
  double q = 0.0;
  for (int s = 0; s < m; ++s) {
    const double d = v[s] - mu;
    q += d * d;
  }
  mean[c] = mu;
  var[c] = m > 1 ? q / (m - 1) : 0.0;
}

// Time-resolved MLMC: per level l, common time k and QoI q, mean and unbiased variance over
// the m_l samples of Y = s_f[l][(k+1) df_l - 1][q][i] - s_c[l][(k+1) dc_l - 1][q][i] (no coarse
// term on level 0).  Block (k*nq + q, l); out: Ymean, V [L+1][r0][nq].
struct SeriesLevels {
  enum { MAXL = 8 };
  int L, nq, r0;
  int m[MAXL], df[MAXL], dc[MAXL];
  const double* f[MAXL];
  const double* c[MAXL];
};

__global__ void __launch_bounds__(256) k_series_moments(SeriesLevels sl, double* __restrict__ Ymean,
                                                        double* __restrict__ V) {
  __shared__ double lds[256];
  const int kq = blockIdx.x, l = blockIdx.y;
  const int k = kq / sl.nq, q = kq - k * sl.nq;
  const int m = sl.m[l];
  const double* gf = sl.f[l] + ((size_t)((k + 1) * sl.df[l] - 1) * sl.nq + q) * m;
  const double* gc = l > 0 ? sl.c[l] + ((size_t)((k + 1) * sl.dc[l] - 1) * sl.nq + q) * m : nullptr;
  double a = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) a += gf[i] - (gc ? gc[i] : 0.0);
  const double mean = block_sum_256(a, lds) / m;
  double v = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    const double d = gf[i] - (gc ? gc[i] : 0.0) - mean;
    v += d * d;
  }
  const double ss = block_sum_256(v, lds);
  if (threadIdx.x == 0) {
    const size_t o = ((size_t)l * sl.r0 + k) * sl.nq + q;
    Ymean[o] = mean;
    V[o] = m > 1 ? ss / (m - 1) : 0.0;
  }
}

// mean[k][q] = sum_l Ymean[l][k][q], var_of_estimator[k][q] = sum_l V[l][k][q] / m_l (level order)
__global__ void k_series_combine(SeriesLevels sl, const double* __restrict__ Ymean, const double* __restrict__ V,
                                 double* __restrict__ mean, double* __restrict__ var) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = sl.r0 * sl.nq;
  if (t >= n) return;
  double mu = 0.0, va = 0.0;
  for (int l = 0; l <= sl.L; ++l) {
    mu += Ymean[(size_t)l * n + t];
    va += V[(size_t)l * n + t] / sl.m[l];
  }
  if (mean) mean[t] = mu;
  if (var) var[t] = va;
}

struct FieldLevels {
  enum { MAXL = 8 };
  int L;
  int nx[MAXL];
  long long off[MAXL];
};

// Telescoping field moments on the finest grid with piecewise-constant injection.
__global__ void k_field_accumulate(FieldLevels fl, int nxL, int nyL, const double* __restrict__ tmp,
                                   double* __restrict__ mean, double* __restrict__ var) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nxL * nyL) return;
  const int j = c / nxL, i = c - j * nxL;
  double mu = 0.0, va = 0.0;
  for (int l = 0; l <= fl.L; ++l) {
    const int sh = fl.L - l;
    const int il = i >> sh, jl = j >> sh;
    const int nxl = fl.nx[l];
    const int nyl = nyL >> sh;
    const int ncl = nxl * nyl;
    const double* t = tmp + fl.off[l];
    mu += t[jl * nxl + il];
    va += t[ncl + jl * nxl + il];
    if (l > 0) {
      const int nxc = nxl >> 1, ncc = ncl >> 2;
      const int ic = il >> 1, jc = jl >> 1;
      mu -= t[2 * ncl + jc * nxc + ic];
      va -= t[2 * ncl + ncc + jc * nxc + ic];
    }
  }
  if (mean) mean[c] = mu;
  if (var) var[c] = va;
}

}  // namespace henry
