// Batched band LU with partial pivoting of the coarsest multigrid grid (Gaussian elimination on
// the coarse grid, section 2.3), one workgroup per sample.
#pragma once

#include <hip/hip_runtime.h>

namespace henry {

// Scalar unknowns r = 2q + a, cells q = i * nyc + j (j fastest), a = 0 pressure, 1 concentration.
// The five-point 2x2-block operator then has kl = ku = 2 nyc + 1 scalar diagonals on either
// side.  Partial pivoting picks, at step j, the first row of largest magnitude among rows
// j .. j + kl of column j (the rows below hold exact zeros, which never win and stay zero), so
// the pivots, multipliers and rows of U are those of Gaussian elimination with partial pivoting
// of the dense matrix; the row interchanges widen U to kl + ku superdiagonals.
// Factor storage per sample: U [n][GB_C] (row j: U(j, j .. j + kl + ku), diagonal first), then
// L [n][kl] (column j: the multipliers of rows j + 1 .. j + kl after step j's interchange);
// piv [n]: step j exchanged rows j and j + piv[j].
__host__ __device__ inline int gb_kl(int nyc) { return 2 * nyc + 1; }
__host__ __device__ inline int gb_cols(int nyc) { return 2 * gb_kl(nyc) + 1; }
__host__ __device__ inline size_t gb_stride(int nxc, int nyc) {
  const size_t n = 2 * (size_t)nxc * nyc;
  return n * (gb_cols(nyc) + gb_kl(nyc));
}
template <typename T>
__host__ __device__ inline size_t gb_factor_lds(int nyc) {
  return (size_t)(gb_kl(nyc) + 1) * gb_cols(nyc) * sizeof(T);
}
constexpr int GB_THREADS = 256;
constexpr int GB_CH = 16;   // steps per staged chunk of the solves
template <typename T>
__host__ __device__ inline size_t gb_solve_lds(int nxc, int nyc) {
  return (2 * (size_t)nxc * nyc + (size_t)GB_CH * (gb_cols(nyc) + gb_kl(nyc))) * sizeof(T) + GB_CH * sizeof(int);
}

// scalar entry (r, c) of the coarse operator, 0 outside the stencil or the matrix
template <typename T>
__device__ __forceinline__ T gb_entry(const T* __restrict__ J, size_t N, int S, int s, int nxc, int nyc, int r, int c) {
  const int n = 2 * nxc * nyc;
  if (r < 0 || c < 0 || r >= n || c >= n) return (T)0;
  const int q = r >> 1, a = r & 1, q2 = c >> 1, b = c & 1, d = q2 - q;
  const int i = q / nyc, j = q - i * nyc;
  int blk = -1;
  if (d == 0) blk = 0;
  else if (d == -1 && j > 0) blk = 3;
  else if (d == 1 && j < nyc - 1) blk = 4;
  else if (d == -nyc && i > 0) blk = 1;
  else if (d == nyc && i < nxc - 1) blk = 2;
  if (blk < 0) return (T)0;
  return J[(blk * 4 + a * 2 + b) * N + ((size_t)j * nxc + i) * S + s];
}

// Factorisation.  The active window, rows j .. j + kl by columns j .. j + kl + ku, lives in LDS
// as a circular buffer in both directions; after step j row j leaves (written out as a row of
// U) and row j + kl + 1 of the matrix enters in its slot, and column j's slot takes column
// j + kl + ku + 1 (zero above the entering row: no row above it reaches that far).
// Launch: grid S, block GB_THREADS, dynamic LDS gb_factor_lds<T>(nyc); needs kl + 1 <= 64.
template <typename T>
__global__ void __launch_bounds__(GB_THREADS) k_gb_factor(int S, int nxc, int nyc, const T* __restrict__ J,
                                                          T* __restrict__ LU, int* __restrict__ piv) {
  extern __shared__ unsigned char smem_raw[];
  T* W = reinterpret_cast<T*>(smem_raw);
  __shared__ int sp;
  const int s = blockIdx.x, t = threadIdx.x;
  const int n = 2 * nxc * nyc, kl = gb_kl(nyc), R = kl + 1, C = gb_cols(nyc), ku2 = C - 1;
  const size_t N = (size_t)nxc * nyc * S;
  T* Ug = LU + (size_t)s * gb_stride(nxc, nyc);
  T* Lg = Ug + (size_t)n * C;
  int* pg = piv + (size_t)s * n;
  auto w = [&](int r, int c) -> T& { return W[(r % R) * C + (c % C)]; };
  for (int e = t; e < R * C; e += GB_THREADS) {
    const int r = e / C, c = e - r * C;
    w(r, c) = (c - r <= kl && r - c <= kl) ? gb_entry<T>(J, N, S, s, nxc, nyc, r, c) : (T)0;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int km = (n - 1 - j) < kl ? (n - 1 - j) : kl;
    if (t < 64) {   // pivot: first row of largest magnitude (wave reduction, lowest index on ties)
      T v = t <= km ? fabs(w(j + t, j)) : (T)-1;
      int idx = t;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const T v2 = __shfl_xor(v, off);
        const int i2 = __shfl_xor(idx, off);
        if (v2 > v || (v2 == v && i2 < idx)) {
          v = v2;
          idx = i2;
        }
      }
      if (t == 0) {
        sp = idx;
        pg[j] = idx;
      }
    }
    __syncthreads();
    const int p = sp;
    for (int c = t; c < C; c += GB_THREADS) {   // interchange rows j and j + p; row j of U out
      const T a = w(j, j + c), b = w(j + p, j + c);
      if (p) {
        w(j, j + c) = b;
        w(j + p, j + c) = a;
      }
      Ug[(size_t)j * C + c] = p ? b : a;
    }
    __syncthreads();
    const T pv = w(j, j);
    for (int i = t; i < km; i += GB_THREADS) {
      const T l = w(j + 1 + i, j) / pv;
      w(j + 1 + i, j) = l;
      Lg[(size_t)j * kl + i] = l;
    }
    __syncthreads();
    for (int e = t; e < km * ku2; e += GB_THREADS) {   // rank-1 update of the trailing window
      const int i = e / ku2, c = e - i * ku2;
      w(j + 1 + i, j + 1 + c) -= w(j + 1 + i, j) * w(j, j + 1 + c);
    }
    __syncthreads();
    const int rn = j + R;   // entering row: its band is exactly the window's columns j+1 .. j+C
    for (int c = t; c < C; c += GB_THREADS) {
      const int col = j + 1 + c;
      w(rn, col) = gb_entry<T>(J, N, S, s, nxc, nyc, rn, col);
    }
    for (int i = t; i < kl; i += GB_THREADS) w(j + 1 + i, j + C) = (T)0;
    __syncthreads();
  }
}

// x = A^{-1} b (TR = false) or A^{-T} b (TR = true) with the factors of k_gb_factor, one wavefront
// per sample; the right-hand side lives in LDS, the factor rows are staged GB_CH steps at a time.
//   A = P_0 L_0 P_1 L_1 ... P_{n-1} L_{n-1} U  (P_j: the interchange of step j, L_j: its multipliers)
//   A x = b:    for j up: swap, y_{j+i} -= l_j[i] y_j;          then U x = y with rows of U (dots)
//   A^T x = b:  U^T z = b with rows of U (axpy, j up);          then for j down:
//               z_j -= sum_i l_j[i] z_{j+i}, swap
// Launch: grid S, block 64, dynamic LDS gb_solve_lds<T>(nxc, nyc).
template <typename T, bool TR>
__global__ void __launch_bounds__(64) k_gb_solve(int S, int nxc, int nyc, const T* __restrict__ LU,
                                                 const int* __restrict__ piv, const T* __restrict__ b,
                                                 T* __restrict__ x) {
  extern __shared__ unsigned char smem_raw[];
  const int s = blockIdx.x, lane = threadIdx.x;
  const int nc = nxc * nyc, n = 2 * nc, kl = gb_kl(nyc), C = gb_cols(nyc), ku2 = C - 1;
  T* y = reinterpret_cast<T*>(smem_raw);
  T* Us = y + n;                            // [GB_CH][C]
  T* Ls = Us + (size_t)GB_CH * C;           // [GB_CH][kl]
  int* ps = reinterpret_cast<int*>(Ls + (size_t)GB_CH * kl);
  const size_t N = (size_t)nc * S;
  const T* Ug = LU + (size_t)s * gb_stride(nxc, nyc);
  const T* Lg = Ug + (size_t)n * C;
  const int* pg = piv + (size_t)s * n;
  for (int q = lane; q < nc; q += 64) {
    const int i = q / nyc, j = q - i * nyc;
    const size_t g = ((size_t)j * nxc + i) * S + s;
    y[2 * q] = b[g];
    y[2 * q + 1] = b[N + g];
  }
  // stage steps [j0, j1): U rows, L columns and pivots
  auto stage = [&](int j0, int j1, bool wantU, bool wantL) {
    if (wantU)
      for (int e = lane; e < (j1 - j0) * C; e += 64) Us[e] = Ug[(size_t)j0 * C + e];
    if (wantL) {
      for (int e = lane; e < (j1 - j0) * kl; e += 64) Ls[e] = Lg[(size_t)j0 * kl + e];
      for (int e = lane; e < j1 - j0; e += 64) ps[e] = pg[j0 + e];
    }
    __syncthreads();
  };
  if (!TR) {
    for (int j0 = 0; j0 < n; j0 += GB_CH) {   // y = L_{n-1}^{-1} P_{n-1} ... L_0^{-1} P_0 b
      const int j1 = j0 + GB_CH < n ? j0 + GB_CH : n;
      stage(j0, j1, false, true);
      for (int j = j0; j < j1; ++j) {
        const int p = ps[j - j0], km = (n - 1 - j) < kl ? (n - 1 - j) : kl;
        const T yj = y[j], yp = y[j + p];   // after the interchange y_j = yp, y_{j+p} = yj
        const int i = lane + 1;
        T v = 0;
        if (i <= km) v = (i == p ? yj : y[j + i]) - Ls[(j - j0) * kl + lane] * yp;
        __syncthreads();
        if (i <= km) y[j + i] = v;
        if (lane == 0) y[j] = yp;
        __syncthreads();
      }
      __syncthreads();
    }
    for (int j1 = n; j1 > 0; j1 -= GB_CH) {   // U x = y, row by row from the bottom
      const int j0 = j1 - GB_CH > 0 ? j1 - GB_CH : 0;
      stage(j0, j1, true, false);
      for (int j = j1 - 1; j >= j0; --j) {
        const T* u = Us + (size_t)(j - j0) * C;
        const int m = (n - 1 - j) < ku2 ? (n - 1 - j) : ku2;
        T acc = 0;
        for (int i = lane + 1; i <= m; i += 64) acc += u[i] * y[j + i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        const T xj = (y[j] - acc) / u[0];
        __syncthreads();
        if (lane == 0) y[j] = xj;
        __syncthreads();
      }
      __syncthreads();
    }
  } else {
    for (int j0 = 0; j0 < n; j0 += GB_CH) {   // U^T z = b, column by column from the top
      const int j1 = j0 + GB_CH < n ? j0 + GB_CH : n;
      stage(j0, j1, true, false);
      for (int j = j0; j < j1; ++j) {
        const T* u = Us + (size_t)(j - j0) * C;
        const int m = (n - 1 - j) < ku2 ? (n - 1 - j) : ku2;
        const T zj = y[j] / u[0];
        for (int i = lane + 1; i <= m; i += 64) y[j + i] -= u[i] * zj;
        if (lane == 0) y[j] = zj;
        __syncthreads();
      }
      __syncthreads();
    }
    for (int j1 = n; j1 > 0; j1 -= GB_CH) {   // then L_j^{-T} and the interchange, j down
      const int j0 = j1 - GB_CH > 0 ? j1 - GB_CH : 0;
      stage(j0, j1, false, true);
      for (int j = j1 - 1; j >= j0; --j) {
        const int p = ps[j - j0], km = (n - 1 - j) < kl ? (n - 1 - j) : kl;
        T acc = 0;
        if (lane < km) acc = Ls[(j - j0) * kl + lane] * y[j + 1 + lane];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        const T zj = y[j] - acc, zp = y[j + p];
        __syncthreads();
        if (lane == 0) {
          y[j] = zp;        // interchange after the update (p = 0 leaves zj in place)
          y[j + p] = zj;
        }
        __syncthreads();
      }
      __syncthreads();
    }
  }
  for (int q = lane; q < nc; q += 64) {
    const int i = q / nyc, j = q - i * nyc;
    const size_t g = ((size_t)j * nxc + i) * S + s;
    x[g] = y[2 * q];
    x[N + g] = y[2 * q + 1];
  }
}

}  // namespace henry
