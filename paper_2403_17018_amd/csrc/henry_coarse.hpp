// Batched block-banded LU of the coarsest multigrid grid (one wavefront per sample).
#pragma once

#include <hip/hip_runtime.h>

namespace henry {

// ==========================================================================
// a6: batched block-banded LU of the coarsest grid (one wavefront per sample)
// ==========================================================================
// Unknowns ordered cell-by-cell with j fastest (q = i*ny + j), so the 2x2-block
// matrix has block bandwidth m = ny.  No pivoting: the diagonal blocks of this
// operator are nonsingular and the pressure block is an M-matrix.  The active
// (m+1)x(m+1)-block window lives in LDS as a circular buffer; finished rows of U,
// columns of L and inverted diagonal blocks are written to the sample's factor
// storage, laid out per sample: [Dinv n][L n*m][U n*m] blocks of 4.
template <typename T>
__device__ __forceinline__ void band_orig(const T* __restrict__ J, size_t N, int S, int s, int nxc, int nyc, int q,
                                          int d, T out[4]) {
  // block (row q, column q + d) of the coarse Jacobian, zero outside the stencil
  const int i = q / nyc, j = q - i * nyc;
  int blk = -1;
  if (d == 0) blk = 0;
  else if (d == -1 && j > 0) blk = 3;
  else if (d == 1 && j < nyc - 1) blk = 4;
  else if (d == -nyc && i > 0) blk = 1;
  else if (d == nyc && i < nxc - 1) blk = 2;
  if (blk < 0) {
    out[0] = out[1] = out[2] = out[3] = (T)0;
    return;
  }
  const size_t id = ((size_t)j * nxc + i) * S + s;
#pragma unroll
  for (int e = 0; e < 4; ++e) out[e] = J[(blk * 4 + e) * N + id];
}

template <typename T>
__global__ void __launch_bounds__(64) k_band_factor(int S, int nxc, int nyc, const T* __restrict__ J,
                                                    T* __restrict__ LU) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* W = reinterpret_cast<T*>(smem_raw);
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = nxc * nyc, mb = nyc, w = mb + 1;
  const size_t N = (size_t)n * S;
  T* Dg = LU + (size_t)s * n * (2 * mb + 1) * 4;
  T* Lg = Dg + (size_t)n * 4;
  T* Ug = Lg + (size_t)n * mb * 4;
  // initial window: rows/cols 0..min(w,n)-1
  const int w0 = w < n ? w : n;
  for (int t = lane; t < w0 * w0; t += 64) {
    const int a = t / w0, b = t - a * w0;
    T blk[4];
    const int d = b - a;
    if (d >= -mb && d <= mb) band_orig<T>(J, N, S, s, nxc, nyc, a, d, blk);
    else blk[0] = blk[1] = blk[2] = blk[3] = (T)0;
#pragma unroll
    for (int e = 0; e < 4; ++e) W[((a % w) * w + (b % w)) * 4 + e] = blk[e];
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const int rk = k % w;
    const T* Dk = &W[(rk * w + rk) * 4];
    const T det = Dk[0] * Dk[3] - Dk[1] * Dk[2];
    const T i00 = Dk[3] / det, i01 = -Dk[1] / det, i10 = -Dk[2] / det, i11 = Dk[0] / det;
    const int nrow = (n - 1 - k) < mb ? (n - 1 - k) : mb;
    __syncthreads();
    // L_ik = A_ik Dinv_k (stored in the window column k); U row k written out
    for (int t = lane; t < nrow; t += 64) {
      const int ri = (k + 1 + t) % w;
      T* A = &W[(ri * w + rk) * 4];
      const T l00 = A[0] * i00 + A[1] * i10, l01 = A[0] * i01 + A[1] * i11;
      const T l10 = A[2] * i00 + A[3] * i10, l11 = A[2] * i01 + A[3] * i11;
      A[0] = l00; A[1] = l01; A[2] = l10; A[3] = l11;
      T* Lo = Lg + ((size_t)k * mb + t) * 4;
      Lo[0] = l00; Lo[1] = l01; Lo[2] = l10; Lo[3] = l11;
      const T* Uk = &W[(rk * w + ri) * 4];
      T* Uo = Ug + ((size_t)k * mb + t) * 4;
      Uo[0] = Uk[0]; Uo[1] = Uk[1]; Uo[2] = Uk[2]; Uo[3] = Uk[3];
    }
    if (lane == 0) {
      T* Do = Dg + (size_t)k * 4;
      Do[0] = i00; Do[1] = i01; Do[2] = i10; Do[3] = i11;
    }
    __syncthreads();
    // trailing update A_ij -= L_ik U_kj
    for (int t = lane; t < nrow * nrow; t += 64) {
      const int a = t / nrow, b = t - a * nrow;
      const int ri = (k + 1 + a) % w, cj = (k + 1 + b) % w;
      const T* L = &W[(ri * w + rk) * 4];
      const T* U = &W[(rk * w + cj) * 4];
      T* A = &W[(ri * w + cj) * 4];
      A[0] -= L[0] * U[0] + L[1] * U[2];
      A[1] -= L[0] * U[1] + L[1] * U[3];
      A[2] -= L[2] * U[0] + L[3] * U[2];
      A[3] -= L[2] * U[1] + L[3] * U[3];
    }
    __syncthreads();
    // slide: slot rk becomes row and column k + w
    const int kn = k + w;
    if (kn < n) {
      for (int t = lane; t < w + mb; t += 64) {
        T blk[4];
        int slot;
        if (t < w) {          // new row kn, columns kn-mb .. kn
          const int col = kn - mb + t;
          band_orig<T>(J, N, S, s, nxc, nyc, kn, col - kn, blk);
          slot = (rk * w + (col % w)) * 4;
        } else {              // new column kn, rows k+1 .. k+mb
          const int row = k + 1 + (t - w);
          band_orig<T>(J, N, S, s, nxc, nyc, row, kn - row, blk);
          slot = ((row % w) * w + rk) * 4;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) W[slot + e] = blk[e];
      }
    }
    __syncthreads();
  }
}

// Forward/backward substitution with the banded factors: x = (LU)^{-1} b, one
// wavefront per sample.  The whole right-hand side lives in LDS; the factor blocks
// are staged into LDS in chunks of CH block rows, so a global-load latency is paid
// once per chunk instead of once per row.  One barrier per row.
// LDS layout (T): y[2n] | x[2n] | stage[CH*mb*4 + (CH+mb)*mb*4 + CH*4]
template <typename T>
__global__ void __launch_bounds__(64) k_band_solve(int S, int nxc, int nyc, int CH, const T* __restrict__ LU,
                                                   const T* __restrict__ b, T* __restrict__ x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = nxc * nyc, mb = nyc;
  T* y = reinterpret_cast<T*>(smem_raw);
  T* xs = y + 2 * n;
  T* Ls = xs + 2 * n;                    // [CH][mb][4]
  T* Us = Ls + (size_t)CH * mb * 4;      // [CH+mb][mb][4]
  T* Ds = Us + (size_t)(CH + mb) * mb * 4;  // [CH][4]
  const size_t N = (size_t)n * S;
  const T* Dg = LU + (size_t)s * n * (2 * mb + 1) * 4;
  const T* Lg = Dg + (size_t)n * 4;
  const T* Ug = Lg + (size_t)n * mb * 4;
  for (int q = lane; q < n; q += 64) {
    const int i = q / nyc, j = q - i * nyc;
    const size_t g = ((size_t)j * nxc + i) * S + s;
    y[2 * q] = b[g];
    y[2 * q + 1] = b[N + g];
  }
  // forward: y = L^{-1} b, column oriented
  for (int k0 = 0; k0 < n; k0 += CH) {
    const int k1 = (k0 + CH < n ? k0 + CH : n);
    for (int t = lane; t < (k1 - k0) * mb * 4; t += 64) Ls[t] = Lg[(size_t)k0 * mb * 4 + t];
    __syncthreads();
    for (int k = k0; k < k1; ++k) {
      const T y0 = y[2 * k], y1 = y[2 * k + 1];
      const int nrow = (n - 1 - k) < mb ? (n - 1 - k) : mb;
      if (lane < nrow) {
        const T* L = Ls + ((k - k0) * mb + lane) * 4;
        const int r = k + 1 + lane;
        y[2 * r] -= L[0] * y0 + L[1] * y1;
        y[2 * r + 1] -= L[2] * y0 + L[3] * y1;
      }
      __syncthreads();
    }
  }
  // backward: x = U^{-1} y, U = Dinv^{-1} + strict upper part, column oriented.
  // Steps k in [k0, k1) (descending) need Dinv_k and U rows [k0 - mb, k1 - 1].
  for (int k1 = n; k1 > 0; k1 -= CH) {
    const int k0 = (k1 - CH > 0 ? k1 - CH : 0);
    const int r0 = (k0 - mb > 0 ? k0 - mb : 0);
    for (int t = lane; t < (k1 - r0) * mb * 4; t += 64) Us[t] = Ug[(size_t)r0 * mb * 4 + t];
    for (int t = lane; t < (k1 - k0) * 4; t += 64) Ds[t] = Dg[(size_t)k0 * 4 + t];
    __syncthreads();
    for (int k = k1 - 1; k >= k0; --k) {
      const T* Di = Ds + (k - k0) * 4;
      const T v0 = y[2 * k], v1 = y[2 * k + 1];
      const T x0 = Di[0] * v0 + Di[1] * v1, x1 = Di[2] * v0 + Di[3] * v1;
      const int nrow = k < mb ? k : mb;
      if (lane < nrow) {
        const int row = k - 1 - lane;    // U_{row, k} = U block (row, lane)
        const T* U = Us + ((row - r0) * mb + lane) * 4;
        y[2 * row] -= U[0] * x0 + U[1] * x1;
        y[2 * row + 1] -= U[2] * x0 + U[3] * x1;
      }
      if (lane == 0) {
        xs[2 * k] = x0;
        xs[2 * k + 1] = x1;
      }
      __syncthreads();
    }
  }
  for (int q = lane; q < n; q += 64) {
    const int i = q / nyc, j = q - i * nyc;
    const size_t g = ((size_t)j * nxc + i) * S + s;
    x[g] = xs[2 * q];
    x[N + g] = xs[2 * q + 1];
  }
}

// Transposed solve x = (LU)^{-T} b = L^{-T} U^{-T} b with the same factors:
// forward with U^T (lower, diagonal blocks D^T), then backward with L^T (unit upper).
// LDS layout (T): y[2n] | stage[(CH+mb)*mb*4 + CH*4 + (CH+mb)*mb*4]
template <typename T>
__global__ void __launch_bounds__(64) k_band_solve_T(int S, int nxc, int nyc, int CH, const T* __restrict__ LU,
                                                     const T* __restrict__ b, T* __restrict__ x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = nxc * nyc, mb = nyc;
  T* y = reinterpret_cast<T*>(smem_raw);
  T* Us = y + 2 * n;                         // [CH][mb][4]  U rows of the chunk
  T* Ds = Us + (size_t)CH * mb * 4;          // [CH][4]
  T* Ls = Ds + (size_t)CH * 4;               // [CH+mb][mb][4] L columns
  const size_t N = (size_t)n * S;
  const T* Dg = LU + (size_t)s * n * (2 * mb + 1) * 4;
  const T* Lg = Dg + (size_t)n * 4;
  const T* Ug = Lg + (size_t)n * mb * 4;
  for (int q = lane; q < n; q += 64) {
    const int i = q / nyc, j = q - i * nyc;
    const size_t g = ((size_t)j * nxc + i) * S + s;
    y[2 * q] = b[g];
    y[2 * q + 1] = b[N + g];
  }
  // forward: U^T z = b; z_k = Dinv_k^T b_k, then b_j -= U_{k,j}^T z_k for j = k+1..k+mb
  for (int k0 = 0; k0 < n; k0 += CH) {
    const int k1 = (k0 + CH < n ? k0 + CH : n);
    for (int t = lane; t < (k1 - k0) * mb * 4; t += 64) Us[t] = Ug[(size_t)k0 * mb * 4 + t];
    for (int t = lane; t < (k1 - k0) * 4; t += 64) Ds[t] = Dg[(size_t)k0 * 4 + t];
    __syncthreads();
    for (int k = k0; k < k1; ++k) {
      const T* Di = Ds + (k - k0) * 4;
      const T v0 = y[2 * k], v1 = y[2 * k + 1];
      const T z0 = Di[0] * v0 + Di[2] * v1, z1 = Di[1] * v0 + Di[3] * v1;
      const int nrow = (n - 1 - k) < mb ? (n - 1 - k) : mb;
      if (lane < nrow) {
        const T* U = Us + ((k - k0) * mb + lane) * 4;   // U_{k, k+1+lane}
        const int r = k + 1 + lane;
        y[2 * r] -= U[0] * z0 + U[2] * z1;
        y[2 * r + 1] -= U[1] * z0 + U[3] * z1;
      }
      __syncthreads();
      if (lane == 0) {
        y[2 * k] = z0;
        y[2 * k + 1] = z1;
      }
      __syncthreads();
    }
  }
  // backward: L^T x = z; x_k = z_k, then z_i -= L_{k,i}^T x_k for i = k-mb..k-1,
  // with L_{k,i} = column i's block (k - i - 1).  Steps [k0, k1) need columns [k0 - mb, k1 - 1].
  for (int k1 = n; k1 > 0; k1 -= CH) {
    const int k0 = (k1 - CH > 0 ? k1 - CH : 0);
    const int r0 = (k0 - mb > 0 ? k0 - mb : 0);
    for (int t = lane; t < (k1 - r0) * mb * 4; t += 64) Ls[t] = Lg[(size_t)r0 * mb * 4 + t];
    __syncthreads();
    for (int k = k1 - 1; k >= k0; --k) {
      const T x0 = y[2 * k], x1 = y[2 * k + 1];
      const int nrow = k < mb ? k : mb;
      if (lane < nrow) {
        const int col = k - 1 - lane;              // L_{k, col} = Lg[col][k - col - 1] = Lg[col][lane]
        const T* L = Ls + ((col - r0) * mb + lane) * 4;
        y[2 * col] -= L[0] * x0 + L[2] * x1;
        y[2 * col + 1] -= L[1] * x0 + L[3] * x1;
      }
      __syncthreads();
    }
  }
  for (int q = lane; q < n; q += 64) {
    const int i = q / nyc, j = q - i * nyc;
    const size_t g = ((size_t)j * nxc + i) * S + s;
    x[g] = y[2 * q];
    x[N + g] = y[2 * q + 1];
  }
}

}  // namespace henry
