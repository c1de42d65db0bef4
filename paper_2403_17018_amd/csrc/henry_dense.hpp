// Batched dense LU with partial pivoting of the coarsest multigrid operator (gfx950).
//
// Gaussian elimination on the coarse grid (paper section 2.3), one matrix per sample.
// The 2x2-block 5-point coarse Jacobian is expanded into a dense n x n matrix, n = 2 * cells,
// unknown u = 2 q + component with q = j * nx + i, stored row-major per sample.
//
// Factorisation: one workgroup (16 wavefronts) per sample, blocked right-looking LU with
// partial pivoting, panel width NB.  Each panel of NB columns is factored in LDS (pivot search
// by a fixed-order block reduction, so the pivots are run-to-run deterministic); its row
// interchanges are then applied to every other column (LAPACK form: P A = L U with one
// permutation P); the block row of U is formed by forward substitution with the panel's unit
// lower triangle, and the trailing matrix is updated with the rank-NB product L21 U12 on the
// matrix cores (16x16x4 MFMA, FP64 or FP32 by the operator's precision).  The permutation is
// stored as perm[i] = the original row that ends up in row i.
//
// Solves: one workgroup per sample, right-hand side staged in LDS; forward and backward
// substitution by blocks of DB rows, each block's off-diagonal contribution a coalesced
// sweep over contiguous row segments and its diagonal block solved in LDS.  The transposed
// solve (adjoint) works through columns of the same factors in the axpy form, again reading
// contiguous row segments only.
#pragma once

#include <hip/hip_runtime.h>

namespace henry {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core step acc += a b for one wavefront: lane l supplies a = A[l % 16][l / 16]
// and b = B[l / 16][l % 16]; it holds acc[v] = C[mfma_row<T>(l, v)][l % 16], where the FP64
// instruction spreads a lane's four rows 4 apart and the FP32 one keeps them adjacent
// (both checked on the device).
__device__ __forceinline__ void mfma16x16x4(double a, double b, mf_d4& acc) {
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}
__device__ __forceinline__ void mfma16x16x4(float a, float b, mf_f4& acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}
template <typename T>
__device__ __forceinline__ int mfma_row(int lane, int v) {
  return sizeof(T) == 8 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}
template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  typedef mf_d4 type;
};
template <>
struct MfmaAcc<float> {
  typedef mf_f4 type;
};

constexpr int DENSE_THREADS = 1024;  // factorisation workgroup: 16 wavefronts (one workgroup fills a CU's LDS)
constexpr int DENSE_SOLVE_THREADS = 256;
constexpr int DENSE_CHUNK = 64;   // trailing-update column chunk: 4 MFMA tiles, each taken by 4 wavefronts
constexpr int DENSE_DB = 64;      // row block of the triangular solves

// LDS bytes of the factorisation: the panel (n x NB), the U12 chunk (NB x CHUNK), the
// pivot-search scratch and every pivot of the sample (n).
template <typename T>
__host__ __device__ constexpr size_t dense_factor_lds(int n, int NB) {
  return (size_t)n * NB * sizeof(T) + (size_t)NB * DENSE_CHUNK * sizeof(T) +
         DENSE_THREADS * (sizeof(T) + sizeof(int)) + (size_t)n * sizeof(int);
}
// LDS bytes of a solve: the vector (n) and one diagonal block (DB x DB)
template <typename T>
__host__ __device__ constexpr size_t dense_solve_lds(int n) {
  return (size_t)n * sizeof(T) + (size_t)DENSE_DB * DENSE_DB * sizeof(T);
}

// Dense row-major matrix of one sample from the 2x2-block 5-point operator J [20][cells][S]
// (blocks centre, west, east, south, north).  Block (row r, sample s) per workgroup.
template <typename T>
__global__ void __launch_bounds__(256) k_dense_build(int S, int nxc, int nyc, const T* __restrict__ J,
                                                     T* __restrict__ A) {
  const int r = blockIdx.x, s = blockIdx.y;
  const int nc = nxc * nyc, n = 2 * nc;
  const size_t N = (size_t)nc * S;
  const int q = r >> 1, comp = r & 1;
  const int j = q / nxc, i = q - j * nxc;
  T* row = A + (size_t)s * n * n + (size_t)r * n;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int qc = c >> 1, cc = c & 1;
    int blk = -1;
    if (qc == q) blk = 0;
    else if (qc == q - 1 && i > 0) blk = 1;
    else if (qc == q + 1 && i < nxc - 1) blk = 2;
    else if (qc == q - nxc) blk = 3;
    else if (qc == q + nxc) blk = 4;
    row[c] = blk < 0 ? (T)0 : J[(size_t)(blk * 4 + comp * 2 + cc) * N + (size_t)q * S + s];
  }
}

// Blocked LU with partial pivoting, one workgroup per sample; n % NB == 0 (NB = 16: the
// trailing update works on whole 16 x 16 matrix-core tiles).
template <typename T, int NB>
__global__ void __launch_bounds__(DENSE_THREADS) k_dense_factor(int n, T* __restrict__ LU, int* __restrict__ perm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* P = reinterpret_cast<T*>(smem_raw);                 // panel [n - k0][NB]
  T* Uc = P + (size_t)n * NB;                            // U12 chunk [NB][DENSE_CHUNK]
  T* rv = Uc + NB * DENSE_CHUNK;                         // pivot search values [DENSE_THREADS]
  int* ri = reinterpret_cast<int*>(rv + DENSE_THREADS);  // pivot search rows
  int* pv = ri + DENSE_THREADS;                          // pivots: row k0 + j swapped with k0 + pv[k0 + j]
  const int s = blockIdx.x, t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  T* A = LU + (size_t)s * n * n;
  typedef typename MfmaAcc<T>::type acc_t;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int m = n - k0;
    for (int e = t; e < m * NB; e += DENSE_THREADS) {
      const int r = e / NB, c = e - r * NB;
      P[e] = A[(size_t)(k0 + r) * n + k0 + c];
    }
    __syncthreads();
    for (int j = 0; j < NB; ++j) {
      // pivot: the largest |P[r][j]|, r >= j; ties to the smaller row (fixed-order reduction)
      T best = (T)-1;
      int bi = j;
      for (int r = j + t; r < m; r += DENSE_THREADS) {
        const T v = fabs(P[r * NB + j]);
        if (v > best) {
          best = v;
          bi = r;
        }
      }
      rv[t] = best;
      ri[t] = bi;
      __syncthreads();
      for (int w = DENSE_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) {
          const T a = rv[t], b = rv[t + w];
          if (b > a || (b == a && ri[t + w] < ri[t])) {
            rv[t] = b;
            ri[t] = ri[t + w];
          }
        }
        __syncthreads();
      }
      const int p = ri[0];
      if (t == 0) pv[k0 + j] = p;
      if (p != j && t < NB) {
        const T a = P[j * NB + t];
        P[j * NB + t] = P[p * NB + t];
        P[p * NB + t] = a;
      }
      __syncthreads();
      const T d = P[j * NB + j];
      const T dinv = d != (T)0 ? (T)1 / d : (T)0;   // an exactly singular column leaves L = 0 (the solve then fails visibly)
      for (int r = j + 1 + t; r < m; r += DENSE_THREADS) P[r * NB + j] *= dinv;
      __syncthreads();
      const int w2 = NB - j - 1;
      if (w2 > 0) {
        for (int e = t; e < (m - j - 1) * w2; e += DENSE_THREADS) {
          const int r = j + 1 + e / w2, c = j + 1 + e % w2;
          P[r * NB + c] -= P[r * NB + j] * P[j * NB + c];
        }
      }
      __syncthreads();
    }
    for (int e = t; e < m * NB; e += DENSE_THREADS) {
      const int r = e / NB, c = e - r * NB;
      A[(size_t)(k0 + r) * n + k0 + c] = P[e];
    }
    // the panel's interchanges on every other column: each thread owns its columns, so the
    // sequence of swaps needs no barrier
    for (int c = t; c < n - NB; c += DENSE_THREADS) {
      const int col = c < k0 ? c : c + NB;
      for (int j = 0; j < NB; ++j) {
        const int p = pv[k0 + j];
        if (p != j) {
          T* a = A + (size_t)(k0 + j) * n + col;
          T* b = A + (size_t)(k0 + p) * n + col;
          const T x = *a;
          *a = *b;
          *b = x;
        }
      }
    }
    __syncthreads();
    // trailing columns in chunks: U12 = L11^{-1} A12, then A22 -= L21 U12 on the matrix cores
    for (int cb = k0 + NB; cb < n; cb += DENSE_CHUNK) {
      const int wdt = (n - cb) < DENSE_CHUNK ? (n - cb) : DENSE_CHUNK;
      if (t < wdt) {
        T u[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          T v = A[(size_t)(k0 + i) * n + cb + t];
#pragma unroll
          for (int k = 0; k < i; ++k) v -= P[i * NB + k] * u[k];
          u[i] = v;
          Uc[i * DENSE_CHUNK + t] = v;
          A[(size_t)(k0 + i) * n + cb + t] = v;
        }
      }
      __syncthreads();
      // wavefront w: 16-column tile w % 4 of the chunk, every fourth 16-row tile from w / 4
      const int ct = wave & 3, rg = wave >> 2;
      const int col = cb + 16 * ct;
      if (16 * ct < wdt) {
        for (int r0 = k0 + NB + 16 * rg; r0 < n; r0 += 64) {
          acc_t acc;
          T* Ct = A + (size_t)r0 * n + col + (lane & 15);
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[v] = Ct[(size_t)mfma_row<T>(lane, v) * n];
#pragma unroll
          for (int kk = 0; kk < NB; kk += 4) {
            const T a = -P[(r0 - k0 + (lane & 15)) * NB + kk + (lane >> 4)];
            const T b = Uc[(kk + (lane >> 4)) * DENSE_CHUNK + 16 * ct + (lane & 15)];
            mfma16x16x4(a, b, acc);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) Ct[(size_t)mfma_row<T>(lane, v) * n] = acc[v];
        }
      }
      __syncthreads();
    }
  }
  // the permutation: every interchange, in order, applied to the identity (in LDS, where the
  // panel was), so that row i of L U is row perm[i] of the matrix
  int* pr = reinterpret_cast<int*>(P);
  for (int i = t; i < n; i += DENSE_THREADS) pr[i] = i;
  __syncthreads();
  if (t == 0) {
    for (int k = 0; k < n; ++k) {
      const int p = k - k % NB + pv[k];
      const int a = pr[k];
      pr[k] = pr[p];
      pr[p] = a;
    }
  }
  __syncthreads();
  for (int i = t; i < n; i += DENSE_THREADS) perm[(size_t)s * n + i] = pr[i];
}

// Fixed-order sum over one wavefront (xor butterfly).
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// x = A^{-1} b (TR: x = A^{-T} b) with P A = L U from k_dense_factor, one workgroup per sample.
// b, x: coarse-grid vectors [component][cell][S] (Nc = cells * S), T precision.
template <typename T, bool TR>
__global__ void __launch_bounds__(DENSE_SOLVE_THREADS) k_dense_solve(int S, int nc, const T* __restrict__ LU,
                                                               const int* __restrict__ perm, const T* __restrict__ b,
                                                               T* __restrict__ x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = 2 * nc;
  T* y = reinterpret_cast<T*>(smem_raw);   // [n]
  T* D = y + n;                            // diagonal block [DENSE_DB][DENSE_DB]
  const int s = blockIdx.x, t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const size_t Nc = (size_t)nc * S;
  const T* A = LU + (size_t)s * n * n;
  const int* pr = perm + (size_t)s * n;
  auto at = [&](int u) { return (size_t)(u & 1) * Nc + (size_t)(u >> 1) * S + s; };
  for (int i = t; i < n; i += DENSE_SOLVE_THREADS) y[i] = b[at(TR ? i : pr[i])];
  __syncthreads();
  const int nblk = (n + DENSE_DB - 1) / DENSE_DB;
  auto load_diag = [&](int r0, int db) {
    for (int e = t; e < db * db; e += DENSE_SOLVE_THREADS) {
      const int i = e / db, k = e - i * db;
      D[i * DENSE_DB + k] = A[(size_t)(r0 + i) * n + r0 + k];
    }
  };
  if (!TR) {
    // L y = P b: rows by blocks, the part left of the block as row dot products
    for (int bk = 0; bk < nblk; ++bk) {
      const int r0 = bk * DENSE_DB, db = min(DENSE_DB, n - r0);
      for (int i = wave; i < db; i += DENSE_SOLVE_THREADS / 64) {
        const T* row = A + (size_t)(r0 + i) * n;
        T a = 0;
        for (int k = lane; k < r0; k += 64) a += row[k] * y[k];
        a = wave_sum(a);
        if (lane == 0) y[r0 + i] -= a;
      }
      load_diag(r0, db);
      __syncthreads();
      if (wave == 0) {
        T v = lane < db ? y[r0 + lane] : (T)0;
        for (int k = 0; k < db; ++k) {
          const T vk = __shfl(v, k, 64);
          if (lane > k && lane < db) v -= D[lane * DENSE_DB + k] * vk;
        }
        if (lane < db) y[r0 + lane] = v;
      }
      __syncthreads();
    }
    // U x = y: blocks from the bottom, the part right of the block as row dot products
    for (int bk = nblk - 1; bk >= 0; --bk) {
      const int r0 = bk * DENSE_DB, db = min(DENSE_DB, n - r0), r1 = r0 + db;
      for (int i = wave; i < db; i += DENSE_SOLVE_THREADS / 64) {
        const T* row = A + (size_t)(r0 + i) * n;
        T a = 0;
        for (int k = r1 + lane; k < n; k += 64) a += row[k] * y[k];
        a = wave_sum(a);
        if (lane == 0) y[r0 + i] -= a;
      }
      load_diag(r0, db);
      __syncthreads();
      if (wave == 0) {
        T v = lane < db ? y[r0 + lane] : (T)0;
        for (int k = db - 1; k >= 0; --k) {
          if (lane == k) v /= D[k * DENSE_DB + k];
          const T vk = __shfl(v, k, 64);
          if (lane < k) v -= D[lane * DENSE_DB + k] * vk;
        }
        if (lane < db) y[r0 + lane] = v;
      }
      __syncthreads();
    }
    for (int i = t; i < n; i += DENSE_SOLVE_THREADS) x[at(i)] = y[i];
  } else {
    // U^T z = b: column blocks forward; each finished block updates the later entries with
    // its rows of U (axpy form: contiguous row segments)
    for (int bk = 0; bk < nblk; ++bk) {
      const int c0 = bk * DENSE_DB, db = min(DENSE_DB, n - c0), c1 = c0 + db;
      load_diag(c0, db);
      __syncthreads();
      if (wave == 0) {
        T v = lane < db ? y[c0 + lane] : (T)0;
        for (int k = 0; k < db; ++k) {
          if (lane == k) v /= D[k * DENSE_DB + k];
          const T vk = __shfl(v, k, 64);
          if (lane > k && lane < db) v -= D[k * DENSE_DB + lane] * vk;
        }
        if (lane < db) y[c0 + lane] = v;
      }
      __syncthreads();
      for (int c = c1 + t; c < n; c += DENSE_SOLVE_THREADS) {
        T a = 0;
        for (int r = c0; r < c1; ++r) a += A[(size_t)r * n + c] * y[r];
        y[c] -= a;
      }
      __syncthreads();
    }
    // L^T w = z: column blocks backward, unit diagonal
    for (int bk = nblk - 1; bk >= 0; --bk) {
      const int c0 = bk * DENSE_DB, db = min(DENSE_DB, n - c0), c1 = c0 + db;
      load_diag(c0, db);
      __syncthreads();
      if (wave == 0) {
        T v = lane < db ? y[c0 + lane] : (T)0;
        for (int k = db - 1; k >= 0; --k) {
          const T vk = __shfl(v, k, 64);
          if (lane < k) v -= D[k * DENSE_DB + lane] * vk;
        }
        if (lane < db) y[c0 + lane] = v;
      }
      __syncthreads();
      for (int c = t; c < c0; c += DENSE_SOLVE_THREADS) {
        T a = 0;
        for (int r = c0; r < c1; ++r) a += A[(size_t)r * n + c] * y[r];
        y[c] -= a;
      }
      __syncthreads();
    }
    // x = P^T w
    for (int i = t; i < n; i += DENSE_SOLVE_THREADS) x[at(pr[i])] = y[i];
  }
}

}  // namespace henry
