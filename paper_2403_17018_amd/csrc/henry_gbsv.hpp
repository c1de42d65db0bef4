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
// Factor storage per sample: U by rows [n][GB_C] (row j: U(j, j .. j + kl + ku), diagonal
// first), U by columns [n][GB_C] (column j: U(j - d, j) for d = 0 .. kl + ku), then L [n][kl]
// (column j: the multipliers of rows j + 1 .. j + kl after step j's interchange); piv [n]:
// step j exchanged rows j and j + piv[j].
__host__ __device__ inline int gb_kl(int nyc) { return 2 * nyc + 1; }
__host__ __device__ inline int gb_cols(int nyc) { return 2 * gb_kl(nyc) + 1; }
__host__ __device__ inline size_t gb_stride(int nxc, int nyc) {
  const size_t n = 2 * (size_t)nxc * nyc;
  return n * (2 * gb_cols(nyc) + gb_kl(nyc));
}
constexpr int GB_THREADS = 256;
constexpr int GB_PF = 16;       // entering rows of the factorisation staged per chunk
constexpr int GB_CH = 16;       // steps of a triangular solve staged per chunk
constexpr int GB_CMAX = 79;     // widest band row the register staging holds (kl <= 39)
constexpr int GB_UPD = 12;      // trailing-update elements per thread: kl * 2 kl <= GB_THREADS * GB_UPD
template <typename T>
__host__ __device__ inline size_t gb_factor_lds(int nyc) {
  const int kl = gb_kl(nyc), C = gb_cols(nyc);
  return ((size_t)(kl + 2) * (C + 1) + (size_t)GB_PF * C + C) * sizeof(T) + 16;
}
template <typename T>
__host__ __device__ inline size_t gb_solve_lds(int nxc, int nyc) {
  return (2 * (size_t)nxc * nyc + 2 * (size_t)GB_CH * gb_cols(nyc)) * sizeof(T) + 2 * GB_CH * sizeof(int);
}

// Barrier for LDS traffic only: this wavefront's LDS operations complete, then every wavefront
// of the workgroup arrives.  Unlike __syncthreads() it does not wait for global loads and stores
// in flight (prefetches for later steps, factor output nobody in the kernel reads back), which
// would put a memory latency on every step.  The memory clobber keeps the compiler from moving
// memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

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
// in a circular buffer one row and one column larger than the window, so that in each step the
// row entering (j + kl + 1) and the column entering (j + kl + ku + 1, zero above the entering
// row) land in the slots of row and column j - 1, which nothing reads any more.  Two barriers
// per step: wavefront 0 finds the pivot and copies its row aside (the row of U, written out
// by rows and by columns); then every thread updates the trailing window as if rows j and
// j + p had been exchanged (row j + p takes row j's old values; no row is moved), computes
// its multiplier with the reciprocal of the pivot, and the entering row and column are
// written.  The entering rows come from the matrix GB_PF steps ahead: loaded into registers
// one chunk early, stored to LDS at the chunk's start.
// Launch: grid S, block GB_THREADS, dynamic LDS gb_factor_lds<T>(nyc); needs kl + 1 <= 64.
template <typename T>
__global__ void __launch_bounds__(GB_THREADS) k_gb_factor(int S, int nxc, int nyc, const T* __restrict__ J,
                                                          T* __restrict__ LU, int* __restrict__ piv) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = 2 * nxc * nyc, kl = gb_kl(nyc), R = kl + 1, C = gb_cols(nyc), ku2 = C - 1;
  const int RR = R + 1, CC = C + 1;
  T* W = reinterpret_cast<T*>(smem_raw);   // [RR][CC] window
  T* Ws = W + (size_t)RR * CC;               // [GB_PF][C] entering rows of this chunk
  T* prow = Ws + (size_t)GB_PF * C;          // [C] pivot row of this step
  int& sp = *reinterpret_cast<int*>(prow + C);   // the step's pivot offset (inside the aligned dynamic
                                                 // region: a static variable before it would misalign
                                                 // every 8-byte window access)
  const int s = blockIdx.x, t = threadIdx.x;
  const size_t N = (size_t)nxc * nyc * S;
  T* Ug = LU + (size_t)s * gb_stride(nxc, nyc);
  T* Ucg = Ug + (size_t)n * C;
  T* Lg = Ucg + (size_t)n * C;
  int* pg = piv + (size_t)s * n;
  constexpr int NPF = (GB_PF * GB_CMAX + GB_THREADS - 1) / GB_THREADS;
  T pf[NPF];
  auto fetch = [&](int j0) {   // entering rows of steps j0 .. j0 + GB_PF - 1 (zero beyond n)
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int e = t + k * GB_THREADS;
      if (e < GB_PF * C) {
        const int q = e / C, c = e - q * C;
        pf[k] = gb_entry<T>(J, N, S, s, nxc, nyc, j0 + R + q, j0 + q + 1 + c);
      }
    }
  };
  for (int e = t; e < R * C; e += GB_THREADS) {
    const int r = e / C, c = e - r * C;
    W[r * CC + c] = (c - r <= kl && r - c <= kl) ? gb_entry<T>(J, N, S, s, nxc, nyc, r, c) : (T)0;
  }
  // This thread's elements of the trailing update, (row j + 1 + ui, column j + uc), fixed for
  // the whole factorisation; their slots advance by one row and one column per step.
  int ui[GB_UPD], uc[GB_UPD], urs[GB_UPD], ucs[GB_UPD];
#pragma unroll
  for (int k = 0; k < GB_UPD; ++k) {
    const int e = t + k * GB_THREADS;
    ui[k] = e < kl * ku2 ? e / ku2 : kl;   // kl: never updated
    uc[k] = e < kl * ku2 ? 1 + (e - (e / ku2) * ku2) : 1;
    urs[k] = (1 + ui[k]) % RR;
    ucs[k] = uc[k] % CC;
  }
  auto wrapR = [&](int a) { return a >= RR ? a - RR : a; };
  auto wrapC = [&](int a) { return a >= CC ? a - CC : a; };
  fetch(0);
  lds_barrier();
  int rj = 0, cj = 0;   // slots of row j and column j
  for (int j = 0; j < n; ++j) {
    if (j % GB_PF == 0) {   // the previous chunk's last reads of Ws ended at the last barrier
#pragma unroll
      for (int k = 0; k < NPF; ++k) {
        const int e = t + k * GB_THREADS;
        if (e < GB_PF * C) Ws[e] = pf[k];
      }
      fetch(j + GB_PF);
    }
    const int km = (n - 1 - j) < kl ? (n - 1 - j) : kl;
    if (t < 64) {   // pivot: first row of largest magnitude (wave reduction, lowest index on ties)
      T v = t <= km ? fabs(W[wrapR(rj + t) * CC + cj]) : (T)-1;
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
      const int p = __shfl(idx, 0);
      const T* pr = W + wrapR(rj + p) * CC;
      for (int c = t; c < C; c += 64) {
        const T u = pr[wrapC(cj + c)];
        prow[c] = u;
        Ug[(size_t)j * C + c] = u;
        if (j + c < n) Ucg[(size_t)(j + c) * C + c] = u;
      }
      if (t == 0) {
        sp = p;
        pg[j] = p;
      }
    }
    lds_barrier();
    const int p = sp;
    const T rp = (T)1 / prow[0];
#pragma unroll
    for (int k = 0; k < GB_UPD; ++k) {   // rank-1 update of the trailing window
      if (ui[k] < km) {
        const bool moved = ui[k] + 1 == p;   // row j + p now holds row j's old values
        const int rs = moved ? rj : urs[k];
        const T l = W[rs * CC + cj] * rp;
        const T base = W[rs * CC + ucs[k]];
        W[urs[k] * CC + ucs[k]] = base - l * prow[uc[k]];
        if (uc[k] == 1) Lg[(size_t)j * kl + ui[k]] = l;
      }
      urs[k] = urs[k] + 1 == RR ? 0 : urs[k] + 1;
      ucs[k] = ucs[k] + 1 == CC ? 0 : ucs[k] + 1;
    }
    // row j + kl + 1 enters the slot of row j - 1, column j + kl + ku + 1 that of column j - 1
    const T* wsr = Ws + (size_t)(j % GB_PF) * C;
    T* er = W + (rj == 0 ? RR - 1 : rj - 1) * CC;
    for (int c = t; c < C; c += GB_THREADS) er[wrapC(cj + 1 + c)] = wsr[c];
    const int ec = cj == 0 ? CC - 1 : cj - 1;
    for (int i = t; i < kl; i += GB_THREADS) W[wrapR(rj + 1 + i) * CC + ec] = (T)0;
    rj = rj + 1 == RR ? 0 : rj + 1;
    cj = cj + 1 == CC ? 0 : cj + 1;
    lds_barrier();
  }
}

// x = A^{-1} b (TR = false) or A^{-T} b (TR = true) with the factors of k_gb_factor, one wavefront
// per sample; the right-hand side lives in LDS, the factor data of GB_CH steps at a time is
// loaded into registers one chunk ahead and stored to the LDS buffer the next chunk reads.
//   A = P_0 L_0 P_1 L_1 ... P_{n-1} L_{n-1} U  (P_j: the interchange of step j, L_j: its multipliers)
//   A x = b:    for j up: interchange, y_{j+i} -= l_j[i] y_j;   then for j down (U by columns):
//               x_j = y_j / u_jj, y_{j-d} -= U(j-d, j) x_j
//   A^T x = b:  for j up (U by rows): z_j = y_j / u_jj, y_{j+d} -= U(j, j+d) z_j;   then for j
//               down: z_j -= sum_i l_j[i] z_{j+i}, interchange
// Every step is one barrier; no lane reads in a step what another lane writes in it.
// Launch: grid S, block 64, dynamic LDS gb_solve_lds<T>(nxc, nyc).
template <typename T, bool TR>
__global__ void __launch_bounds__(64) k_gb_solve(int S, int nxc, int nyc, const T* __restrict__ LU,
                                                 const int* __restrict__ piv, const T* __restrict__ b,
                                                 T* __restrict__ x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int s = blockIdx.x, lane = threadIdx.x;
  const int nc = nxc * nyc, n = 2 * nc, kl = gb_kl(nyc), C = gb_cols(nyc), ku2 = C - 1;
  T* y = reinterpret_cast<T*>(smem_raw);
  // two staging buffers, addressed from the LDS base (a pointer picked from an array would lose
  // its address space and turn every access into a flat access that also waits for memory)
  T* const buf0 = y + n;
  int* const pbuf0 = reinterpret_cast<int*>(y + n + 2 * (size_t)GB_CH * C);
  auto buf = [&](int k) { return buf0 + (size_t)(k & 1) * GB_CH * C; };
  auto pbuf = [&](int k) { return pbuf0 + (k & 1) * GB_CH; };
  const size_t N = (size_t)nc * S;
  const T* Ug = LU + (size_t)s * gb_stride(nxc, nyc);
  const T* Ucg = Ug + (size_t)n * C;
  const T* Lg = Ucg + (size_t)n * C;
  const int* pg = piv + (size_t)s * n;
  for (int q = lane; q < nc; q += 64) {
    const int i = q / nyc, j = q - i * nyc;
    const size_t g = ((size_t)j * nxc + i) * S + s;
    y[2 * q] = b[g];
    y[2 * q + 1] = b[N + g];
  }
  constexpr int NR = (GB_CH * GB_CMAX + 63) / 64;
  T reg[NR];
  int preg = 0;
  const int nch = (n + GB_CH - 1) / GB_CH;
  // chunk k of a pass: steps [j0, j1), counted from the bottom (up) or the top (down)
  auto bounds = [&](int k, bool up, int& j0, int& j1) {
    if (up) {
      j0 = k * GB_CH;
      j1 = j0 + GB_CH < n ? j0 + GB_CH : n;
    } else {
      j1 = n - k * GB_CH;
      j0 = j1 - GB_CH > 0 ? j1 - GB_CH : 0;
    }
  };
  // Loads are unconditional (clamped to the chunk's last value) so that each register stays
  // live from its load to its store and is never reused, which would make a step wait for it.
  auto fetch = [&](const T* src, int width, bool pivots, int k, bool up) {
    int j0, j1;
    bounds(k, up, j0, j1);
    const int last = (j1 - j0) * width - 1;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int e = lane + 64 * r;
      reg[r] = src[(size_t)j0 * width + (e < last ? e : last)];
    }
    if (pivots) preg = pg[j0 + (lane < j1 - j0 ? lane : j1 - j0 - 1)];
  };
  auto store = [&](int k, int width, bool pivots, bool up) {
    int j0, j1;
    bounds(k, up, j0, j1);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int e = lane + 64 * r;
      if (e < (j1 - j0) * width) buf(k)[e] = reg[r];
    }
    if (pivots && lane < j1 - j0) pbuf(k)[lane] = preg;
  };
  // one pass over all chunks; step(j, data of step j, its pivot)
  auto pass = [&](const T* src, int width, bool pivots, bool up, auto&& step) {
    fetch(src, width, pivots, 0, up);
    store(0, width, pivots, up);
    lds_barrier();
    if (nch > 1) fetch(src, width, pivots, 1, up);
    for (int k = 0; k < nch; ++k) {
      int j0, j1;
      bounds(k, up, j0, j1);
      const T* cur = buf(k);
      const int* pc = pbuf(k);
      if (up)
        for (int j = j0; j < j1; ++j) step(j, cur + (size_t)(j - j0) * width, pivots ? pc[j - j0] : 0);
      else
        for (int j = j1 - 1; j >= j0; --j) step(j, cur + (size_t)(j - j0) * width, pivots ? pc[j - j0] : 0);
      if (k + 1 < nch) store(k + 1, width, pivots, up);   // buffer (k+1)&1 was last read by chunk k-1
      lds_barrier();
      if (k + 2 < nch) fetch(src, width, pivots, k + 2, up);
    }
  };
  if (!TR) {
    pass(Lg, kl, true, true, [&](int j, const T* l, int p) {
      const int km = (n - 1 - j) < kl ? (n - 1 - j) : kl;
      const T yj = y[j], yp = y[j + p];   // after the interchange y_j = yp, y_{j+p} = yj
      const int i = lane + 1;
      if (i <= km) y[j + i] = (i == p ? yj : y[j + i]) - l[lane] * yp;
      if (lane == 0) y[j] = yp;
      lds_barrier();
    });
    pass(Ucg, C, false, false, [&](int j, const T* u, int) {
      const T xj = y[j] / u[0];
      const int m = j < ku2 ? j : ku2;
      for (int d = lane + 1; d <= m; d += 64) y[j - d] -= u[d] * xj;
      if (lane == 0) y[j] = xj;
      lds_barrier();
    });
  } else {
    pass(Ug, C, false, true, [&](int j, const T* u, int) {
      const T zj = y[j] / u[0];
      const int m = (n - 1 - j) < ku2 ? (n - 1 - j) : ku2;
      for (int d = lane + 1; d <= m; d += 64) y[j + d] -= u[d] * zj;
      if (lane == 0) y[j] = zj;
      lds_barrier();
    });
    pass(Lg, kl, true, false, [&](int j, const T* l, int p) {
      const int km = (n - 1 - j) < kl ? (n - 1 - j) : kl;
      T acc = lane < km ? l[lane] * y[j + 1 + lane] : (T)0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      const T zj = y[j] - acc, zp = y[j + p];
      if (lane == 0) {
        y[j] = zp;   // interchange after the update (p = 0 leaves zj in place)
        y[j + p] = zj;
      }
      lds_barrier();
    });
  }
  for (int q = lane; q < nc; q += 64) {
    const int i = q / nyc, j = q - i * nyc;
    const size_t g = ((size_t)j * nxc + i) * S + s;
    x[g] = y[2 * q];
    x[N + g] = y[2 * q + 1];
  }
}

}  // namespace henry
