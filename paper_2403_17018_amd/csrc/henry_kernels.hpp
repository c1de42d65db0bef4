// HIP kernels of the batched Henry solve for gfx950 (MI355X).
//
// Data layout ("SoA by sample"): every per-cell quantity is its own array indexed
// [cell][s] = (j*nx + i)*S + s, sample fastest.  A wavefront therefore reads 64
// consecutive samples of one cell (or, for S < 64, several whole cells), so every
// field access is a contiguous, coalesced load for any batch size S.  Two-component
// vectors (p, c) are [comp][cell][s]; the 2x2-block 5-point Jacobian is 20 arrays
// [blk*4 + row*2 + col][cell][s] with blk = centre, west, east, south, north.
//
// Thread map: blockDim = (SX, CY) with SX = min(S, 64) samples by CY = 256/SX cells;
// the 1-D grid enumerates (sample block, cell block) pairs.  Kernels that feed a
// per-sample reduction loop over CPT cells per thread and reduce over the CY rows
// of the block in LDS in a fixed order, so every FP64 sum is run-to-run deterministic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace henry {

struct Map {
  int S;    // samples in the batch
  int SX;   // blockDim.x
  int CY;   // blockDim.y
  int nsb;  // number of sample blocks
  int CPT;  // cells per thread (reduction kernels)
  int ncb;  // number of cell blocks
};

struct Grid2 {
  int nx, ny, ncell;
};

// Physical constants and mesh spacing of one grid.
struct Phys {
  double rho0, drho, rho1, mu, g, Dm, c_left;
  double hx, hy, vol, tau, Ly, Lx;
  int right_dir;
};

// Analytic KL modes: e_k(x,y) = fx_k(x) fy_k(y), fx = cos or sin of w (x - centre), normalised.
struct KLModes {
  int n;
  double sqrt_lam[8];
  double wx[8], wy[8], normx[8], normy[8];
  int oddx[8], oddy[8];
  double xc, yc;
};

struct FieldParams {
  double phi_mean, phi_amp, phi_min, phi_max, lnK_mean, logK_amp, q_in, q_in_amp;
  int n_phi, n_logK;
};

__device__ __forceinline__ bool map_cell(const Map& m, int ncell, int& s, int& cell, int& sblk, int& cblk) {
  const int bid = blockIdx.x;
  sblk = bid % m.nsb;
  cblk = bid / m.nsb;
  s = sblk * m.SX + (int)threadIdx.x;
  cell = cblk * m.CY + (int)threadIdx.y;
  return s < m.S && cell < ncell;
}

// --------------------------------------------------------------------------
// Block reduction over threadIdx.y for each threadIdx.x (fixed order).
template <int NV>
__device__ __forceinline__ void block_sum_y(double (&v)[NV], double* lds /* [NV][CY][SX] */) {
  const int tx = threadIdx.x, ty = threadIdx.y, SX = blockDim.x, CY = blockDim.y;
  __syncthreads();   // lds may still be read by a previous reduction
#pragma unroll
  for (int q = 0; q < NV; ++q) lds[(q * CY + ty) * SX + tx] = v[q];
  __syncthreads();
  for (int w = 1; w < CY; w <<= 1) {
    if ((ty % (2 * w)) == 0 && ty + w < CY) {
#pragma unroll
      for (int q = 0; q < NV; ++q) lds[(q * CY + ty) * SX + tx] += lds[(q * CY + ty + w) * SX + tx];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = lds[(q * CY) * SX + tx];
}

template <int NV>
__device__ __forceinline__ void block_max_y(double (&v)[NV], double* lds) {
  const int tx = threadIdx.x, ty = threadIdx.y, SX = blockDim.x, CY = blockDim.y;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) lds[(q * CY + ty) * SX + tx] = v[q];
  __syncthreads();
  for (int w = 1; w < CY; w <<= 1) {
    if ((ty % (2 * w)) == 0 && ty + w < CY) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        double a = lds[(q * CY + ty) * SX + tx], b = lds[(q * CY + ty + w) * SX + tx];
        lds[(q * CY + ty) * SX + tx] = (b > a || b != b) ? b : a;   // NaN propagates
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = lds[(q * CY) * SX + tx];
}

// ==========================================================================
// a1: random fields at cell centres
// ==========================================================================
__device__ __forceinline__ double kl_1d(double w, int odd, double nrm, double t) {
  double a = w * t;
  return (odd ? sin(a) : cos(a)) / nrm;
}

__global__ void k_fields(Map m, Grid2 G, Phys P, KLModes kl, FieldParams fp, const double* __restrict__ theta,
                         double* __restrict__ phi, double* __restrict__ K, double* __restrict__ uin) {
  int s, cell, sb, cb;
  if (!map_cell(m, G.ncell, s, cell, sb, cb)) return;
  const int j = cell / G.nx, i = cell - j * G.nx;
  const double x = (i + 0.5) * P.hx;
  const double y = -P.Ly + (j + 0.5) * P.hy;
  const double* th = theta + (size_t)s * 13;
  double sp = 0.0, sk = 0.0;
  for (int k = 0; k < kl.n; ++k) {
    const double e = kl_1d(kl.wx[k], kl.oddx[k], kl.normx[k], x - kl.xc) *
                     kl_1d(kl.wy[k], kl.oddy[k], kl.normy[k], y - kl.yc);
    if (k < fp.n_phi) sp += kl.sqrt_lam[k] * th[k] * e;
    if (k < fp.n_logK) sk += kl.sqrt_lam[k] * th[4 + k] * e;
  }
  const size_t id = (size_t)cell * m.S + s;
  if (phi) phi[id] = fmin(fmax(fp.phi_mean * (1.0 + fp.phi_amp * sp), fp.phi_min), fp.phi_max);
  if (K) K[id] = exp(fp.lnK_mean + fp.logK_amp * sk);
  if (uin && cell == 0) uin[s] = fp.q_in * (1.0 + fp.q_in_amp * th[12]);
}

// Initial state: c = 0, p = -rho0 g y (first Newton guess only).
__global__ void k_init_state(Map m, Grid2 G, Phys P, double* __restrict__ p, double* __restrict__ c) {
  int s, cell, sb, cb;
  if (!map_cell(m, G.ncell, s, cell, sb, cb)) return;
  const int j = cell / G.nx;
  const size_t id = (size_t)cell * m.S + s;
  p[id] = -P.rho0 * P.g * (-P.Ly + (j + 0.5) * P.hy);
  c[id] = 0.0;
}

// ==========================================================================
// a2: residual and 2x2-block Jacobian assembly (upwinded two-point fluxes)
// ==========================================================================
// Flux through an interior face in canonical orientation, from L (west/south cell)
// to H (east/north cell), with its derivatives.
struct FaceFlux {
  double F, G;         // fluid and salt mass flux L -> H
  double a;            // dF/dp_L = -dF/dp_H
  double bF;           // dF/dc_L = dF/dc_H
  double dGL, dGH;     // dG/dc_L, dG/dc_H   (dG/dp_* = +-a * cup)
  double cup;
};

__device__ __forceinline__ void face_flux(const Phys& P, bool north, double pL, double cL, double phL, double KL,
                                          double pH, double cH, double phH, double KH, FaceFlux& o) {
  const double d = north ? P.hy : P.hx;
  const double A = north ? P.hx : P.hy;
  const double w = A / d;
  const double Kf = 2.0 * KL * KH / (KL + KH);
  const double rf = 0.5 * ((P.rho0 + P.drho * cL) + (P.rho0 + P.drho * cH));
  const double phif = 0.5 * (phL + phH);
  const double km = Kf / P.mu;
  const double grav = north ? rf * P.g : 0.0;
  const double u = -km * ((pH - pL) / d + grav);
  const double F = rf * u * A;
  const bool upL = F >= 0.0;
  const double cup = upL ? cL : cH;
  const double dc = cH - cL;
  const double dif = rf * phif * P.Dm * w;
  o.F = F;
  o.G = F * cup - dif * dc;
  o.a = rf * km * w;
  const double dudc = north ? -km * P.g * 0.5 * P.drho : 0.0;
  o.bF = 0.5 * P.drho * u * A + rf * A * dudc;
  const double t1 = 0.5 * P.drho * phif * P.Dm * dc * w;
  o.dGL = o.bF * cup + (upL ? F : 0.0) - (t1 - dif);
  o.dGH = o.bF * cup + (upL ? 0.0 : F) - (t1 + dif);
  o.cup = cup;
}

// J block order: 0 centre, 1 west, 2 east, 3 south, 4 north.
template <bool WRITE_R, typename TJ, bool WRITE_J32>
__global__ void __launch_bounds__(256) k_assemble(Map m, Grid2 G, Phys P, const double* __restrict__ p,
                                                  const double* __restrict__ c, const double* __restrict__ c_old,
                                                  const double* __restrict__ phi, const double* __restrict__ K,
                                                  const double* __restrict__ uin, double* __restrict__ R,
                                                  TJ* __restrict__ J, float* __restrict__ J32) {
  int s, cell, sb, cb;
  if (!map_cell(m, G.ncell, s, cell, sb, cb)) return;
  const int S = m.S;
  const size_t N = (size_t)G.ncell * S;
  const int j = cell / G.nx, i = cell - j * G.nx;
  const size_t id = (size_t)cell * S + s;
  const double pP = p[id], cP = c[id], phP = phi[id], KP = K[id];
  const double rP = P.rho0 + P.drho * cP;
  double Rp = 0.0, Rc = 0.0;
  double D[4];
  double NB[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int e = 0; e < 4; ++e) NB[q][e] = 0.0;
  }
  if (WRITE_R) {
    const double co = c_old[id];
    const double ro = P.rho0 + P.drho * co;
    Rp = P.vol * phP * (rP - ro) / P.tau;
    Rc = P.vol * phP * (rP * cP - ro * co) / P.tau;
  }
  D[0] = 0.0;
  D[1] = P.vol * phP * P.drho / P.tau;
  D[2] = 0.0;
  D[3] = P.vol * phP * (P.rho0 + 2.0 * P.drho * cP) / P.tau;

  FaceFlux f;
  // west face: P is the high side
  if (i > 0) {
    const size_t q = id - S;
    face_flux(P, false, p[q], c[q], phi[q], K[q], pP, cP, phP, KP, f);
    Rp -= f.F; Rc -= f.G;
    D[0] += f.a; D[1] -= f.bF; D[2] += f.a * f.cup; D[3] -= f.dGH;
    NB[0][0] = -f.a; NB[0][1] = -f.bF; NB[0][2] = -f.a * f.cup; NB[0][3] = -f.dGL;
  }
  // east face: P is the low side
  if (i < G.nx - 1) {
    const size_t q = id + S;
    face_flux(P, false, pP, cP, phP, KP, p[q], c[q], phi[q], K[q], f);
    Rp += f.F; Rc += f.G;
    D[0] += f.a; D[1] += f.bF; D[2] += f.a * f.cup; D[3] += f.dGL;
    NB[1][0] = -f.a; NB[1][1] = f.bF; NB[1][2] = -f.a * f.cup; NB[1][3] = f.dGH;
  }
  // south face
  if (j > 0) {
    const size_t q = id - (size_t)G.nx * S;
    face_flux(P, true, p[q], c[q], phi[q], K[q], pP, cP, phP, KP, f);
    Rp -= f.F; Rc -= f.G;
    D[0] += f.a; D[1] -= f.bF; D[2] += f.a * f.cup; D[3] -= f.dGH;
    NB[2][0] = -f.a; NB[2][1] = -f.bF; NB[2][2] = -f.a * f.cup; NB[2][3] = -f.dGL;
  }
  // north face
  if (j < G.ny - 1) {
    const size_t q = id + (size_t)G.nx * S;
    face_flux(P, true, pP, cP, phP, KP, p[q], c[q], phi[q], K[q], f);
    Rp += f.F; Rc += f.G;
    D[0] += f.a; D[1] += f.bF; D[2] += f.a * f.cup; D[3] += f.dGL;
    NB[3][0] = -f.a; NB[3][1] = f.bF; NB[3][2] = -f.a * f.cup; NB[3][3] = f.dGH;
  }
  const double wb = P.hy / P.hx;
  // left boundary: prescribed inflow at c_left, diffusive Dirichlet c_left
  if (i == 0) {
    const double F = -(P.rho0 + P.drho * P.c_left) * uin[s] * P.hy;
    Rp += F;
    Rc += F * P.c_left + 2.0 * rP * phP * P.Dm * (cP - P.c_left) * wb;
    D[3] += 2.0 * phP * P.Dm * wb * (P.drho * (cP - P.c_left) + rP);
  }
  // right boundary: hydrostatic seawater pressure; inflow carries rho1 and c = 1
  if (i == G.nx - 1) {
    const double y = -P.Ly + (j + 0.5) * P.hy;
    const double pb = -P.rho1 * P.g * y;
    const double u = -(KP / P.mu) * (pb - pP) / (0.5 * P.hx);
    const bool inflow = u < 0.0;
    const double rb = inflow ? P.rho1 : rP;
    const double F = rb * u * P.hy;
    const double cb = inflow ? 1.0 : cP;
    Rp += F;
    Rc += F * cb;
    const double dFdp = rb * P.hy * (2.0 * KP / (P.mu * P.hx));
    const double dFdc = inflow ? 0.0 : P.drho * u * P.hy;
    D[0] += dFdp;
    D[1] += dFdc;
    D[2] += cb * dFdp;
    D[3] += cb * dFdc + (inflow ? 0.0 : F);
    if (P.right_dir) {
      Rc += 2.0 * rP * phP * P.Dm * (cP - 1.0) * wb;
      D[3] += 2.0 * phP * P.Dm * wb * (P.drho * (cP - 1.0) + rP);
    }
  }
  if (WRITE_R) {
    R[id] = Rp;
    R[N + id] = Rc;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) J[e * N + id] = (TJ)D[e];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int e = 0; e < 4; ++e) J[((q + 1) * 4 + e) * N + id] = (TJ)NB[q][e];
  }
  if (WRITE_J32) {
#pragma unroll
    for (int e = 0; e < 4; ++e) J32[e * N + id] = (float)D[e];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int e = 0; e < 4; ++e) J32[((q + 1) * 4 + e) * N + id] = (float)NB[q][e];
    }
  }
}

// ==========================================================================
// a4/a5: block stencil operations (SpMV, red-black block Gauss-Seidel, transfers)
// ==========================================================================
// (A x)_P for one cell-sample: centre block + the 4 neighbour blocks that exist.
// TR: (A^T x)_P, gathering the transposed blocks A_{Q,P} stored in the neighbours'
// rows (Q east of P holds A_{Q,P} in its west slot, and so on), so no atomics.
template <typename T, typename TA, bool TR = false>
__device__ __forceinline__ void apply_row(const T* __restrict__ J, const T* __restrict__ x, size_t N, size_t id, int i,
                                          int j, int nx, int ny, int S, TA& y0, TA& y1, bool skip_centre) {
  TA a0 = 0, a1 = 0;
  // block at (slot, row q): y += B x_q or B^T x_q
  auto acc = [&](int slot, size_t q, size_t xq) {
    const TA x0 = x[xq], x1 = x[N + xq];
    const TA b0 = (TA)J[(slot * 4 + 0) * N + q], b1 = (TA)J[(slot * 4 + 1) * N + q];
    const TA b2 = (TA)J[(slot * 4 + 2) * N + q], b3 = (TA)J[(slot * 4 + 3) * N + q];
    if (TR) {
      a0 += b0 * x0 + b2 * x1;
      a1 += b1 * x0 + b3 * x1;
    } else {
      a0 += b0 * x0 + b1 * x1;
      a1 += b2 * x0 + b3 * x1;
    }
  };
  if (!skip_centre) acc(0, id, id);
  const size_t row = (size_t)nx * S;
  if (i > 0) acc(TR ? 2 : 1, TR ? id - S : id, id - S);
  if (i < nx - 1) acc(TR ? 1 : 2, TR ? id + S : id, id + S);
  if (j > 0) acc(TR ? 4 : 3, TR ? id - row : id, id - row);
  if (j < ny - 1) acc(TR ? 3 : 4, TR ? id + row : id, id + row);
  y0 = a0;
  y1 = a1;
}

// One colour of a red-black 2x2-block Gauss-Seidel sweep: x_P = D_P^{-1}(b_P - sum_nb A_nb x_nb)
// for every cell with (i + j) % 2 == colour.  x_zero: x is zero on entry (first pass
// of a V-cycle level), so neighbours are not read.
template <typename T, bool TR = false>
__global__ void __launch_bounds__(256) k_gs_colour(Map m, Grid2 G, int colour, int x_zero, const T* __restrict__ J,
                                                   const T* __restrict__ b, T* __restrict__ x) {
  int s, mc, sb, cb;
  const int half = (G.nx + 1) >> 1;
  if (!map_cell(m, G.ny * half, s, mc, sb, cb)) return;
  const int j = mc / half;
  const int i = 2 * (mc - j * half) + ((j + colour) & 1);
  if (i >= G.nx) return;
  const int S = m.S;
  const size_t N = (size_t)G.ncell * S;
  const size_t id = ((size_t)j * G.nx + i) * S + s;
  T r0 = b[id], r1 = b[N + id];
  if (!x_zero) {
    T a0, a1;
    apply_row<T, T, TR>(J, x, N, id, i, j, G.nx, G.ny, S, a0, a1, true);
    r0 -= a0;
    r1 -= a1;
  }
  const T d00 = J[id], d11 = J[3 * N + id];
  const T d01 = TR ? J[2 * N + id] : J[N + id], d10 = TR ? J[N + id] : J[2 * N + id];
  const T det = d00 * d11 - d01 * d10;
  x[id] = (d11 * r0 - d01 * r1) / det;
  x[N + id] = (d00 * r1 - d10 * r0) / det;
}

// Fused residual and restriction: b_H(I,J) = sum over the 2x2 children of (b - A x).
// red_only: the last smoothing pass was the black one, which leaves a zero residual
// on black cells, so only the two red children are evaluated.
template <typename T, bool TR = false>
__global__ void __launch_bounds__(256) k_residual_restrict(Map m, Grid2 Gf, Grid2 Gc, int red_only,
                                                           const T* __restrict__ J, const T* __restrict__ b,
                                                           const T* __restrict__ x, T* __restrict__ bH) {
  int s, cc, sb, cb;
  if (!map_cell(m, Gc.ncell, s, cc, sb, cb)) return;
  const int S = m.S;
  const size_t Nf = (size_t)Gf.ncell * S, Nc = (size_t)Gc.ncell * S;
  const int Jc = cc / Gc.nx, Ic = cc - Jc * Gc.nx;
  T s0 = 0, s1 = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 2 * Ic + (q & 1), j = 2 * Jc + (q >> 1);
    if (red_only && ((i + j) & 1)) continue;
    const size_t id = ((size_t)j * Gf.nx + i) * S + s;
    T a0, a1;
    apply_row<T, T, TR>(J, x, Nf, id, i, j, Gf.nx, Gf.ny, S, a0, a1, false);
    s0 += b[id] - a0;
    s1 += b[Nf + id] - a1;
  }
  const size_t idc = (size_t)cc * S + s;
  bH[idc] = s0;
  bH[Nc + idc] = s1;
}

// Bilinear cell-centred prolongation (weights 9/16, 3/16, 3/16, 1/16; missing
// neighbours at the boundary replaced by the cell itself) and correction x += P e.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong_correct(Map m, Grid2 Gf, Grid2 Gc, const T* __restrict__ e,
                                                         T* __restrict__ x) {
  int s, cell, sb, cb;
  if (!map_cell(m, Gf.ncell, s, cell, sb, cb)) return;
  const int S = m.S;
  const size_t Nf = (size_t)Gf.ncell * S, Nc = (size_t)Gc.ncell * S;
  const int j = cell / Gf.nx, i = cell - j * Gf.nx;
  const int I = i >> 1, Jc = j >> 1;
  int I2 = I + ((i & 1) ? 1 : -1), J2 = Jc + ((j & 1) ? 1 : -1);
  I2 = I2 < 0 ? 0 : (I2 >= Gc.nx ? Gc.nx - 1 : I2);
  J2 = J2 < 0 ? 0 : (J2 >= Gc.ny ? Gc.ny - 1 : J2);
  const size_t c00 = ((size_t)Jc * Gc.nx + I) * S + s, c10 = ((size_t)Jc * Gc.nx + I2) * S + s;
  const size_t c01 = ((size_t)J2 * Gc.nx + I) * S + s, c11 = ((size_t)J2 * Gc.nx + I2) * S + s;
  const size_t id = (size_t)cell * S + s;
  const T w9 = (T)0.5625, w3 = (T)0.1875, w1 = (T)0.0625;
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
    const size_t o = comp * Nc;
    const T v = w9 * e[o + c00] + w3 * e[o + c10] + w3 * e[o + c01] + w1 * e[o + c11];
    x[comp * Nf + id] += v;
  }
}

// Restriction of state and coefficients for rediscretised coarse Jacobians:
// p, c, phi arithmetic means of the 4 children; K geometric mean (mean of log K).
__global__ void k_restrict_state(Map m, Grid2 Gf, Grid2 Gc, const double* __restrict__ pf,
                                 const double* __restrict__ cf, double* __restrict__ pc, double* __restrict__ cc) {
  int s, cell, sb, cb;
  if (!map_cell(m, Gc.ncell, s, cell, sb, cb)) return;
  const int S = m.S;
  const int Jc = cell / Gc.nx, Ic = cell - Jc * Gc.nx;
  double sp = 0.0, sc = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const size_t id = ((size_t)(2 * Jc + (q >> 1)) * Gf.nx + 2 * Ic + (q & 1)) * S + s;
    sp += pf[id];
    sc += cf[id];
  }
  const size_t o = (size_t)cell * S + s;
  pc[o] = 0.25 * sp;
  cc[o] = 0.25 * sc;
}

__global__ void k_restrict_coef(Map m, Grid2 Gf, Grid2 Gc, const double* __restrict__ phif,
                                const double* __restrict__ Kf, double* __restrict__ phic, double* __restrict__ Kc) {
  int s, cell, sb, cb;
  if (!map_cell(m, Gc.ncell, s, cell, sb, cb)) return;
  const int S = m.S;
  const int Jc = cell / Gc.nx, Ic = cell - Jc * Gc.nx;
  double sp = 0.0, sk = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const size_t id = ((size_t)(2 * Jc + (q >> 1)) * Gf.nx + 2 * Ic + (q & 1)) * S + s;
    sp += phif[id];
    sk += log(Kf[id]);
  }
  const size_t o = (size_t)cell * S + s;
  phic[o] = 0.25 * sp;
  Kc[o] = exp(0.25 * sk);
}

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
  extern __shared__ unsigned char smem_raw[];
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
  extern __shared__ unsigned char smem_raw[];
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
  extern __shared__ unsigned char smem_raw[];
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

// ==========================================================================
// precision converters (a9)
// ==========================================================================
template <typename TI, typename TO>
__global__ void k_convert(size_t n, const TI* __restrict__ a, TO* __restrict__ b) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = (TO)a[t];
}

// ==========================================================================
// a3/a4: batched BiCGStab (FP64), per-sample scalars, fused dots
// ==========================================================================
// per-sample scalar slots
enum { SC_RHO = 0, SC_ALPHA, SC_OMEGA, SC_BETA, SC_R0, SC_RNORM, SC_ACTIVE, SC_ITS, SC_NSLOT };

// r = sign * R (zero for samples with ndone[s] set; ndone may be NULL), rhat = r, x = 0; partial |r|^2
__global__ void __launch_bounds__(256) k_bicg_init(Map m, int ncell, const double* __restrict__ R, double sign,
                                                   const int* __restrict__ ndone, double* __restrict__ r,
                                                   double* __restrict__ rhat, double* __restrict__ x,
                                                   double* __restrict__ part) {
  __shared__ double lds[256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  const size_t N = (size_t)ncell * m.S;
  double acc[1] = {0.0};
  const double msk = (sv && !(ndone && ndone[s])) ? sign : 0.0;
  for (int k = 0; k < m.CPT; ++k) {
    const int cell = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || cell >= ncell) continue;
    const size_t id = (size_t)cell * m.S + s;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      const double v = R[comp * N + id] * msk;
      r[comp * N + id] = v;
      rhat[comp * N + id] = v;
      x[comp * N + id] = 0.0;
      acc[0] += v * v;
    }
  }
  block_sum_y<1>(acc, lds);
  if (threadIdx.y == 0 && sv) part[(size_t)cblk * m.S + s] = acc[0];
}

// p = r (first) or r + beta (p - omega v)
__global__ void __launch_bounds__(256) k_bicg_p(Map m, int ncell, int first, const double* __restrict__ sc,
                                                const double* __restrict__ r, const double* __restrict__ v,
                                                double* __restrict__ p) {
  int s, cell, sb, cb;
  if (!map_cell(m, ncell, s, cell, sb, cb)) return;
  const size_t N = (size_t)ncell * m.S, id = (size_t)cell * m.S + s;
  const double beta = first ? 0.0 : sc[SC_BETA * m.S + s];
  const double om = sc[SC_OMEGA * m.S + s];
#pragma unroll
  for (int comp = 0; comp < 2; ++comp) {
    const size_t q = comp * N + id;
    p[q] = first ? r[q] : r[q] + beta * (p[q] - om * v[q]);
  }
}

// y = A x with per-sample partial dot products: NDOT = 1: (d0, y); NDOT = 2: (y, d0), (y, y)
template <int NDOT, bool TR = false>
__global__ void __launch_bounds__(256) k_spmv_dot(Map m, Grid2 G, const double* __restrict__ J,
                                                  const double* __restrict__ x, double* __restrict__ y,
                                                  const double* __restrict__ d0, double* __restrict__ part) {
  __shared__ double lds[2 * 256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  const size_t N = (size_t)G.ncell * m.S;
  double acc[NDOT];
#pragma unroll
  for (int q = 0; q < NDOT; ++q) acc[q] = 0.0;
  for (int k = 0; k < m.CPT; ++k) {
    const int cell = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || cell >= G.ncell) continue;
    const int j = cell / G.nx, i = cell - j * G.nx;
    const size_t id = (size_t)cell * m.S + s;
    double y0, y1;
    apply_row<double, double, TR>(J, x, N, id, i, j, G.nx, G.ny, m.S, y0, y1, false);
    y[id] = y0;
    y[N + id] = y1;
    if (NDOT == 1) {
      acc[0] += d0[id] * y0 + d0[N + id] * y1;
    } else {
      acc[0] += y0 * d0[id] + y1 * d0[N + id];
      acc[NDOT - 1] += y0 * y0 + y1 * y1;
    }
  }
  block_sum_y<NDOT>(acc, lds);
  if (threadIdx.y == 0 && sv) {
#pragma unroll
    for (int q = 0; q < NDOT; ++q) part[((size_t)q * m.ncb + cblk) * m.S + s] = acc[q];
  }
}

// s = r - alpha v
__global__ void __launch_bounds__(256) k_bicg_s(Map m, int ncell, const double* __restrict__ sc,
                                                const double* __restrict__ r, const double* __restrict__ v,
                                                double* __restrict__ sv_) {
  int s, cell, sb, cb;
  if (!map_cell(m, ncell, s, cell, sb, cb)) return;
  const size_t N = (size_t)ncell * m.S, id = (size_t)cell * m.S + s;
  const double al = sc[SC_ALPHA * m.S + s];
  sv_[id] = r[id] - al * v[id];
  sv_[N + id] = r[N + id] - al * v[N + id];
}

// x += alpha ph + omega sh; r = s - omega t; partials (rhat, r), (r, r)
__global__ void __launch_bounds__(256) k_bicg_xr(Map m, int ncell, const double* __restrict__ sc,
                                                 const double* __restrict__ ph, const double* __restrict__ sh,
                                                 const double* __restrict__ sv_, const double* __restrict__ t,
                                                 const double* __restrict__ rhat, double* __restrict__ x,
                                                 double* __restrict__ r, double* __restrict__ part) {
  __shared__ double lds[2 * 256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  const size_t N = (size_t)ncell * m.S;
  double acc[2] = {0.0, 0.0};
  const double al = sv ? sc[SC_ALPHA * m.S + s] : 0.0, om = sv ? sc[SC_OMEGA * m.S + s] : 0.0;
  for (int k = 0; k < m.CPT; ++k) {
    const int cell = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || cell >= ncell) continue;
    const size_t id = (size_t)cell * m.S + s;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      const size_t q = comp * N + id;
      x[q] += al * ph[q] + om * sh[q];
      const double rv = sv_[q] - om * t[q];
      r[q] = rv;
      acc[0] += rhat[q] * rv;
      acc[1] += rv * rv;
    }
  }
  block_sum_y<2>(acc, lds);
  if (threadIdx.y == 0 && sv) {
    part[(size_t)cblk * m.S + s] = acc[0];
    part[((size_t)m.ncb + cblk) * m.S + s] = acc[1];
  }
}

// Sum NQ partial arrays [q][ncb][S] over cell blocks in a fixed order.
template <int NQ>
__device__ __forceinline__ void reduce_partials(const Map& m, const double* __restrict__ part, int s, double (&out)[NQ],
                                                double* lds) {
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  if (s < m.S) {
    const int st = blockDim.y;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double* pq = part + (size_t)q * m.ncb * m.S + s;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int cb = threadIdx.y;
      for (; cb + 3 * st < m.ncb; cb += 4 * st) {
        a0 += pq[(size_t)cb * m.S];
        a1 += pq[(size_t)(cb + st) * m.S];
        a2 += pq[(size_t)(cb + 2 * st) * m.S];
        a3 += pq[(size_t)(cb + 3 * st) * m.S];
      }
      for (; cb < m.ncb; cb += st) a0 += pq[(size_t)cb * m.S];
      v[q] = (a0 + a1) + (a2 + a3);
    }
  }
  block_sum_y<NQ>(v, lds);
#pragma unroll
  for (int q = 0; q < NQ; ++q) out[q] = v[q];
}

template <int NQ>
__device__ __forceinline__ void reduce_partials_max(const Map& m, const double* __restrict__ part, int s,
                                                    double (&out)[NQ], double* lds) {
  double v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = 0.0;
  if (s < m.S) {
    for (int cb = threadIdx.y; cb < m.ncb; cb += blockDim.y) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const double a = part[((size_t)q * m.ncb + cb) * m.S + s];
        v[q] = (a > v[q] || a != a) ? a : v[q];
      }
    }
  }
  block_max_y<NQ>(v, lds);
#pragma unroll
  for (int q = 0; q < NQ; ++q) out[q] = v[q];
}

// Finalisation kernels: blockDim = (64, FIN_Y), grid = ceil(S/64).  ctrl[0] counts active samples.
constexpr int FIN_Y = 16;

__global__ void __launch_bounds__(64 * FIN_Y) k_fin_init(Map m, const double* __restrict__ part, double* __restrict__ sc,
                                                  int* __restrict__ ctrl) {
  __shared__ double lds[64 * FIN_Y];
  const int s = blockIdx.x * 64 + threadIdx.x;
  double v[1];
  reduce_partials<1>(m, part, s, v, lds);
  if (threadIdx.y == 0 && s < m.S) {
    const int S = m.S;
    sc[SC_RHO * S + s] = v[0];          // (rhat, r) = |r|^2 with rhat = r
    sc[SC_R0 * S + s] = v[0];
    sc[SC_RNORM * S + s] = v[0];
    sc[SC_ALPHA * S + s] = 0.0;
    sc[SC_OMEGA * S + s] = 0.0;
    sc[SC_BETA * S + s] = 0.0;
    const int act = v[0] > 0.0;
    sc[SC_ACTIVE * S + s] = act;
    sc[SC_ITS * S + s] = 0.0;
    if (act) atomicAdd(&ctrl[0], 1);
  }
}

__global__ void __launch_bounds__(64 * FIN_Y) k_fin_alpha(Map m, const double* __restrict__ part,
                                                          double* __restrict__ sc, int* __restrict__ status) {
  __shared__ double lds[64 * FIN_Y];
  const int s = blockIdx.x * 64 + threadIdx.x;
  double v[1];
  reduce_partials<1>(m, part, s, v, lds);
  if (threadIdx.y == 0 && s < m.S) {
    const int S = m.S;
    double al = 0.0;
    if (sc[SC_ACTIVE * S + s] != 0.0) {
      if (v[0] != 0.0 && isfinite(v[0])) {
        al = sc[SC_RHO * S + s] / v[0];
      } else {
        sc[SC_ACTIVE * S + s] = 0.0;   // breakdown: (rhat, A p) = 0
        if (status) status[s] = 2;
      }
    }
    sc[SC_ALPHA * S + s] = al;
  }
}

__global__ void __launch_bounds__(64 * FIN_Y) k_fin_omega(Map m, const double* __restrict__ part,
                                                          double* __restrict__ sc) {
  __shared__ double lds[2 * 64 * FIN_Y];
  const int s = blockIdx.x * 64 + threadIdx.x;
  double v[2];
  reduce_partials<2>(m, part, s, v, lds);
  if (threadIdx.y == 0 && s < m.S) {
    const int S = m.S;
    double om = 0.0;
    if (sc[SC_ACTIVE * S + s] != 0.0 && v[1] > 0.0) om = v[0] / v[1];
    sc[SC_OMEGA * S + s] = om;
  }
}

__global__ void __launch_bounds__(64 * FIN_Y) k_fin_rho(Map m, const double* __restrict__ part,
                                                        double* __restrict__ sc, double rtol2, int* __restrict__ status,
                                                        int* __restrict__ ctrl) {
  __shared__ double lds[2 * 64 * FIN_Y];
  const int s = blockIdx.x * 64 + threadIdx.x;
  double v[2];
  reduce_partials<2>(m, part, s, v, lds);
  if (threadIdx.y == 0 && s < m.S) {
    const int S = m.S;
    if (sc[SC_ACTIVE * S + s] != 0.0) {
      const double rho_new = v[0], rr = v[1];
      const double om = sc[SC_OMEGA * S + s];
      sc[SC_ITS * S + s] += 1.0;
      sc[SC_RNORM * S + s] = rr;
      bool act = true;
      if (!(rr <= rtol2 * sc[SC_R0 * S + s])) {
        if (om == 0.0 || rho_new == 0.0 || !isfinite(rho_new)) {
          act = false;   // breakdown before convergence
          if (status) status[s] = 2;
        } else {
          sc[SC_BETA * S + s] = (rho_new / sc[SC_RHO * S + s]) * (sc[SC_ALPHA * S + s] / om);
          sc[SC_RHO * S + s] = rho_new;
        }
      } else {
        act = false;     // converged
      }
      if (!act) {
        sc[SC_ACTIVE * S + s] = 0.0;
        sc[SC_BETA * S + s] = 0.0;
      } else {
        atomicAdd(&ctrl[0], 1);
      }
    }
    if (sc[SC_ACTIVE * S + s] == 0.0) {
      sc[SC_ALPHA * S + s] = 0.0;
      sc[SC_OMEGA * S + s] = 0.0;
    }
  }
}

// ==========================================================================
// a3: Newton update with per-sample damping and convergence
// ==========================================================================
// partial max |dp|, |dc| per sample
__global__ void __launch_bounds__(256) k_delta_max(Map m, int ncell, const double* __restrict__ d,
                                                   double* __restrict__ part) {
  __shared__ double lds[2 * 256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  const size_t N = (size_t)ncell * m.S;
  double acc[2] = {0.0, 0.0};
  for (int k = 0; k < m.CPT; ++k) {
    const int cell = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || cell >= ncell) continue;
    const size_t id = (size_t)cell * m.S + s;
    const double a = fabs(d[id]), b = fabs(d[N + id]);
    acc[0] = (a > acc[0] || a != a) ? a : acc[0];
    acc[1] = (b > acc[1] || b != b) ? b : acc[1];
  }
  block_max_y<2>(acc, lds);
  if (threadIdx.y == 0 && sv) {
    part[(size_t)cblk * m.S + s] = acc[0];
    part[((size_t)m.ncb + cblk) * m.S + s] = acc[1];
  }
}

// Per sample: damping factor lambda = min(1, dc_max/|dc|_inf); convergence on the
// undamped update; non-finite updates freeze the sample.  ctrl[1] counts samples
// still iterating.  stats[s][0] counts Newton iterations.
__global__ void __launch_bounds__(64 * FIN_Y) k_fin_newton(Map m, const double* __restrict__ part, double p_ref,
                                                           double tol, double dc_max, double* __restrict__ lam,
                                                           int* __restrict__ ndone, int* __restrict__ status,
                                                           double* __restrict__ stats, int* __restrict__ ctrl) {
  __shared__ double lds[2 * 64 * FIN_Y];
  const int s = blockIdx.x * 64 + threadIdx.x;
  double v[2];
  reduce_partials_max<2>(m, part, s, v, lds);
  if (threadIdx.y != 0 || s >= m.S) return;
  const double mp = v[0], mc = v[1];
  if (ndone[s]) {
    lam[s] = 0.0;
    return;
  }
  stats[(size_t)s * 4] += 1.0;
  if (!isfinite(mp) || !isfinite(mc)) {
    lam[s] = 0.0;
    ndone[s] = 1;
    status[s] = 3;
    return;
  }
  lam[s] = mc > dc_max ? dc_max / mc : 1.0;
  const double size = fmax(mc, mp / p_ref);
  if (size <= tol) ndone[s] = 1;
  else atomicAdd(&ctrl[1], 1);
}

__global__ void __launch_bounds__(256) k_newton_update(Map m, int ncell, const double* __restrict__ lam,
                                                       const double* __restrict__ d, double* __restrict__ p,
                                                       double* __restrict__ c) {
  int s, cell, sb, cb;
  if (!map_cell(m, ncell, s, cell, sb, cb)) return;
  const size_t N = (size_t)ncell * m.S, id = (size_t)cell * m.S + s;
  const double l = lam[s];
  if (l != 0.0) {
    p[id] += l * d[id];
    c[id] += l * d[N + id];
  }
}

// ==========================================================================
// a7: mass balance, range check and QoI
// ==========================================================================
// Per sample partial sums: [0] fluid storage change, [1] salt storage change,
// [2] tau * fluid boundary outflux, [3] tau * salt boundary outflux, [4] min c, [5] max c
__global__ void __launch_bounds__(256) k_balance(Map m, Grid2 G, Phys P, const double* __restrict__ p,
                                                 const double* __restrict__ c, const double* __restrict__ c_old,
                                                 const double* __restrict__ phi, const double* __restrict__ K,
                                                 const double* __restrict__ uin, double* __restrict__ part) {
  __shared__ double lds[4 * 256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double mn[1] = {0.0}, mx[1] = {0.0};
  for (int k = 0; k < m.CPT; ++k) {
    const int cell = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || cell >= G.ncell) continue;
    const int j = cell / G.nx, i = cell - j * G.nx;
    const size_t id = (size_t)cell * m.S + s;
    const double cP = c[id], co = c_old[id], ph = phi[id];
    const double r = P.rho0 + P.drho * cP, ro = P.rho0 + P.drho * co;
    acc[0] += P.vol * ph * (r - ro);
    acc[1] += P.vol * ph * (r * cP - ro * co);
    const double wb = P.hy / P.hx;
    if (i == 0) {
      const double F = -(P.rho0 + P.drho * P.c_left) * uin[s] * P.hy;
      acc[2] += P.tau * F;
      acc[3] += P.tau * (F * P.c_left + 2.0 * r * ph * P.Dm * (cP - P.c_left) * wb);
    }
    if (i == G.nx - 1) {
      const double y = -P.Ly + (j + 0.5) * P.hy;
      const double u = -(K[id] / P.mu) * (-P.rho1 * P.g * y - p[id]) / (0.5 * P.hx);
      const bool inflow = u < 0.0;
      const double F = (inflow ? P.rho1 : r) * u * P.hy;
      double Gs = F * (inflow ? 1.0 : cP);
      if (P.right_dir) Gs += 2.0 * r * ph * P.Dm * (cP - 1.0) * wb;
      acc[2] += P.tau * F;
      acc[3] += P.tau * Gs;
    }
    mn[0] = (cP < mn[0] || cP != cP) ? cP : mn[0];
    mx[0] = (cP > mx[0] || cP != cP) ? cP : mx[0];
  }
  block_sum_y<4>(acc, lds);
  for (int q = 0; q < 1; ++q) mn[q] = -mn[q];
  block_max_y<1>(mn, lds);
  block_max_y<1>(mx, lds);
  if (threadIdx.y == 0 && sv) {
#pragma unroll
    for (int q = 0; q < 4; ++q) part[((size_t)q * m.ncb + cblk) * m.S + s] = acc[q];
    part[((size_t)4 * m.ncb + cblk) * m.S + s] = mn[0];   // -min c
    part[((size_t)5 * m.ncb + cblk) * m.S + s] = mx[0];
  }
}

// stats[s][2..3] = running max of |storage change + tau * boundary outflux| / (tau rho0 u_in Ly)
__global__ void __launch_bounds__(64 * FIN_Y) k_fin_balance(Map m, Phys P, const double* __restrict__ part,
                                                            const double* __restrict__ uin, double c_tol,
                                                            double* __restrict__ stats, int* __restrict__ status) {
  __shared__ double lds[4 * 64 * FIN_Y];
  const int s = blockIdx.x * 64 + threadIdx.x;
  double a[4];
  reduce_partials<4>(m, part, s, a, lds);
  double e[2];
  reduce_partials_max<2>(m, part + (size_t)4 * m.ncb * m.S, s, e, lds);   // [4] = -min c, [5] = max c
  if (threadIdx.y != 0 || s >= m.S) return;
  const double mn = -e[0], mx = e[1];
  const double scale = P.tau * P.rho0 * uin[s] * P.Ly;
  const double df = fabs(a[0] + a[2]) / scale, ds = fabs(a[1] + a[3]) / scale;
  double* st = stats + (size_t)s * 4;
  st[2] = fmax(st[2], df);
  st[3] = fmax(st[3], ds);
  if ((!(mn >= -c_tol) || !(mx <= 1.0 + c_tol)) && status[s] == 0) status[s] = 4;
}

// Q = sum over cells with centre x > Lx/2 of c rho(c) h^2 (partials)
__global__ void __launch_bounds__(256) k_qoi(Map m, Grid2 G, Phys P, const double* __restrict__ c,
                                             double* __restrict__ part) {
  __shared__ double lds[256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  double acc[1] = {0.0};
  for (int k = 0; k < m.CPT; ++k) {
    const int cell = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || cell >= G.ncell) continue;
    const int j = cell / G.nx, i = cell - j * G.nx;
    if ((i + 0.5) * P.hx > 0.5 * P.Lx) {
      const double cP = c[(size_t)cell * m.S + s];
      acc[0] += cP * (P.rho0 + P.drho * cP);
    }
  }
  block_sum_y<1>(acc, lds);
  if (threadIdx.y == 0 && sv) part[(size_t)cblk * m.S + s] = acc[0];
}

__global__ void __launch_bounds__(64 * FIN_Y) k_fin_sum(Map m, const double* __restrict__ part, double scale,
                                                        double* __restrict__ out) {
  __shared__ double lds[64 * FIN_Y];
  const int s = blockIdx.x * 64 + threadIdx.x;
  double a[1];
  reduce_partials<1>(m, part, s, a, lds);
  if (threadIdx.y == 0 && s < m.S) out[s] = a[0] * scale;
}

}  // namespace henry
