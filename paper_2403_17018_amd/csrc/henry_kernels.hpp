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
  double uin_fac;   // time factor of the left inflow for the step being solved
  double qoi_xmin;  // QoI region: cells whose centre lies in x > qoi_xmin
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
  double phi_mean, phi_amp, phi_min, phi_max, lnK_mean, logK_amp, q_in, q_in_amp, kappa_kc;
  int n_phi, n_logK;
  int model;   // 0: KL fields; 1: the section-4 porosity with Kozeny-Carman permeability
};

__device__ __forceinline__ bool map_cell(const Map& m, int ncell, int& s, int& cell, int& sblk, int& cblk) {
  const int bid = blockIdx.x;
  sblk = bid % m.nsb;
  cblk = bid / m.nsb;
  s = sblk * m.SX + (int)threadIdx.x;
  cell = cblk * m.CY + (int)threadIdx.y;
  return s < m.S && cell < ncell;
}

// SP adjacent samples per thread (the stencil kernels' wide form): a Map built by
// make_map_wide holds SX threads of SP samples each per row, and the batch size is a
// multiple of SP, so a thread's first sample s < S brings s + 1 .. s + SP - 1 with it.
// Its values are held as a vector of SP lanes, loaded and stored in one access each.
template <int SP>
__device__ __forceinline__ bool map_cell_sp(const Map& m, int ncell, int& s, int& cell, int& sblk, int& cblk) {
  const int bid = blockIdx.x;
  sblk = bid % m.nsb;
  cblk = bid / m.nsb;
  s = SP * (sblk * m.SX + (int)threadIdx.x);
  cell = cblk * m.CY + (int)threadIdx.y;
  return s < m.S && cell < ncell;
}

template <typename T, int SP> struct VecOf { typedef T __attribute__((ext_vector_type(SP))) type; };
template <typename T> struct VecOf<T, 1> { typedef T type; };
// load SP consecutive samples of type T at p as the value type VA (converted lane by lane)
template <int SP, typename VA, typename T>
__device__ __forceinline__ VA ldv(const T* p) {
  if constexpr (SP == 1) {
    return (VA)*p;
  } else {
    const typename VecOf<T, SP>::type v = *(const typename VecOf<T, SP>::type*)p;
    return __builtin_convertvector(v, VA);
  }
}
template <int SP, typename VA, typename T>
__device__ __forceinline__ VA ldv_nt(const T* p) {
  if constexpr (SP == 1) {
    return (VA)__builtin_nontemporal_load(p);
  } else {
    const typename VecOf<T, SP>::type v = __builtin_nontemporal_load((const typename VecOf<T, SP>::type*)p);
    return __builtin_convertvector(v, VA);
  }
}
template <int SP, typename T, typename V>
__device__ __forceinline__ void stv(T* p, V v) {
  if constexpr (SP == 1) *p = v;
  else *(typename VecOf<T, SP>::type*)p = v;
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
  const size_t id = (size_t)cell * m.S + s;
  if (fp.model == 1) {
    // section 4, eq. poro_2levels: a second layer below y = -0.8, large-scale and
    // small-scale periodic factors; K by Kozeny-Carman (eq. e_perm_Kozeny_Carman)
    const double xi1 = th[0], xi2 = th[1];
    const double c0 = y < -0.8 ? 1.2 * (1.0 + 0.2 * xi1) : 1.0;
    const double c1 = 1.0 + 0.15 * (xi2 * cospi(0.5 * x) - xi2 * sinpi(2.0 * y) + xi1 * cospi(2.0 * x));
    const double c2 = 1.0 + 0.2 * (xi1 * sinpi(64.0 * x) + xi2 * sinpi(32.0 * y));
    const double ph = fp.phi_mean * c0 * c1 * c2;
    if (phi) phi[id] = ph;
    if (K) K[id] = fp.kappa_kc * ph * ph * ph / (1.0 - ph * ph);
  } else {
    double sp = 0.0, sk = 0.0;
    for (int k = 0; k < kl.n; ++k) {
      const double e = kl_1d(kl.wx[k], kl.oddx[k], kl.normx[k], x - kl.xc) *
                       kl_1d(kl.wy[k], kl.oddy[k], kl.normy[k], y - kl.yc);
      if (k < fp.n_phi) sp += kl.sqrt_lam[k] * th[k] * e;
      if (k < fp.n_logK) sk += kl.sqrt_lam[k] * th[4 + k] * e;
    }
    if (phi) phi[id] = fmin(fmax(fp.phi_mean * (1.0 + fp.phi_amp * sp), fp.phi_min), fp.phi_max);
    if (K) K[id] = exp(fp.lnK_mean + fp.logK_amp * sk);
  }
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

// Thread map of the assembly: a workgroup takes ASM_TX x ASM_TY cells (a tile) of one sample
// block, blockDim = (SX, ASM_TY * ASM_TX) (one row of threads per cell); the grid enumerates
// (sample block, tile) pairs.  The tile's p, c, phi, K and those of its one-cell halo (the
// neighbours across its four sides) are staged in LDS, so each value is read from memory
// (T + H) / T = 2.5 times for a 4 x 2 tile (once as a cell, as a halo cell of the tiles around
// it otherwise) instead of five times.  4 x 2 measured faster than 4 x 4 and 4 x 1 at level 3
// in both precisions (812 / 857 / 825 us per FP64 launch).
constexpr int ASM_TX = 4, ASM_TY = 2, ASM_T = ASM_TX * ASM_TY, ASM_H = 2 * (ASM_TX + ASM_TY);
__host__ __device__ inline int asm_tiles(int nx, int ny) {
  return ((nx + ASM_TX - 1) / ASM_TX) * ((ny + ASM_TY - 1) / ASM_TY);
}
__host__ __device__ inline size_t asm_lds(int SX) { return (size_t)4 * (ASM_T + ASM_H) * SX * sizeof(double); }

// J block order: 0 centre, 1 west, 2 east, 3 south, 4 north.  Each neighbour block is
// stored as soon as its face is done (zeros for a missing neighbour), so only the centre
// block and the residual stay live across the faces.
template <bool WRITE_R, typename TJ, bool WRITE_J32, bool WRITE_J = true>
__global__ void __launch_bounds__(1024) k_assemble(Map m, Grid2 G, Phys P, const double* __restrict__ p,
                                                   const double* __restrict__ c, const double* __restrict__ c_old,
                                                   const double* __restrict__ phi, const double* __restrict__ K,
                                                   const double* __restrict__ uin, double* __restrict__ R,
                                                   TJ* __restrict__ J, float* __restrict__ J32) {
  extern __shared__ double asm_sh[];   // [field p, c, phi, K][tile cell, then halo][SX]
  const int SX = m.SX, tx = threadIdx.x, ty = threadIdx.y;
  const int sb = blockIdx.x % m.nsb, tile = blockIdx.x / m.nsb;
  const int ntx = (G.nx + ASM_TX - 1) / ASM_TX;
  const int i0 = (tile % ntx) * ASM_TX, j0 = (tile / ntx) * ASM_TY;
  const int di = ty % ASM_TX, dj = ty / ASM_TX;
  const int i = i0 + di, j = j0 + dj;
  const int s = sb * SX + tx;
  const int S = m.S;
  const bool sv = s < S;
  const bool inside = sv && i < G.nx && j < G.ny;
  auto slot = [&](int f, int q) -> double& { return asm_sh[((size_t)f * (ASM_T + ASM_H) + q) * SX + tx]; };
  const size_t id = ((size_t)j * G.nx + i) * S + s;
  // the cell's own old concentration and its sample's inflow are loaded here, beside the
  // tile's staging loads: issued later, their waits would also wait for every Jacobian store
  // issued before them
  const double co = (WRITE_R && inside) ? c_old[id] : 0.0;
  const double u_in = (inside && i == 0) ? uin[s] : 0.0;
  if (inside) {
    slot(0, ty) = p[id];
    slot(1, ty) = c[id];
    slot(2, ty) = phi[id];
    slot(3, ty) = K[id];
  }
  // halo cells: [0, TY) west column, [TY, 2 TY) east column, [2 TY, 2 TY + TX) south row,
  // [2 TY + TX, 2 TY + 2 TX) north row
  for (int h = ty; h < ASM_H; h += ASM_T) {
    int hi, hj;
    if (h < ASM_TY) {
      hi = i0 - 1;
      hj = j0 + h;
    } else if (h < 2 * ASM_TY) {
      hi = i0 + ASM_TX;
      hj = j0 + h - ASM_TY;
    } else if (h < 2 * ASM_TY + ASM_TX) {
      hi = i0 + h - 2 * ASM_TY;
      hj = j0 - 1;
    } else {
      hi = i0 + h - 2 * ASM_TY - ASM_TX;
      hj = j0 + ASM_TY;
    }
    if (sv && hi >= 0 && hi < G.nx && hj >= 0 && hj < G.ny) {
      const size_t hq = ((size_t)hj * G.nx + hi) * S + s;
      slot(0, ASM_T + h) = p[hq];
      slot(1, ASM_T + h) = c[hq];
      slot(2, ASM_T + h) = phi[hq];
      slot(3, ASM_T + h) = K[hq];
    }
  }
  __syncthreads();
  if (!inside) return;
  // LDS slot of a neighbour: inside the tile, or the halo cell across the tile's side
  const int qW = di > 0 ? ty - 1 : ASM_T + dj, qE = di < ASM_TX - 1 ? ty + 1 : ASM_T + ASM_TY + dj;
  const int qS = dj > 0 ? ty - ASM_TX : ASM_T + 2 * ASM_TY + di;
  const int qN = dj < ASM_TY - 1 ? ty + ASM_TX : ASM_T + 2 * ASM_TY + ASM_TX + di;
  const size_t N = (size_t)G.ncell * S;
  const double pP = slot(0, ty), cP = slot(1, ty), phP = slot(2, ty), KP = slot(3, ty);
  const double rP = P.rho0 + P.drho * cP;
  double Rp = 0.0, Rc = 0.0;
  double D[4];
  auto put = [&](int slot, double b0, double b1, double b2, double b3) {
    if (!WRITE_J) return;
    const double v[4] = {b0, b1, b2, b3};
    // written once here and read by later kernels, never from cache: non-temporal stores
#pragma unroll
    for (int e = 0; e < 4; ++e) __builtin_nontemporal_store((TJ)v[e], J + (slot * 4 + e) * N + id);
    if (WRITE_J32) {
#pragma unroll
      for (int e = 0; e < 4; ++e) __builtin_nontemporal_store((float)v[e], J32 + (slot * 4 + e) * N + id);
    }
  };
  if (WRITE_R) {
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
    face_flux(P, false, slot(0, qW), slot(1, qW), slot(2, qW), slot(3, qW), pP, cP, phP, KP, f);
    Rp -= f.F; Rc -= f.G;
    D[0] += f.a; D[1] -= f.bF; D[2] += f.a * f.cup; D[3] -= f.dGH;
    put(1, -f.a, -f.bF, -f.a * f.cup, -f.dGL);
  } else {
    put(1, 0.0, 0.0, 0.0, 0.0);
  }
  // east face: P is the low side
  if (i < G.nx - 1) {
    face_flux(P, false, pP, cP, phP, KP, slot(0, qE), slot(1, qE), slot(2, qE), slot(3, qE), f);
    Rp += f.F; Rc += f.G;
    D[0] += f.a; D[1] += f.bF; D[2] += f.a * f.cup; D[3] += f.dGL;
    put(2, -f.a, f.bF, -f.a * f.cup, f.dGH);
  } else {
    put(2, 0.0, 0.0, 0.0, 0.0);
  }
  // south face
  if (j > 0) {
    face_flux(P, true, slot(0, qS), slot(1, qS), slot(2, qS), slot(3, qS), pP, cP, phP, KP, f);
    Rp -= f.F; Rc -= f.G;
    D[0] += f.a; D[1] -= f.bF; D[2] += f.a * f.cup; D[3] -= f.dGH;
    put(3, -f.a, -f.bF, -f.a * f.cup, -f.dGL);
  } else {
    put(3, 0.0, 0.0, 0.0, 0.0);
  }
  // north face
  if (j < G.ny - 1) {
    face_flux(P, true, pP, cP, phP, KP, slot(0, qN), slot(1, qN), slot(2, qN), slot(3, qN), f);
    Rp += f.F; Rc += f.G;
    D[0] += f.a; D[1] += f.bF; D[2] += f.a * f.cup; D[3] += f.dGL;
    put(4, -f.a, f.bF, -f.a * f.cup, f.dGH);
  } else {
    put(4, 0.0, 0.0, 0.0, 0.0);
  }
  const double wb = P.hy / P.hx;
  // left boundary: prescribed inflow at c_left, diffusive Dirichlet c_left
  if (i == 0) {
    const double F = -(P.rho0 + P.drho * P.c_left) * u_in * P.uin_fac * P.hy;
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
  put(0, D[0], D[1], D[2], D[3]);
}


// ==========================================================================
// a4/a5: block stencil operations (SpMV, red-black block Gauss-Seidel, transfers)
// ==========================================================================
// (A x)_P for one cell-sample: centre block + the 4 neighbour blocks that exist.
// TR: (A^T x)_P, gathering the transposed blocks A_{Q,P} stored in the neighbours'
// rows (Q east of P holds A_{Q,P} in its west slot, and so on), so no atomics.
// xv(q, dir) returns the 2-vector x at row index q (dir: 0 centre, 1 W, 2 E, 3 S, 4 N).
// SP > 1: the row of SP adjacent samples at once, TA a vector of SP lanes.
template <typename T, typename TA, bool TR, int SP = 1, typename XV>
__device__ __forceinline__ void apply_row_f(const T* __restrict__ J, XV&& xv, size_t N, size_t id, int i, int j,
                                            int nx, int ny, int S, TA& y0, TA& y1, bool skip_centre) {
  // All blocks' loads are issued before any is used: a neighbour outside the grid reads the
  // cell's own x (dir 0) and centre block instead, valid addresses the cell reads anyway, and
  // its term is selected away (a select, so whatever those values hold cannot leak in).
  // Each Jacobian entry is read once per kernel: non-temporal loads keep the cache for the
  // neighbours' x, which other threads read again.
  const size_t row = (size_t)nx * S;
  const bool ok[4] = {i > 0, i < nx - 1, j > 0, j < ny - 1};
  TA xa[5], xb[5], jb[5][4];
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    if (n == 0 && skip_centre) continue;
    const bool on = n == 0 || ok[n - 1];
    const long long d = n == 1 ? -(long long)S : n == 2 ? (long long)S : n == 3 ? -(long long)row : (long long)row;
    const size_t xq = (n == 0 || !on) ? id : id + d;
    // slot of the block: P's own row (W 1, E 2, S 3, N 4), or, transposed, the neighbour's
    // row at the mirrored slot
    const int slot = n == 0 ? 0 : TR ? (n == 1 ? 2 : n == 2 ? 1 : n == 3 ? 4 : 3) : n;
    const size_t q = (TR && on) ? xq : id;
    const size_t jo = (size_t)(on ? slot : 0) * 4 * N + q;
    xv(xq, on ? n : 0, xa[n], xb[n]);
#pragma unroll
    for (int e = 0; e < 4; ++e) jb[n][e] = ldv_nt<SP, TA>(J + jo + (size_t)e * N);
  }
  TA a0 = 0, a1 = 0;
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    if (n == 0 && skip_centre) continue;
    const bool on = n == 0 || ok[n - 1];
    TA t0, t1;
    if (TR) {
      t0 = jb[n][0] * xa[n] + jb[n][2] * xb[n];
      t1 = jb[n][1] * xa[n] + jb[n][3] * xb[n];
    } else {
      t0 = jb[n][0] * xa[n] + jb[n][1] * xb[n];
      t1 = jb[n][2] * xa[n] + jb[n][3] * xb[n];
    }
    a0 += on ? t0 : (TA)0;
    a1 += on ? t1 : (TA)0;
  }
  y0 = a0;
  y1 = a1;
}

template <typename T, typename TA, bool TR = false, int SP = 1>
__device__ __forceinline__ void apply_row(const T* __restrict__ J, const T* __restrict__ x, size_t N, size_t id, int i,
                                          int j, int nx, int ny, int S, TA& y0, TA& y1, bool skip_centre) {
  auto xv = [&](size_t q, int, TA& x0, TA& x1) {
    x0 = ldv<SP, TA>(x + q);
    x1 = ldv<SP, TA>(x + N + q);
  };
  apply_row_f<T, TA, TR, SP>(J, xv, N, id, i, j, nx, ny, S, y0, y1, skip_centre);
}

// Bilinear cell-centred prolongation of the coarse correction e to fine cell (i, j):
// weights 9/16, 3/16, 3/16, 1/16, a missing neighbour at the boundary replaced by the
// cell itself.
template <typename T, int SP = 1, typename V = T>
__device__ __forceinline__ void prolong_at(const T* __restrict__ e, size_t Nc, int S, int s, int i, int j, Grid2 Gc,
                                           V& v0, V& v1) {
  const int I = i >> 1, Jc = j >> 1;
  int I2 = I + ((i & 1) ? 1 : -1), J2 = Jc + ((j & 1) ? 1 : -1);
  I2 = I2 < 0 ? 0 : (I2 >= Gc.nx ? Gc.nx - 1 : I2);
  J2 = J2 < 0 ? 0 : (J2 >= Gc.ny ? Gc.ny - 1 : J2);
  const size_t c00 = ((size_t)Jc * Gc.nx + I) * S + s, c10 = ((size_t)Jc * Gc.nx + I2) * S + s;
  const size_t c01 = ((size_t)J2 * Gc.nx + I) * S + s, c11 = ((size_t)J2 * Gc.nx + I2) * S + s;
  const T w9 = (T)0.5625, w3 = (T)0.1875, w1 = (T)0.0625;
  v0 = w9 * ldv<SP, V>(e + c00) + w3 * ldv<SP, V>(e + c10) + w3 * ldv<SP, V>(e + c01) + w1 * ldv<SP, V>(e + c11);
  v1 = w9 * ldv<SP, V>(e + Nc + c00) + w3 * ldv<SP, V>(e + Nc + c10) + w3 * ldv<SP, V>(e + Nc + c01) +
       w1 * ldv<SP, V>(e + Nc + c11);
}

// One colour of a red-black 2x2-block Gauss-Seidel sweep: x_P = D_P^{-1}(b_P - sum_nb A_nb x_nb)
// for every cell with (i + j) % 2 == colour.
// MODE 0: plain pass.  MODE 1: x is zero on entry (first pass of a V-cycle level), so
// neighbours are not read.  MODE 2: first post-smoothing pass after the coarse-grid
// correction x += P e: the neighbours are read as x_Q + (P e)_Q on the fly.  The
// corrected values of this pass's own colour are never needed (the pass overwrites
// them) and those of the other colour are only read here (the next pass overwrites
// them), so the correction is never written back.  MODE 3: the second pass of a
// single pre-smoothing sweep from x = 0: the other colour's x is D^{-1} b there, and is
// formed on the fly from the neighbours' diagonal blocks and right-hand sides instead of
// being stored by a first pass (the next value of that colour is computed without it).
// SP > 1: SP adjacent samples per thread (a Map from make_map_wide), the same arithmetic
// lane by lane.
template <typename T, bool TR = false, int MODE = 0, int SP = 1>
__global__ void __launch_bounds__(256) k_gs_colour(Map m, Grid2 G, Grid2 Gc, int colour, const T* __restrict__ J,
                                                   const T* __restrict__ b, T* __restrict__ x,
                                                   const T* __restrict__ e) {
  typedef typename VecOf<T, SP>::type V;
  int s, mc, sb, cb;
  const int half = (G.nx + 1) >> 1;
  if (!map_cell_sp<SP>(m, G.ny * half, s, mc, sb, cb)) return;
  const int j = mc / half;
  const int i = 2 * (mc - j * half) + ((j + colour) & 1);
  if (i >= G.nx) return;
  const int S = m.S;
  const size_t N = (size_t)G.ncell * S;
  const size_t id = ((size_t)j * G.nx + i) * S + s;
  V r0 = ldv_nt<SP, V>(b + id), r1 = ldv_nt<SP, V>(b + N + id);
  if (MODE == 0) {
    V a0, a1;
    apply_row<T, V, TR, SP>(J, x, N, id, i, j, G.nx, G.ny, S, a0, a1, true);
    r0 -= a0;
    r1 -= a1;
  } else if (MODE == 2) {
    const size_t Nc = (size_t)Gc.ncell * S;
    auto xv = [&](size_t q, int dir, V& x0, V& x1) {
      const int qi = i + (dir == 1 ? -1 : dir == 2 ? 1 : 0), qj = j + (dir == 3 ? -1 : dir == 4 ? 1 : 0);
      V v0, v1;
      prolong_at<T, SP, V>(e, Nc, S, s, qi, qj, Gc, v0, v1);
      x0 = ldv<SP, V>(x + q) + v0;
      x1 = ldv<SP, V>(x + N + q) + v1;
    };
    V a0, a1;
    apply_row_f<T, V, TR, SP>(J, xv, N, id, i, j, G.nx, G.ny, S, a0, a1, true);
    r0 -= a0;
    r1 -= a1;
  } else if (MODE == 3) {
    auto xv = [&](size_t q, int, V& x0, V& x1) {
      const V q00 = ldv<SP, V>(J + q), q11 = ldv<SP, V>(J + 3 * N + q);
      const V q01 = TR ? ldv<SP, V>(J + 2 * N + q) : ldv<SP, V>(J + N + q);
      const V q10 = TR ? ldv<SP, V>(J + N + q) : ldv<SP, V>(J + 2 * N + q);
      const V c0 = ldv<SP, V>(b + q), c1 = ldv<SP, V>(b + N + q);
      const V qdet = q00 * q11 - q01 * q10;
      x0 = (q11 * c0 - q01 * c1) / qdet;
      x1 = (q00 * c1 - q10 * c0) / qdet;
    };
    V a0, a1;
    apply_row_f<T, V, TR, SP>(J, xv, N, id, i, j, G.nx, G.ny, S, a0, a1, true);
    r0 -= a0;
    r1 -= a1;
  }
  const V d00 = ldv_nt<SP, V>(J + id), d11 = ldv_nt<SP, V>(J + 3 * N + id);
  const V j1 = ldv_nt<SP, V>(J + N + id), j2 = ldv_nt<SP, V>(J + 2 * N + id);
  const V d01 = TR ? j2 : j1, d10 = TR ? j1 : j2;
  const V det = d00 * d11 - d01 * d10;
  stv<SP>(x + id, (d11 * r0 - d01 * r1) / det);
  stv<SP>(x + N + id, (d00 * r1 - d10 * r0) / det);
}

// Fused residual and restriction: b_H(I,J) = sum over the 2x2 children of (b - A x).
// red_only: the last smoothing pass was the black one, which leaves a zero residual
// on black cells, so only the two red children are evaluated.  red_only == 2: in
// addition the red cells hold x = D^{-1} b (one pre-smoothing sweep from x = 0, its
// red half never stored), so their residual is minus the off-diagonal part alone.
template <typename T, bool TR = false, int SP = 1>
__global__ void __launch_bounds__(256) k_residual_restrict(Map m, Grid2 Gf, Grid2 Gc, int red_only,
                                                           const T* __restrict__ J, const T* __restrict__ b,
                                                           const T* __restrict__ x, T* __restrict__ bH) {
  typedef typename VecOf<T, SP>::type V;
  int s, cc, sb, cb;
  if (!map_cell_sp<SP>(m, Gc.ncell, s, cc, sb, cb)) return;
  const int S = m.S;
  const size_t Nf = (size_t)Gf.ncell * S, Nc = (size_t)Gc.ncell * S;
  const int Jc = cc / Gc.nx, Ic = cc - Jc * Gc.nx;
  V s0 = 0, s1 = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 2 * Ic + (q & 1), j = 2 * Jc + (q >> 1);
    if (red_only && ((i + j) & 1)) continue;
    const size_t id = ((size_t)j * Gf.nx + i) * S + s;
    V a0, a1;
    if (red_only == 2) {
      apply_row<T, V, TR, SP>(J, x, Nf, id, i, j, Gf.nx, Gf.ny, S, a0, a1, true);
      s0 -= a0;
      s1 -= a1;
    } else {
      apply_row<T, V, TR, SP>(J, x, Nf, id, i, j, Gf.nx, Gf.ny, S, a0, a1, false);
      s0 += ldv<SP, V>(b + id) - a0;
      s1 += ldv<SP, V>(b + Nf + id) - a1;
    }
  }
  const size_t idc = (size_t)cc * S + s;
  stv<SP>(bH + idc, s0);
  stv<SP>(bH + Nc + idc, s1);
}

// Prolongation and correction x += P e (used only when there is no post-smoothing pass
// to fuse it into).
template <typename T, int SP = 1>
__global__ void __launch_bounds__(256) k_prolong_correct(Map m, Grid2 Gf, Grid2 Gc, const T* __restrict__ e,
                                                         T* __restrict__ x) {
  typedef typename VecOf<T, SP>::type V;
  int s, cell, sb, cb;
  if (!map_cell_sp<SP>(m, Gf.ncell, s, cell, sb, cb)) return;
  const int S = m.S;
  const size_t Nf = (size_t)Gf.ncell * S, Nc = (size_t)Gc.ncell * S;
  const int j = cell / Gf.nx, i = cell - j * Gf.nx;
  const size_t id = (size_t)cell * S + s;
  V v0, v1;
  prolong_at<T, SP, V>(e, Nc, S, s, i, j, Gc, v0, v1);
  stv<SP>(x + id, ldv<SP, V>(x + id) + v0);
  stv<SP>(x + Nf + id, ldv<SP, V>(x + Nf + id) + v1);
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
enum { SC_RHO = 0, SC_ALPHA, SC_OMEGA, SC_BETA, SC_R0, SC_RNORM, SC_ACTIVE, SC_ITS, SC_HALF, SC_NSLOT };

// r = sign * R (zero for samples with ndone[s] set; ndone may be NULL), rhat = r, p = r; partial |r|^2
// b = sign * R (0 for samples flagged in ndone); r0 = b - A x0, where A x0 is given in ax
// (warm start) or x0 = 0 (ax == nullptr).  Writes p = r0 (the first iteration reads r0
// from p) and, unless rhat is NULL (the caller uses R itself as the shadow residual),
// rhat = r0.  Partials |r0|^2 and |b|^2.
__global__ void __launch_bounds__(256) k_bicg_init(Map m, int ncell, const double* __restrict__ R, double sign,
                                                   const double* __restrict__ ax, const int* __restrict__ ndone,
                                                   double* __restrict__ rhat, double* __restrict__ p,
                                                   double* __restrict__ part) {
  __shared__ double lds[2 * 256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  const size_t N = (size_t)ncell * m.S;
  double acc[2] = {0.0, 0.0};
  const bool act = sv && !(ndone && ndone[s]);
  const double msk = act ? sign : 0.0;
  for (int k = 0; k < m.CPT; ++k) {
    const int cell = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || cell >= ncell) continue;
    const size_t id = (size_t)cell * m.S + s;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
      const double b = R[comp * N + id] * msk;
      const double v = ax && act ? b - ax[comp * N + id] : b;
      if (rhat) rhat[comp * N + id] = v;
      p[comp * N + id] = v;     // first search direction p0 = r0
      acc[0] += v * v;
      acc[1] += b * b;
    }
  }
  block_sum_y<2>(acc, lds);
  if (threadIdx.y == 0 && sv) {
    part[(size_t)cblk * m.S + s] = acc[0];
    part[((size_t)m.ncb + cblk) * m.S + s] = acc[1];
  }
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

// y = A x with per-sample partial dot products: NDOT = 1: (d0, y); NDOT = 2: (y, d0), (y, y).
// yb (or NULL): when x is the output of a V-cycle whose last pass on this grid was the black
// Gauss-Seidel pass, that pass solved the black rows exactly, (A x)_black = b_black with b the
// cycle's right-hand side; y takes yb there (equal up to rounding, or up to the rounding of
// the Jacobian for an FP32 cycle) and only red rows are multiplied out.
// TJ: the Jacobian's storage precision (FP32 for the Newton systems of the FP32-multigrid
// path, whose forward solves keep only the FP32 copy); TX: that of x (FP32 when x is the
// output of an FP32 multigrid cycle); y and the sums are FP64.
template <int NDOT, bool TR = false, typename TJ = double, typename TX = double>
__global__ void __launch_bounds__(256) k_spmv_dot(Map m, Grid2 G, const TJ* __restrict__ J,
                                                  const TX* __restrict__ x, double* __restrict__ y,
                                                  const double* __restrict__ d0, double* __restrict__ part,
                                                  const double* __restrict__ yb) {
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
    if (yb && ((i + j) & 1)) {
      y0 = yb[id];
      y1 = yb[N + id];
    } else {
      auto xv = [&](size_t q, int, double& x0, double& x1) {
        x0 = (double)x[q];
        x1 = (double)x[N + q];
      };
      apply_row_f<TJ, double, TR>(J, xv, N, id, i, j, G.nx, G.ny, m.S, y0, y1, false);
    }
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
                                                double* __restrict__ sv_, double* __restrict__ part) {
  __shared__ double lds[256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool ok = s < m.S;
  const size_t N = (size_t)ncell * m.S;
  const double al = ok ? sc[SC_ALPHA * m.S + s] : 0.0;
  double acc[1] = {0.0};
  for (int k = 0; k < m.CPT; ++k) {
    const int cell = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!ok || cell >= ncell) continue;
    const size_t id = (size_t)cell * m.S + s;
    const double s0 = r[id] - al * v[id], s1 = r[N + id] - al * v[N + id];
    sv_[id] = s0;
    sv_[N + id] = s1;
    acc[0] += s0 * s0 + s1 * s1;
  }
  block_sum_y<1>(acc, lds);
  if (threadIdx.y == 0 && ok) part[(size_t)cblk * m.S + s] = acc[0];
}

// x += alpha ph + omega sh (first iteration: x = alpha ph + omega sh, x0 = 0 is never
// stored); r = s - omega t; partials (rhat, r), (r, r).  TP: precision of the preconditioned
// directions ph, sh (FP32 straight from an FP32 multigrid cycle; the sums are FP64).
template <typename TP = double>
__global__ void __launch_bounds__(256) k_bicg_xr(Map m, int ncell, int first, const double* __restrict__ sc,
                                                 const TP* __restrict__ ph, const TP* __restrict__ sh,
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
      // omega == 0 (half-step exit or inactive): s-hat and t may be stale, do not read them
      const double dx = om != 0.0 ? al * (double)ph[q] + om * (double)sh[q] : al * (double)ph[q];
      x[q] = first ? dx : x[q] + dx;
      const double rv = om != 0.0 ? sv_[q] - om * t[q] : sv_[q];
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

// Finalisation kernels: 64 * FIN_Y threads per block, blockDim.x samples by blockDim.y
// threads that share each sample's partial sums (fewer samples per block, more threads per
// sample for small batches).  ctrl[0] counts active samples.
constexpr int FIN_Y = 16;

// nhist (Newton systems only, else NULL): per sample [size of the last undamped update
// (0: none), |R|^2 of the previous iterate].  A sample whose predicted next update
// size * |R_k| / |R_{k-1}| is <= pred_tol is declared converged without solving.
__global__ void __launch_bounds__(64 * FIN_Y) k_fin_init(Map m, const double* __restrict__ part, double* __restrict__ sc,
                                                  int* __restrict__ ctrl, double* __restrict__ nhist,
                                                  int* __restrict__ ndone, double pred_tol, double rtol2,
                                                  double rhat_sign) {
  __shared__ double lds[2 * 64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[2];
  reduce_partials<2>(m, part, s, v, lds);
  if (threadIdx.y == 0 && s < m.S) {
    const int S = m.S;
    sc[SC_RHO * S + s] = rhat_sign * v[0];   // (rhat, r0) with rhat = rhat_sign r0
    sc[SC_R0 * S + s] = v[1];           // the tolerance is relative to |b| (= |r0| from x0 = 0)
    sc[SC_RNORM * S + s] = v[0];
    sc[SC_ALPHA * S + s] = 0.0;
    sc[SC_OMEGA * S + s] = 0.0;
    sc[SC_BETA * S + s] = 0.0;
    int act = v[0] > 0.0 && v[0] > rtol2 * v[1];
    if (nhist && act) {
      const double last = nhist[2 * s], r2prev = nhist[2 * s + 1];
      if (pred_tol > 0.0 && last > 0.0 && r2prev > 0.0 && last * sqrt(v[0] / r2prev) <= pred_tol) {
        act = 0;
        ndone[s] = 1;
      }
      nhist[2 * s + 1] = v[0];
    }
    if (nhist && !ndone[s]) atomicAdd(&ctrl[1], 1);   // Newton samples still iterating
    sc[SC_ACTIVE * S + s] = act;
    sc[SC_ITS * S + s] = 0.0;
    if (act) atomicAdd(&ctrl[0], 1);
  }
}

__global__ void __launch_bounds__(64 * FIN_Y) k_fin_alpha(Map m, const double* __restrict__ part,
                                                          double* __restrict__ sc, double breakdown,
                                                          int* __restrict__ status) {
  __shared__ double lds[64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[1];
  reduce_partials<1>(m, part, s, v, lds);
  if (threadIdx.y == 0 && s < m.S) {
    const int S = m.S;
    double al = 0.0;
    if (sc[SC_ACTIVE * S + s] != 0.0) {
      const double rho = sc[SC_RHO * S + s];
      if (v[0] != 0.0 && isfinite(v[0]) && !(fabs(v[0]) <= breakdown * fabs(rho))) {
        al = rho / v[0];
      } else {
        sc[SC_ACTIVE * S + s] = 0.0;   // (near) breakdown: (rhat, A p) = 0 or |alpha| >= 1/breakdown
        if (status) status[s] = 2;
      }
    }
    sc[SC_ALPHA * S + s] = al;
  }
}

// Half-step test: a sample whose |s| already meets the tolerance stops after the
// alpha update (omega = 0 makes the rest of the iteration a no-op for it).  ctrl[0]
// counts samples that still need the second half.
__global__ void __launch_bounds__(64 * FIN_Y) k_fin_half(Map m, const double* __restrict__ part,
                                                         double* __restrict__ sc, double rtol2, int* __restrict__ ctrl) {
  __shared__ double lds[64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[1];
  reduce_partials<1>(m, part, s, v, lds);
  if (threadIdx.y == 0 && s < m.S) {
    const int S = m.S;
    int half = 0;
    if (sc[SC_ACTIVE * S + s] != 0.0) {
      if (v[0] <= rtol2 * sc[SC_R0 * S + s]) {
        half = 1;
        sc[SC_OMEGA * S + s] = 0.0;
      } else {
        atomicAdd(&ctrl[0], 1);
      }
    }
    sc[SC_HALF * S + s] = half;
  }
}

__global__ void __launch_bounds__(64 * FIN_Y) k_fin_omega(Map m, const double* __restrict__ part,
                                                          double* __restrict__ sc) {
  __shared__ double lds[2 * 64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[2];
  reduce_partials<2>(m, part, s, v, lds);
  if (threadIdx.y == 0 && s < m.S) {
    const int S = m.S;
    double om = 0.0;
    if (sc[SC_ACTIVE * S + s] != 0.0 && sc[SC_HALF * S + s] == 0.0 && v[1] > 0.0) om = v[0] / v[1];
    sc[SC_OMEGA * S + s] = om;
  }
}

__global__ void __launch_bounds__(64 * FIN_Y) k_fin_rho(Map m, const double* __restrict__ part,
                                                        double* __restrict__ sc, double rtol2, int* __restrict__ status,
                                                        int* __restrict__ ctrl) {
  __shared__ double lds[2 * 64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
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
      if (!(rr <= rtol2 * sc[SC_R0 * S + s]) && sc[SC_HALF * S + s] == 0.0) {
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
                                                           double* __restrict__ stats, int* __restrict__ ctrl,
                                                           double* __restrict__ nhist, double jac_reuse) {
  __shared__ double lds[2 * 64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
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
  nhist[2 * s] = mc > dc_max ? 0.0 : size;   // no prediction after a damped update
  if (size <= tol) {
    ndone[s] = 1;
  } else {
    atomicAdd(&ctrl[1], 1);
    if (!(size <= jac_reuse)) atomicAdd(&ctrl[2], 1);   // this sample wants a fresh Jacobian
  }
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
      const double F = -(P.rho0 + P.drho * P.c_left) * uin[s] * P.uin_fac * P.hy;
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
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
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

// Q = sum over cells with centre x > qoi_xmin of c rho(c) h^2 (partials)
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
    if ((i + 0.5) * P.hx > P.qoi_xmin) {
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
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double a[1];
  reduce_partials<1>(m, part, s, a, lds);
  if (threadIdx.y == 0 && s < m.S) out[s] = a[0] * scale;
}

}  // namespace henry
