// The paper's vertex-centred finite-volume discretisation (section 2.3): unknowns at the vertices
// of the element grid, boxes around vertices, fluxes through the four box faces inside each
// element, partial upwind for the convective salt flux.  Batched over samples: vectors are
// [component][vertex][S] with vertex v = j (nx + 1) + i, the Jacobian is [36][vertex][S] of
// 2x2 blocks for the 3 x 3 vertices around v, block b = (dj + 1) * 3 + (di + 1) (4 = centre),
// entry [b * 4 + a * 2 + k] = d R^a_v / d u^k_{v + (di, dj)} (a, k: 0 pressure, 1 concentration).
#pragma once

#include <hip/hip_runtime.h>

namespace henry {

constexpr int VC_BLK = 9;
// VC_LAST: size of the sample's last undamped Newton update in this step (0: none); VC_R2P: |R|^2
// of its previous Newton iterate (the predictive stop of k_vc_bicg_start)
enum { VC_RHO = 0, VC_ALPHA, VC_OMEGA, VC_R0, VC_ACTIVE, VC_ITS, VC_NEWTON, VC_DONE, VC_LAST, VC_R2P, VC_NSC };

// Element faces: face f separates local vertices a -> b (0 = (i, j), 1 = (i+1, j),
// 2 = (i+1, j+1), 3 = (i, j+1)), is crossed along +x (axis 0) or +y (axis 1), and has its
// integration point at local (s, t).
__device__ __forceinline__ void vc_face_geom(int f, int& a, int& b, int& axis, double& s, double& t) {
  switch (f) {
    case 0: a = 0; b = 1; axis = 0; s = 0.5; t = 0.25; break;
    case 1: a = 1; b = 2; axis = 1; s = 0.75; t = 0.5; break;
    case 2: a = 3; b = 2; axis = 0; s = 0.5; t = 0.75; break;
    default: a = 0; b = 3; axis = 1; s = 0.25; t = 0.5; break;
  }
}

// Fluid and salt mass flux a -> b through face f of one element and their derivatives with
// respect to p_k, c_k of the element's four vertices (the upwind fraction w included).
__device__ __forceinline__ void vc_face(int f, const double (&pk)[4], const double (&ck)[4], double Ke, double phie,
                                        const Phys& P, double& F, double& G, double (&dFp)[4], double (&dFc)[4],
                                        double (&dGp)[4], double (&dGc)[4]) {
  int a, b, axis;
  double s, t;
  vc_face_geom(f, a, b, axis, s, t);
  const double N[4] = {(1 - s) * (1 - t), s * (1 - t), s * t, (1 - s) * t};
  double dN[4];
  if (axis == 0) {
    dN[0] = -(1 - t) / P.hx; dN[1] = (1 - t) / P.hx; dN[2] = t / P.hx; dN[3] = -t / P.hx;
  } else {
    dN[0] = -(1 - s) / P.hy; dN[1] = -s / P.hy; dN[2] = s / P.hy; dN[3] = (1 - s) / P.hy;
  }
  const double L = axis == 0 ? 0.5 * P.hy : 0.5 * P.hx;
  const double h = axis == 0 ? P.hx : P.hy;
  double r = 0.0, gp = 0.0, gc = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r += N[k] * (P.rho0 + P.drho * ck[k]);
    gp += pk[k] * dN[k];
    gc += ck[k] * dN[k];
  }
  const double kk = Ke / P.mu;
  const double qn = -kk * (gp + (axis == 1 ? r * P.g : 0.0));
  F = r * qn * L;
  const double Df = r * phie * P.Dm * L / h;
  const double aF = fabs(F);
  double w = 0.0;
  if (aF > 0.0) w = fmax(0.0, 1.0 - 2.0 * Df / aF);
  const bool upa = F >= 0.0;
  const int up = upa ? a : b;
  const double cup = ck[up], cm = 0.5 * (ck[a] + ck[b]);
  const double cconv = cm + w * (cup - cm);
  G = F * cconv - r * phie * P.Dm * gc * L;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    dFp[k] = r * L * (-kk * dN[k]);
    dFc[k] = L * (N[k] * P.drho * qn + r * (axis == 1 ? -kk * P.g * N[k] * P.drho : 0.0));
    double dwp = 0.0, dwc = 0.0;
    if (w > 0.0) {
      const double sg = F > 0.0 ? 1.0 : -1.0;
      const double dDf = N[k] * P.drho * phie * P.Dm * L / h;
      dwp = 2.0 * Df * sg * dFp[k] / (F * F);
      dwc = -2.0 * dDf / aF + 2.0 * Df * sg * dFc[k] / (F * F);
    }
    const double dcc_c = ((k == a || k == b) ? 0.5 * (1.0 - w) : 0.0) + (k == up ? w : 0.0) + (cup - cm) * dwc;
    const double dcc_p = (cup - cm) * dwp;
    const double dGd_c = phie * P.Dm * L * (N[k] * P.drho * gc + r * dN[k]);
    dGp[k] = dFp[k] * cconv + F * dcc_p;
    dGc[k] = dFc[k] * cconv + F * dcc_c - dGd_c;
  }
}

// Residual (and Jacobian) of one implicit-Euler step at every vertex: a thread per (vertex,
// sample) gathers the two faces of each element around its vertex that bound its box.
// E: the element grid; phi, K: [element][S]; uin: [S] (times P.uin_fac).
// TJ: the Jacobian's storage type (float for the FP32 multigrid and its Krylov products)
template <bool WRITE_J, typename TJ = double>
__global__ void __launch_bounds__(256) k_vc_assemble(Map m, Grid2 E, Phys P, const double* __restrict__ phi,
                                                     const double* __restrict__ K, const double* __restrict__ uin,
                                                     const double* __restrict__ p, const double* __restrict__ c,
                                                     const double* __restrict__ c_old, double* __restrict__ R,
                                                     TJ* __restrict__ J) {
  const int nvx = E.nx + 1, nvy = E.ny + 1, nv = nvx * nvy;
  int s, v, sb, cb;
  if (!map_cell(m, nv, s, v, sb, cb)) return;
  const int S = m.S;
  const size_t NV = (size_t)nv * S;
  const int j = v / nvx, i = v - j * nvx;
  const size_t id = (size_t)v * S + s;
  const double y = -P.Ly + j * P.hy;
  double Jb[36];
#pragma unroll
  for (int q = 0; q < 36; ++q) Jb[q] = 0.0;
  double Rp = 0.0, Rc = 0.0;
  if (i == E.nx) {   // seaside: p = -rho1 g y, c = 1
    Rp = p[id] + P.rho1 * P.g * y;
    Rc = c[id] - 1.0;
    Jb[16] = 1.0;
    Jb[19] = 1.0;
  } else {
    double pn[3][3], cn[3][3];
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int qi = i + di, qj = j + dj;
        const bool in = qi >= 0 && qi < nvx && qj >= 0 && qj < nvy;
        const size_t q = ((size_t)(in ? qj : j) * nvx + (in ? qi : i)) * S + s;
        pn[dj + 1][di + 1] = in ? p[q] : 0.0;
        cn[dj + 1][di + 1] = in ? c[q] : 0.0;
      }
    // every load of the vertex is issued here, before any arithmetic: the four elements'
    // phi and K (an element outside the grid reads element 0 of the sample and is skipped
    // below), the old concentration and the sample's inflow.  Issued where they are used,
    // each would be a separate trip to memory, and at two wavefronts per SIMD little of
    // that latency is hidden.
    double phi_e[4], K_e[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int xi = i + (t & 1) - 1, xj = j + (t >> 1) - 1;
      const bool ok = xi >= 0 && xi < E.nx && xj >= 0 && xj < E.ny;
      const size_t e = ok ? ((size_t)xj * E.nx + xi) * S + s : (size_t)s;
      phi_e[t] = phi[e];
      K_e[t] = K[e];
    }
    const double co = c_old[id];
    const double u_in = uin[s];
    double box = 0.0;
#pragma unroll
    for (int ej = -1; ej <= 0; ++ej)
#pragma unroll
      for (int ei = -1; ei <= 0; ++ei) {
        const int xi = i + ei, xj = j + ej;
        if (xi < 0 || xi >= E.nx || xj < 0 || xj >= E.ny) continue;
        const int t = (ej + 1) * 2 + (ei + 1);
        const double phie = phi_e[t], Ke = K_e[t];
        box += 0.25 * P.hx * P.hy * phie;
        const int kv = ei == 0 ? (ej == 0 ? 0 : 3) : (ej == 0 ? 1 : 2);   // local index of v
        double pk[4], ck[4];
        int dik[4], djk[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          dik[k] = ei + ((k == 1 || k == 2) ? 1 : 0);
          djk[k] = ej + ((k == 2 || k == 3) ? 1 : 0);
          pk[k] = pn[djk[k] + 1][dik[k] + 1];
          ck[k] = cn[djk[k] + 1][dik[k] + 1];
        }
        // the two faces of this element that touch local vertex kv
        const int f0 = kv == 0 ? 0 : kv == 1 ? 0 : kv == 2 ? 1 : 2;
        const int f1 = kv == 0 ? 3 : kv == 1 ? 1 : kv == 2 ? 2 : 3;
#pragma unroll
        for (int ff = 0; ff < 2; ++ff) {
          const int f = ff == 0 ? f0 : f1;
          int a, b, axis;
          double s_, t_;
          vc_face_geom(f, a, b, axis, s_, t_);
          const double sgn = a == kv ? 1.0 : -1.0;   // out of v's box
          double F, G, dFp[4], dFc[4], dGp[4], dGc[4];
          vc_face(f, pk, ck, Ke, phie, P, F, G, dFp, dFc, dGp, dGc);
          Rp += sgn * F;
          Rc += sgn * G;
          if (WRITE_J) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int bl = (djk[k] + 1) * 3 + (dik[k] + 1);
              Jb[bl * 4 + 0] += sgn * dFp[k];
              Jb[bl * 4 + 1] += sgn * dFc[k];
              Jb[bl * 4 + 2] += sgn * dGp[k];
              Jb[bl * 4 + 3] += sgn * dGc[k];
            }
          }
        }
      }
    const double cv = cn[1][1];
    Rp += box * (P.drho * (cv - co)) / P.tau;
    Rc += box * ((P.rho0 + P.drho * cv) * cv - (P.rho0 + P.drho * co) * co) / P.tau;
    Jb[17] += box * P.drho / P.tau;
    Jb[19] += box * (P.rho0 + 2.0 * P.drho * cv) / P.tau;
    if (i == 0) {   // inflow side: mass flux rho(c_left) u_in enters; c = c_left
      const double len = (j == 0 || j == E.ny) ? 0.5 * P.hy : P.hy;
      Rp -= (P.rho0 + P.drho * P.c_left) * u_in * P.uin_fac * len;
      Rc = cv - P.c_left;
#pragma unroll
      for (int bl = 0; bl < VC_BLK; ++bl) {
        Jb[bl * 4 + 2] = 0.0;
        Jb[bl * 4 + 3] = 0.0;
      }
      Jb[19] = 1.0;
    }
  }
  R[id] = Rp;
  R[NV + id] = Rc;
  if (WRITE_J) {
#pragma unroll
    for (int q = 0; q < 36; ++q) J[(size_t)q * NV + id] = (TJ)Jb[q];
  }
}

// y = J x (9 blocks), one thread per (vertex, sample); J stored as TJ, the product in FP64
template <typename TJ>
__global__ void __launch_bounds__(256) k_vc_spmv(Map m, Grid2 E, const TJ* __restrict__ J,
                                                 const double* __restrict__ x, double* __restrict__ y) {
  const int nvx = E.nx + 1, nvy = E.ny + 1, nv = nvx * nvy;
  int s, v, sb, cb;
  if (!map_cell(m, nv, s, v, sb, cb)) return;
  const int S = m.S;
  const size_t NV = (size_t)nv * S;
  const int j = v / nvx, i = v - j * nvx;
  const size_t id = (size_t)v * S + s;
  double y0 = 0.0, y1 = 0.0;
  // all nine blocks' loads first, as in k_vc_gs (absent neighbours read the vertex's own
  // data and are selected away)
  double xa[9], xb[9];
  TJ jb[9][4];
  bool use[9];
#pragma unroll
  for (int bl = 0; bl < 9; ++bl) {
    const int qi = i + bl % 3 - 1, qj = j + bl / 3 - 1;
    use[bl] = qi >= 0 && qi < nvx && qj >= 0 && qj < nvy;
    const size_t q = use[bl] ? ((size_t)qj * nvx + qi) * S + s : id;
    const size_t jo = (size_t)(use[bl] ? bl * 4 : 16) * NV + id;
    xa[bl] = x[q];
    xb[bl] = x[NV + q];
#pragma unroll
    for (int e = 0; e < 4; ++e) jb[bl][e] = J[jo + (size_t)e * NV];
  }
#pragma unroll
  for (int bl = 0; bl < 9; ++bl) {
    const double a0 = (double)jb[bl][0] * xa[bl] + (double)jb[bl][1] * xb[bl];
    const double a1 = (double)jb[bl][2] * xa[bl] + (double)jb[bl][3] * xb[bl];
    y0 += use[bl] ? a0 : 0.0;
    y1 += use[bl] ? a1 : 0.0;
  }
  y[id] = y0;
  y[NV + id] = y1;
}

// One colour ((i & 1) + 2 (j & 1)) of a four-colour block Gauss-Seidel sweep:
// x_v = D_v^{-1} (b_v - sum over the other 8 blocks A_vq x_q); vertices of one colour do not
// touch each other in the nine-point stencil.  The launch covers only the colour's vertices
// (i = 2 u_i + colour & 1, j = 2 u_j + colour >> 1): vc_colour_cells() of colour 0, the largest.
// FIRST: the first forward sweep (colours 0, 1, 2, 3) from x = 0, in which the colours after
// this one still hold zero: their blocks are skipped and x need not be cleared beforehand.
__host__ __device__ inline int vc_colour_cells(int nx, int ny, int colour) {
  return ((nx + 2 - (colour & 1)) >> 1) * ((ny + 2 - (colour >> 1)) >> 1);
}
template <bool FIRST, typename T>
__global__ void __launch_bounds__(256) k_vc_gs(Map m, Grid2 E, int colour, const T* __restrict__ J,
                                               const T* __restrict__ b, T* __restrict__ x) {
  const int nvx = E.nx + 1, nvy = E.ny + 1, nv = nvx * nvy;
  const int ci = colour & 1, cj = colour >> 1;
  const int nci = (nvx + 1 - ci) >> 1, ncj = (nvy + 1 - cj) >> 1;
  int s, u, sb, cb;
  if (!map_cell(m, nci * ncj, s, u, sb, cb)) return;
  const int uj = u / nci;
  const int i = 2 * (u - uj * nci) + ci, j = 2 * uj + cj;
  const int v = j * nvx + i;
  const int S = m.S;
  const size_t NV = (size_t)nv * S;
  const size_t id = (size_t)v * S + s;
  T r0 = b[id], r1 = b[NV + id];
  // Every neighbour's loads are issued before any is used: a block that is absent (outside
  // the grid) or still zero (FIRST) reads the vertex's own x and diagonal block instead,
  // addresses that are valid and cached, and its term is selected away (a select, so
  // whatever those values hold cannot leak in).  With a few wavefronts per SIMD, the nine
  // blocks' loads in flight together rather than one block's at a time decide the time.
  T xa[8], xb[8], jb[8][4];
  bool use[8];
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const int bl = n < 4 ? n : n + 1, di = bl % 3 - 1, dj = bl / 3 - 1;
    const int qi = i + di, qj = j + dj;
    use[n] = qi >= 0 && qi < nvx && qj >= 0 && qj < nvy &&
             !(FIRST && ((ci ^ (di & 1)) + 2 * (cj ^ (dj & 1))) > colour);
    const size_t q = use[n] ? ((size_t)qj * nvx + qi) * S + s : id;
    const size_t jo = (size_t)(use[n] ? bl * 4 : 16) * NV + id;
    xa[n] = x[q];
    xb[n] = x[NV + q];
#pragma unroll
    for (int e = 0; e < 4; ++e) jb[n][e] = J[jo + (size_t)e * NV];
  }
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const T a0 = jb[n][0] * xa[n] + jb[n][1] * xb[n], a1 = jb[n][2] * xa[n] + jb[n][3] * xb[n];
    r0 -= use[n] ? a0 : (T)0;
    r1 -= use[n] ? a1 : (T)0;
  }
  const T d00 = J[(size_t)16 * NV + id], d01 = J[(size_t)17 * NV + id];
  const T d10 = J[(size_t)18 * NV + id], d11 = J[(size_t)19 * NV + id];
  const T det = d00 * d11 - d01 * d10;
  x[id] = (d11 * r0 - d01 * r1) / det;
  x[NV + id] = (d00 * r1 - d10 * r0) / det;
}

// Partial sums over vertex blocks of NQ per-sample dot products sum_v (a_q . b_q) (both
// components), written as part[q][cell block][S] for reduce_partials.
struct VCPairs {
  const double* a[3];
  const double* b[3];
};
template <int NQ>
__global__ void __launch_bounds__(256) k_vc_dots(Map m, int nv, VCPairs ab, double* __restrict__ part) {
  __shared__ double lds[NQ * 256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  const size_t NV = (size_t)nv * m.S;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int k = 0; k < m.CPT; ++k) {
    const int v = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || v >= nv) continue;
    const size_t id = (size_t)v * m.S + s;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double* a = ab.a[q];
      const double* b = ab.b[q];
      acc[q] += a[id] * b[id] + a[NV + id] * b[NV + id];
    }
  }
  block_sum_y<NQ>(acc, lds);
  if (threadIdx.y == 0 && sv)
#pragma unroll
    for (int q = 0; q < NQ; ++q) part[((size_t)q * m.ncb + cblk) * m.S + s] = acc[q];
}

// Per-sample max |dp| and |dc| partials (for the Newton damping and stopping test)
__global__ void __launch_bounds__(256) k_vc_absmax(Map m, int nv, const double* __restrict__ d,
                                                   double* __restrict__ part) {
  __shared__ double lds[2 * 256];
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  const size_t NV = (size_t)nv * m.S;
  double acc[2] = {0.0, 0.0};
  for (int k = 0; k < m.CPT; ++k) {
    const int v = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || v >= nv) continue;
    const size_t id = (size_t)v * m.S + s;
    const double a = fabs(d[id]), b = fabs(d[NV + id]);
    acc[0] = (a > acc[0] || a != a) ? a : acc[0];
    acc[1] = (b > acc[1] || b != b) ? b : acc[1];
  }
  // block max over y (NaN wins)
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  lds[tid] = acc[0];
  lds[256 + tid] = acc[1];
  __syncthreads();
  if (threadIdx.y == 0) {
    for (int yy = 1; yy < (int)blockDim.y; ++yy) {
      const double a = lds[yy * blockDim.x + threadIdx.x], b = lds[256 + yy * blockDim.x + threadIdx.x];
      acc[0] = (a > acc[0] || a != a) ? a : acc[0];
      acc[1] = (b > acc[1] || b != b) ? b : acc[1];
    }
    if (sv) {
      part[(size_t)cblk * m.S + s] = acc[0];
      part[((size_t)m.ncb + cblk) * m.S + s] = acc[1];
    }
  }
}

// ---- BiCGStab per sample (right preconditioned, x0 = 0, r-hat = r0) -----------------------
// sc[q * S + s]: VC_RHO, VC_ALPHA, VC_OMEGA, VC_R0 (|r0|^2), VC_ACTIVE, VC_ITS; ctrl[0]: samples
// still iterating after the kernel.

// after dots (r, r): rho = |r0|^2, active where it is > 0
// Newton's predictive stop (pred_tol > 0): a sample whose predicted update, the last undamped
// update's size times |R_k| / |R_{k-1}|, is at most pred_tol is converged without this solve.
__global__ void k_vc_bicg_start(Map m, const double* __restrict__ part, double* __restrict__ sc,
                                int* __restrict__ ctrl, double pred_tol) {
  __shared__ double lds[64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[1];
  reduce_partials<1>(m, part, s, v, lds);
  if (threadIdx.y != 0 || s >= m.S) return;
  const int S = m.S;
  bool act = v[0] > 0.0 && isfinite(v[0]) && sc[VC_DONE * S + s] == 0.0;
  if (act && pred_tol > 0.0) {
    const double last = sc[VC_LAST * S + s], r2p = sc[VC_R2P * S + s];
    if (last > 0.0 && r2p > 0.0 && last * sqrt(v[0] / r2p) <= pred_tol) {
      act = false;
      sc[VC_DONE * S + s] = 1.0;
    }
    sc[VC_R2P * S + s] = v[0];
  }
  sc[VC_RHO * S + s] = v[0];
  sc[VC_R0 * S + s] = v[0];
  sc[VC_ACTIVE * S + s] = act ? 1.0 : 0.0;
  sc[VC_ALPHA * S + s] = 0.0;
  sc[VC_OMEGA * S + s] = 0.0;
  if (act) atomicAdd(&ctrl[0], 1);
}

// after dots (r-hat, v): alpha = rho / (r-hat, v); 0 (and inactive) on breakdown
__global__ void k_vc_bicg_alpha(Map m, const double* __restrict__ part, double* __restrict__ sc,
                                int* __restrict__ status) {
  __shared__ double lds[64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[1];
  reduce_partials<1>(m, part, s, v, lds);
  if (threadIdx.y != 0 || s >= m.S) return;
  const int S = m.S;
  double al = 0.0;
  if (sc[VC_ACTIVE * S + s] != 0.0) {
    if (v[0] != 0.0 && isfinite(v[0])) {
      al = sc[VC_RHO * S + s] / v[0];
    } else {
      sc[VC_ACTIVE * S + s] = 0.0;
      if (status[s] == 0) status[s] = 2;
    }
  }
  sc[VC_ALPHA * S + s] = al;
}

// after dots (s, s), (t, s), (t, t): omega (0 when s already meets the tolerance)
__global__ void k_vc_bicg_omega(Map m, const double* __restrict__ part, double* __restrict__ sc, double rtol2) {
  __shared__ double lds[3 * 64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[3];
  reduce_partials<3>(m, part, s, v, lds);
  if (threadIdx.y != 0 || s >= m.S) return;
  const int S = m.S;
  double om = 0.0;
  if (sc[VC_ACTIVE * S + s] != 0.0 && !(v[0] <= rtol2 * sc[VC_R0 * S + s]) && v[2] > 0.0) om = v[1] / v[2];
  sc[VC_OMEGA * S + s] = om;
  if (sc[VC_ACTIVE * S + s] != 0.0 && v[0] <= rtol2 * sc[VC_R0 * S + s]) sc[VC_ACTIVE * S + s] = 2.0;   // done
}

// after dots (r-hat, r), (r, r): convergence, beta; ctrl[0] counts samples still iterating
__global__ void k_vc_bicg_beta(Map m, const double* __restrict__ part, double* __restrict__ sc, double rtol2,
                               int* __restrict__ status, int* __restrict__ ctrl) {
  __shared__ double lds[2 * 64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double v[2];
  reduce_partials<2>(m, part, s, v, lds);
  if (threadIdx.y != 0 || s >= m.S) return;
  const int S = m.S;
  const double act = sc[VC_ACTIVE * S + s];
  if (act == 0.0) return;
  sc[VC_ITS * S + s] += 1.0;
  if (act == 2.0 || v[1] <= rtol2 * sc[VC_R0 * S + s]) {
    sc[VC_ACTIVE * S + s] = 0.0;
    return;
  }
  const double om = sc[VC_OMEGA * S + s];
  if (om == 0.0 || v[0] == 0.0 || !isfinite(v[0])) {
    sc[VC_ACTIVE * S + s] = 0.0;
    if (status[s] == 0) status[s] = 2;
    return;
  }
  sc[VC_ALPHA * S + s] = (v[0] / sc[VC_RHO * S + s]) * (sc[VC_ALPHA * S + s] / om);   // beta, kept in ALPHA
  sc[VC_RHO * S + s] = v[0];
  atomicAdd(&ctrl[0], 1);
}

// elementwise updates over [2][nv][S] with per-sample coefficients
__device__ __forceinline__ size_t vc_sample_of(size_t e, size_t NV, int S, int& s) {
  const size_t id = e < NV ? e : e - NV;
  s = (int)(id % (size_t)S);
  return id;
}

// s = r - alpha v
__global__ void k_vc_axpy_s(size_t n2, size_t NV, int S, const double* __restrict__ sc, const double* __restrict__ r,
                            const double* __restrict__ v, double* __restrict__ sv) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= n2) return;
  int s;
  vc_sample_of(e, NV, S, s);
  sv[e] = r[e] - sc[VC_ALPHA * S + s] * v[e];
}

// x += alpha p-hat + omega s-hat; r = s - omega t (samples that iterate)
__global__ void k_vc_update_xr(size_t n2, size_t NV, int S, const double* __restrict__ sc,
                               const double* __restrict__ ph, const double* __restrict__ sh,
                               const double* __restrict__ sv, const double* __restrict__ t, double* __restrict__ x,
                               double* __restrict__ r) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= n2) return;
  int s;
  vc_sample_of(e, NV, S, s);
  if (sc[VC_ACTIVE * S + s] == 0.0) return;
  const double al = sc[VC_ALPHA * S + s], om = sc[VC_OMEGA * S + s];
  x[e] += al * ph[e] + om * sh[e];
  r[e] = sv[e] - om * t[e];
}

// p = r + beta (p - omega v) for samples still iterating (beta kept in ALPHA)
__global__ void k_vc_update_p(size_t n2, size_t NV, int S, const double* __restrict__ sc,
                              const double* __restrict__ r, const double* __restrict__ v, double* __restrict__ p) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= n2) return;
  int s;
  vc_sample_of(e, NV, S, s);
  if (sc[VC_ACTIVE * S + s] == 0.0) return;
  p[e] = r[e] + sc[VC_ALPHA * S + s] * (p[e] - sc[VC_OMEGA * S + s] * v[e]);
}

// right-hand side b = -R for samples still in Newton (0 for converged ones); x = 0, r = p = b
__global__ void k_vc_rhs(size_t n2, size_t NV, int S, const double* __restrict__ sc, const double* __restrict__ R,
                         double* __restrict__ x, double* __restrict__ r, double* __restrict__ p,
                         double* __restrict__ rh) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= n2) return;
  int s;
  vc_sample_of(e, NV, S, s);
  const double b = sc[VC_DONE * S + s] != 0.0 ? 0.0 : -R[e];
  x[e] = 0.0;
  r[e] = b;
  p[e] = b;
  rh[e] = b;
}

// Newton: after |dp|_inf, |dc|_inf partials, damp by min(1, dc_max / |dc|_inf), stop on the
// unscaled update (as the oracle does); ctrl[0] counts samples still iterating.
__global__ void k_vc_newton_fin(Map m, const double* __restrict__ part, double* __restrict__ sc, double tol,
                                double p_ref, double dc_max, int* __restrict__ status, int* __restrict__ ctrl) {
  __shared__ double lds[2 * 64 * FIN_Y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  double e[2];
  reduce_partials_max<2>(m, part, s, e, lds);
  if (threadIdx.y != 0 || s >= m.S) return;
  const int S = m.S;
  if (sc[VC_DONE * S + s] != 0.0) {
    sc[VC_ALPHA * S + s] = 0.0;
    return;
  }
  const double dp = e[0], dc = e[1];
  if (!isfinite(dp) || !isfinite(dc)) {
    status[s] = 3;
    sc[VC_DONE * S + s] = 1.0;
    sc[VC_ALPHA * S + s] = 0.0;
    return;
  }
  sc[VC_ALPHA * S + s] = dc > 0.0 ? fmin(1.0, dc_max / dc) : 1.0;   // damping factor
  sc[VC_LAST * S + s] = dc > dc_max ? 0.0 : fmax(dc, dp / p_ref);     // no prediction after damping
  sc[VC_NEWTON * S + s] += 1.0;
  if (fmax(dc, dp / p_ref) <= tol) sc[VC_DONE * S + s] = 1.0;
  else atomicAdd(&ctrl[0], 1);
}

// p += lambda dp, c += lambda dc (lambda in ALPHA, 0 for samples that had converged)
__global__ void k_vc_newton_update(size_t NV, int S, const double* __restrict__ sc, const double* __restrict__ d,
                                   double* __restrict__ p, double* __restrict__ c) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= NV) return;
  const int s = (int)(e % (size_t)S);
  const double lam = sc[VC_ALPHA * S + s];
  p[e] += lam * d[e];
  c[e] += lam * d[NV + e];
}

// initial state: p = -rho0 g y (-rho1 g y on x = Lx), c = 0 (1 on x = Lx, c_left on x = 0)
__global__ void k_vc_init(Map m, Grid2 E, Phys P, double* __restrict__ p, double* __restrict__ c) {
  const int nvx = E.nx + 1, nv = nvx * (E.ny + 1);
  int s, v, sb, cb;
  if (!map_cell(m, nv, s, v, sb, cb)) return;
  const int j = v / nvx, i = v - j * nvx;
  const size_t id = (size_t)v * m.S + s;
  const double y = -P.Ly + j * P.hy;
  p[id] = -(i == E.nx ? P.rho1 : P.rho0) * P.g * y;
  c[id] = i == E.nx ? 1.0 : (i == 0 ? P.c_left : 0.0);
}

// QoI partials: sum_v c rho(c) |box_v n {x > qoi_xmin}|
__global__ void __launch_bounds__(256) k_vc_qoi(Map m, Grid2 E, Phys P, const double* __restrict__ c,
                                                double* __restrict__ part) {
  __shared__ double lds[256];
  const int nvx = E.nx + 1, nv = nvx * (E.ny + 1);
  const int sblk = blockIdx.x % m.nsb, cblk = blockIdx.x / m.nsb;
  const int s = sblk * m.SX + threadIdx.x;
  const bool sv = s < m.S;
  double acc[1] = {0.0};
  for (int k = 0; k < m.CPT; ++k) {
    const int v = (cblk * m.CPT + k) * m.CY + threadIdx.y;
    if (!sv || v >= nv) continue;
    const int j = v / nvx, i = v - j * nvx;
    const double x = i * P.hx;
    const double lo = fmax(x - 0.5 * P.hx, 0.0), hi = fmin(x + 0.5 * P.hx, P.Lx);
    const double wx = fmax(0.0, hi - fmax(lo, P.qoi_xmin));
    const double wy = (j == 0 || j == E.ny) ? 0.5 * P.hy : P.hy;
    const double cv = c[(size_t)v * m.S + s];
    acc[0] += cv * (P.rho0 + P.drho * cv) * wx * wy;
  }
  block_sum_y<1>(acc, lds);
  if (threadIdx.y == 0 && sv) part[(size_t)cblk * m.S + s] = acc[0];
}

// ---- geometric multigrid on the vertex grids ----------------------------------------------
// Coarse vertex (I, J) is fine vertex (2I, 2J); prolongation is bilinear interpolation and the
// residual restriction its transpose (weights 1, 1/2, 1/4: the mass residuals of the fine boxes
// are shared out to the coarse boxes they overlap, so their sum is kept).  Dirichlet components
// (both on x = Lx, c on x = 0) get no coarse right-hand side and no correction.

// r = b - J x
// zero_colour: the colour swept last, whose residual is zero up to rounding (its rows were
// just solved against the current neighbours): written as 0 without reading J
template <typename T>
__global__ void __launch_bounds__(256) k_vc_resid(Map m, Grid2 E, int zero_colour, const T* __restrict__ J,
                                                  const T* __restrict__ b, const T* __restrict__ x,
                                                  T* __restrict__ r) {
  const int nvx = E.nx + 1, nvy = E.ny + 1, nv = nvx * nvy;
  int s, v, sb, cb;
  if (!map_cell(m, nv, s, v, sb, cb)) return;
  const int S = m.S;
  const size_t NV = (size_t)nv * S;
  const int j = v / nvx, i = v - j * nvx;
  const size_t id = (size_t)v * S + s;
  if ((i & 1) + 2 * (j & 1) == zero_colour) {
    r[id] = 0;
    r[NV + id] = 0;
    return;
  }
  T y0 = b[id], y1 = b[NV + id];
  // all nine blocks' loads first, as in k_vc_gs (absent neighbours read the vertex's own
  // data and are selected away)
  T xa[9], xb[9], jb[9][4];
  bool use[9];
#pragma unroll
  for (int bl = 0; bl < 9; ++bl) {
    const int qi = i + bl % 3 - 1, qj = j + bl / 3 - 1;
    use[bl] = qi >= 0 && qi < nvx && qj >= 0 && qj < nvy;
    const size_t q = use[bl] ? ((size_t)qj * nvx + qi) * S + s : id;
    const size_t jo = (size_t)(use[bl] ? bl * 4 : 16) * NV + id;
    xa[bl] = x[q];
    xb[bl] = x[NV + q];
#pragma unroll
    for (int e = 0; e < 4; ++e) jb[bl][e] = J[jo + (size_t)e * NV];
  }
#pragma unroll
  for (int bl = 0; bl < 9; ++bl) {
    const T a0 = jb[bl][0] * xa[bl] + jb[bl][1] * xb[bl], a1 = jb[bl][2] * xa[bl] + jb[bl][3] * xb[bl];
    y0 -= use[bl] ? a0 : (T)0;
    y1 -= use[bl] ? a1 : (T)0;
  }
  r[id] = y0;
  r[NV + id] = y1;
}

// coarse right-hand side: full weighting of the fine residual (mc: the coarse grid's map)
template <typename T>
__global__ void __launch_bounds__(256) k_vc_restrict(Map mc, Grid2 Ec, Grid2 Ef, const T* __restrict__ rf,
                                                     T* __restrict__ bc) {
  const int nvxc = Ec.nx + 1, nvc = nvxc * (Ec.ny + 1);
  const int nvxf = Ef.nx + 1, nvyf = Ef.ny + 1;
  int s, v, sb, cb;
  if (!map_cell(mc, nvc, s, v, sb, cb)) return;
  const int S = mc.S;
  const size_t NVc = (size_t)nvc * S, NVf = (size_t)nvxf * nvyf * S;
  const int J = v / nvxc, I = v - J * nvxc;
  T a0 = 0, a1 = 0;
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
    for (int di = -1; di <= 1; ++di) {
      const int fi = 2 * I + di, fj = 2 * J + dj;
      if (fi < 0 || fi >= nvxf || fj < 0 || fj >= nvyf) continue;
      const T w = (T)((di == 0 ? 1.0 : 0.5) * (dj == 0 ? 1.0 : 0.5));
      const size_t q = ((size_t)fj * nvxf + fi) * S + s;
      a0 += w * rf[q];
      a1 += w * rf[NVf + q];
    }
  const size_t id = (size_t)v * S + s;
  bc[id] = I == Ec.nx ? (T)0 : a0;
  bc[NVc + id] = (I == Ec.nx || I == 0) ? (T)0 : a1;
}

// x_f += P x_c (bilinear), Dirichlet components untouched (mf: the fine grid's map)
template <typename T>
__global__ void __launch_bounds__(256) k_vc_prolong_add(Map mf, Grid2 Ef, Grid2 Ec, const T* __restrict__ xc,
                                                        T* __restrict__ xf) {
  const int nvxf = Ef.nx + 1, nvf = nvxf * (Ef.ny + 1);
  const int nvxc = Ec.nx + 1, nvc = nvxc * (Ec.ny + 1);
  int s, v, sb, cb;
  if (!map_cell(mf, nvf, s, v, sb, cb)) return;
  const int S = mf.S;
  const size_t NVf = (size_t)nvf * S, NVc = (size_t)nvc * S;
  const int j = v / nvxf, i = v - j * nvxf;
  if (i == Ef.nx) return;
  // the four (possibly coinciding) coarse vertices around (i, j), each with weight 1/4: a
  // coinciding vertex counted 4 or 2 times gives the bilinear weights 1 and 1/2
  const int I0 = i >> 1, J0 = j >> 1, I1 = I0 + (i & 1), J1 = J0 + (j & 1);
  const T w = (T)0.25;
  const size_t c00 = ((size_t)J0 * nvxc + I0) * S + s, c10 = ((size_t)J0 * nvxc + I1) * S + s;
  const size_t c01 = ((size_t)J1 * nvxc + I0) * S + s, c11 = ((size_t)J1 * nvxc + I1) * S + s;
  const T e0 = w * (xc[c00] + xc[c10] + xc[c01] + xc[c11]);
  const T e1 = w * (xc[NVc + c00] + xc[NVc + c10] + xc[NVc + c01] + xc[NVc + c11]);
  const size_t id = (size_t)v * S + s;
  xf[id] += e0;
  if (i != 0) xf[NVf + id] += e1;
}

// coarse state by injection (coarse vertex = fine vertex (2I, 2J))
__global__ void __launch_bounds__(256) k_vc_inject(Map mc, Grid2 Ec, Grid2 Ef, const double* __restrict__ pf,
                                                   const double* __restrict__ cf, const double* __restrict__ cof,
                                                   double* __restrict__ pc, double* __restrict__ cc,
                                                   double* __restrict__ coc) {
  const int nvxc = Ec.nx + 1, nvc = nvxc * (Ec.ny + 1);
  int s, v, sb, cb;
  if (!map_cell(mc, nvc, s, v, sb, cb)) return;
  const int J = v / nvxc, I = v - J * nvxc;
  const size_t q = ((size_t)(2 * J) * (Ef.nx + 1) + 2 * I) * mc.S + s, id = (size_t)v * mc.S + s;
  pc[id] = pf[q];
  cc[id] = cf[q];
  coc[id] = cof[q];
}

// coarse element fields: phi the mean, K the geometric mean of the four children
__global__ void __launch_bounds__(256) k_vc_coarse_fields(Map mce, Grid2 Ec, Grid2 Ef, const double* __restrict__ phif,
                                                          const double* __restrict__ Kf, double* __restrict__ phic,
                                                          double* __restrict__ Kc) {
  int s, e, sb, cb;
  if (!map_cell(mce, Ec.ncell, s, e, sb, cb)) return;
  const int J = e / Ec.nx, I = e - J * Ec.nx;
  double ph = 0.0, lk = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const size_t f = ((size_t)(2 * J + (q >> 1)) * Ef.nx + 2 * I + (q & 1)) * mce.S + s;
    ph += phif[f];
    lk += log(Kf[f]);
  }
  const size_t id = (size_t)e * mce.S + s;
  phic[id] = 0.25 * ph;
  Kc[id] = exp(0.25 * lk);
}

// Coarsest grid solved directly (Gaussian elimination with partial pivoting, section 2.3): the
// dense matrix of its n = 2 nv unknowns (unknown 2 v + component) per sample, held
// column-major in LDS (A[c n + r]).  The factors (P A = L U: L below the diagonal with its
// unit diagonal implied, U above it and the reciprocals of U's diagonal on it) go to global
// memory column-major once per Newton iteration with the row order perm (row i of P A is row
// perm[i] of A), and every V-cycle solves with them.  Lanes own rows l, l + 64 and l + 128.
// n <= VC_DENSE_MAX.
constexpr int VC_DENSE_MAX = 140;
constexpr int VC_DENSE_SLOTS = 3;   // rows per lane
static_assert(VC_DENSE_SLOTS == 3 && 64 * VC_DENSE_SLOTS >= VC_DENSE_MAX, "vc_slot selects among three slots");

// lane `lane`'s value of v (lane uniform across the wavefront)
__device__ __forceinline__ double vc_bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float vc_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
// the slot holding row r (r uniform); scalar arguments keep the slots in registers
template <typename T>
__device__ __forceinline__ T vc_slot(T v0, T v1, T v2, int r) {
  return r < 64 ? v0 : (r < 128 ? v1 : v2);
}

// Factorisation, one workgroup of four wavefronts per sample.  Wavefront w owns the columns
// c = w (mod 4).  Step k: every wavefront reads column k and finds the pivot row p (the first
// row of largest magnitude at or below the diagonal) and the multipliers itself; each swaps rows
// k and p in its own columns and updates its own trailing columns; one barrier ends the step,
// after which the owner of column k stores its multipliers (no wavefront reads column k again).
template <typename T>
__global__ void __launch_bounds__(256) k_vc_dense_factor(int S, Grid2 E, const T* __restrict__ J,
                                                         T* __restrict__ LU, int* __restrict__ perm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nvx = E.nx + 1, nvy = E.ny + 1, nv = nvx * nvy, n = 2 * nv;
  const int s = blockIdx.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const size_t NV = (size_t)nv * S;
  T* A = reinterpret_cast<T*>(smem_raw);   // A[c * n + r]
  int* pr = reinterpret_cast<int*>(A + (size_t)n * n);
  for (int e = t; e < n * n; e += 256) A[e] = 0;
  for (int r = t; r < n; r += 256) pr[r] = r;
  __syncthreads();
  // scatter the nine blocks of every vertex row, four independent loads in flight per thread
  for (int e0 = 0; e0 < nv * 36; e0 += 4 * 256) {
    T val[4];
    int dst[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * 256 + t;
      dst[u] = -1;
      val[u] = 0;
      if (e < nv * 36) {
        const int v = e / 36, q = e - v * 36, bl = q >> 2, a = (q >> 1) & 1, k = q & 1;
        const int i = v % nvx, j = v / nvx, qi = i + bl % 3 - 1, qj = j + bl / 3 - 1;
        if (qi >= 0 && qi < nvx && qj >= 0 && qj < nvy) {
          dst[u] = (2 * (qj * nvx + qi) + k) * n + 2 * v + a;
          val[u] = J[(size_t)q * NV + (size_t)v * S + s];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (dst[u] >= 0) A[dst[u]] = val[u];
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const T* Ak = A + (size_t)k * n;
    T ck[VC_DENSE_SLOTS];
    T vmax = -1;
#pragma unroll
    for (int q = 0; q < VC_DENSE_SLOTS; ++q) {
      const int r = lane + 64 * q;
      ck[q] = r < n ? Ak[r] : (T)0;
      if (r >= k && r < n) vmax = fmax(vmax, fabs(ck[q]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
    int p = k;
#pragma unroll
    for (int q = VC_DENSE_SLOTS - 1; q >= 0; --q) {   // the smallest row attaining the maximum
      const int r = lane + 64 * q;
      const unsigned long long hit = __ballot(r >= k && r < n && fabs(ck[q]) == vmax);
      if (hit) p = 64 * q + __ffsll((long long)hit) - 1;
    }
    const T akk = vc_bcast(vc_slot(ck[0], ck[1], ck[2], k), k & 63);
    const T apk = vc_bcast(vc_slot(ck[0], ck[1], ck[2], p), p & 63);
    const T rp = (T)1 / apk;
    T l[VC_DENSE_SLOTS];
    bool below[VC_DENSE_SLOTS];
#pragma unroll
    for (int q = 0; q < VC_DENSE_SLOTS; ++q) {   // multipliers of the interchanged column k
      const int r = lane + 64 * q;
      below[q] = r > k && r < n;
      l[q] = below[q] ? (r == p ? akk : ck[q]) * rp : (T)0;
    }
    if (p != k) {
      for (int c = w + 4 * lane; c < n; c += 256)   // interchange rows k and p in own columns
        if (c != k) {
          const T a = A[(size_t)c * n + k];
          A[(size_t)c * n + k] = A[(size_t)c * n + p];
          A[(size_t)c * n + p] = a;
        }
      if (t == 0) {
        const int a = pr[k];
        pr[k] = pr[p];
        pr[p] = a;
      }
    }
    // own trailing columns, four at a time: all their reads issued before any write, so the
    // LDS latency is paid once per four columns
    int c = k + 1 + ((w - k - 1) & 3);
    for (; c + 12 < n; c += 16) {
      T u[4], a[4][VC_DENSE_SLOTS];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const T* Ac = A + (size_t)(c + 4 * h) * n;
        u[h] = Ac[k];
#pragma unroll
        for (int q = 0; q < VC_DENSE_SLOTS; ++q) a[h][q] = below[q] ? Ac[lane + 64 * q] : (T)0;
      }
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        T* Ac = A + (size_t)(c + 4 * h) * n;
#pragma unroll
        for (int q = 0; q < VC_DENSE_SLOTS; ++q)
          if (below[q]) Ac[lane + 64 * q] = a[h][q] - l[q] * u[h];
      }
    }
    for (; c < n; c += 4) {
      T* Ac = A + (size_t)c * n;
      const T u = Ac[k];
#pragma unroll
      for (int q = 0; q < VC_DENSE_SLOTS; ++q)
        if (below[q]) Ac[lane + 64 * q] -= l[q] * u;
    }
    __syncthreads();
    if ((k & 3) == w) {   // U's diagonal is stored as its reciprocal, which the solve multiplies by
      T* Akw = A + (size_t)k * n;
#pragma unroll
      for (int q = 0; q < VC_DENSE_SLOTS; ++q) {
        const int r = lane + 64 * q;
        if (r == k) Akw[r] = rp;
        else if (below[q]) Akw[r] = l[q];
      }
    }
  }
  __syncthreads();
  for (int e = t; e < n * n; e += 256) LU[(size_t)s * n * n + e] = A[e];
  for (int r = t; r < n; r += 256) perm[(size_t)s * n + r] = pr[r];
}

// x = A^{-1} b with the factors of k_vc_dense_factor (both [2][nv][S] vectors), one wavefront
// per sample: the factors staged into LDS (a wavefront's LDS operations complete in issue
// order, so no barrier is needed), y = P b gathered into registers, then forward and back
// substitution column by column with the pivot row's value broadcast from its lane; each
// chunk of VC_SOLVE_CH columns is read from LDS ahead of its dependent steps.
constexpr int VC_SOLVE_CH = 8;
template <typename T>
__global__ void __launch_bounds__(64) k_vc_dense_solve(int S, Grid2 E, const T* __restrict__ LU,
                                                       const int* __restrict__ perm, const T* __restrict__ b,
                                                       T* __restrict__ x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nv = (E.nx + 1) * (E.ny + 1), n = 2 * nv;
  const int s = blockIdx.x, t = threadIdx.x;
  const size_t NV = (size_t)nv * S;
  T* A = reinterpret_cast<T*>(smem_raw);   // A[c * n + r]
  {   // n is even, so n^2 sizeof(T) is a multiple of 16 bytes and each sample's factors start
      // 16-byte aligned: staged in 16-byte chunks, 16 loads in flight per lane
    const uint4* src = reinterpret_cast<const uint4*>(LU + (size_t)s * n * n);
    uint4* dst = reinterpret_cast<uint4*>(A);
    const int n2 = (int)((size_t)n * n * sizeof(T) / 16);
    for (int e0 = 0; e0 < n2; e0 += 16 * 64) {
      uint4 v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = e0 + u * 64 + t;
        v[u] = e < n2 ? src[e] : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = e0 + u * 64 + t;
        if (e < n2) dst[e] = v[u];
      }
    }
  }
  T y[VC_DENSE_SLOTS];
#pragma unroll
  for (int q = 0; q < VC_DENSE_SLOTS; ++q) {
    const int r = t + 64 * q;
    y[q] = 0;
    if (r < n) {
      const int g = perm[(size_t)s * n + r];
      y[q] = b[(size_t)(g & 1) * NV + (size_t)(g >> 1) * S + s];
    }
  }
  __builtin_amdgcn_wave_barrier();
  for (int k0 = 0; k0 < n - 1; k0 += VC_SOLVE_CH) {   // L y = P b (unit lower)
    T a[VC_SOLVE_CH][VC_DENSE_SLOTS];
#pragma unroll
    for (int j = 0; j < VC_SOLVE_CH; ++j)
#pragma unroll
      for (int q = 0; q < VC_DENSE_SLOTS; ++q) {
        const int k = k0 + j, r = t + 64 * q;
        a[j][q] = (k < n - 1 && r > k && r < n) ? A[(size_t)k * n + r] : (T)0;
      }
#pragma unroll
    for (int j = 0; j < VC_SOLVE_CH; ++j) {
      const int k = k0 + j;
      if (k < n - 1) {
        const T yk = vc_bcast(vc_slot(y[0], y[1], y[2], k), k & 63);
#pragma unroll
        for (int q = 0; q < VC_DENSE_SLOTS; ++q)
          if (t + 64 * q > k) y[q] -= a[j][q] * yk;
      }
    }
  }
  for (int k0 = n - 1; k0 >= 0; k0 -= VC_SOLVE_CH) {   // U x = y
    T a[VC_SOLVE_CH][VC_DENSE_SLOTS], dk[VC_SOLVE_CH];
#pragma unroll
    for (int j = 0; j < VC_SOLVE_CH; ++j) {
      const int k = k0 - j;
      dk[j] = k >= 0 ? A[(size_t)k * n + k] : (T)1;   // 1 / U_kk
#pragma unroll
      for (int q = 0; q < VC_DENSE_SLOTS; ++q) {
        const int r = t + 64 * q;
        a[j][q] = (k >= 0 && r < k) ? A[(size_t)k * n + r] : (T)0;
      }
    }
#pragma unroll
    for (int j = 0; j < VC_SOLVE_CH; ++j) {
      const int k = k0 - j;
      if (k >= 0) {
        const T xk = vc_bcast(vc_slot(y[0], y[1], y[2], k), k & 63) * dk[j];
#pragma unroll
        for (int q = 0; q < VC_DENSE_SLOTS; ++q) {
          const int r = t + 64 * q;
          if (r == k) y[q] = xk;
          else if (r < k) y[q] -= a[j][q] * xk;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < VC_DENSE_SLOTS; ++q) {
    const int r = t + 64 * q;
    if (r < n) x[(size_t)(r & 1) * NV + (size_t)(r >> 1) * S + s] = y[q];
  }
}

// per-sample step bookkeeping (fin launch shape: threadIdx.y == 0 acts)
__global__ void k_vc_step_start(int S, const int* __restrict__ status, double* __restrict__ sc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.y != 0 || s >= S) return;
  sc[VC_DONE * S + s] = status[s] == 3 ? 1.0 : 0.0;   // a frozen (non-finite) sample stays frozen
  sc[VC_LAST * S + s] = 0.0;                          // no prediction before a step's first update
  sc[VC_R2P * S + s] = 0.0;
}
__global__ void k_vc_step_end(int S, int* __restrict__ status, const double* __restrict__ sc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.y != 0 || s >= S) return;
  if (sc[VC_DONE * S + s] == 0.0 && status[s] == 0) status[s] = 1;   // Newton did not converge
}
// stats[s][0..1]: Newton and BiCGStab iterations over the run
__global__ void k_vc_stats(int S, const double* __restrict__ sc, double* __restrict__ stats) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.y != 0 || s >= S) return;
  stats[2 * (size_t)s] = sc[VC_NEWTON * S + s];
  stats[2 * (size_t)s + 1] = sc[VC_ITS * S + s];
}

}  // namespace henry
