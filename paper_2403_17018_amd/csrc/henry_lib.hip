// libhenry: host runtime and C ABI of the batched Henry / MLMC solver (gfx950).
//
// The host side only sequences kernels: the time loop, Newton iterations and the
// BiCGStab/multigrid schedule.  Every arithmetic step on the data runs in the HIP
// kernels of henry_kernels.hpp and henry_mlmc.hpp.  Per-sample control decisions
// (damping, convergence, breakdown) are taken on the device; the host reads one
// counter per iteration to decide whether to launch another.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <atomic>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/henry.h"
#include "henry_kernels.hpp"
#include "henry_coarse.hpp"
#include "henry_dense.hpp"
#include "henry_gbsv.hpp"
#include "henry_mlmc.hpp"
#include "henry_adjoint.hpp"
#include "henry_vc.hpp"

using namespace henry;

// A roctx range for the lifetime of the object (rocprofv3 --marker-trace shows them): one per
// solve call, per grid of a ragged call, per forward time step and per reverse adjoint step.
// Ranges nest per host thread; without a tool attached the calls return at once.
struct Range {
  explicit Range(const char* fmt, ...) {
    char b[112];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(b, sizeof b, fmt, ap);
    va_end(ap);
    roctxRangePushA(b);
  }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct HenryError {
  int code;
  std::string msg;
};

#define HIPCHK(call)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      throw HenryError{HENRY_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)};          \
  } while (0)

static void fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw HenryError{code, buf};
}

// ---------------------------------------------------------------------------
// KL eigenpairs of exp(-|dx|/b) exp(-|dy|/b) on [0,Lx] x [-Ly,0] (host setup)
// ---------------------------------------------------------------------------
// 1-D modes on an interval of half-length a: even cos(w t) with c cos(wa) = w sin(wa),
// odd sin(w t) with w cos(wa) + c sin(wa) = 0, c = 1/b; lambda = 2c/(w^2 + c^2).
// Roots bracketed in (k pi/a, (k+1/2) pi/a) and ((k+1/2) pi/a, (k+1) pi/a) and found by
// bisection of the sine/cosine forms (no poles) to the last bit.
struct Mode1D {
  double w, lam, norm;
  int odd;
};

static double bisect(double lo, double hi, int odd, double a, double c) {
  auto f = [&](double w) { return odd ? w * std::cos(w * a) + c * std::sin(w * a) : c * std::cos(w * a) - w * std::sin(w * a); };
  double flo = f(lo);
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double fm = f(mid);
    if ((fm < 0) == (flo < 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

static std::vector<Mode1D> modes_1d(double a, double b, int n) {
  const double c = 1.0 / b;
  std::vector<Mode1D> out;
  for (int k = 0; (int)out.size() < n; ++k) {
    for (int odd = 0; odd < 2 && (int)out.size() < n; ++odd) {
      const double lo = (k + 0.5 * odd) * M_PI / a, hi = (k + 0.5 * odd + 0.5) * M_PI / a;
      const double w = bisect(lo, hi, odd, a, c);
      const double s2 = std::sin(2.0 * w * a) / (2.0 * w);
      out.push_back({w, 2.0 * c / (w * w + c * c), std::sqrt(odd ? a - s2 : a + s2), odd});
    }
  }
  return out;
}

static KLModes make_kl(const henry_problem& pr) {
  const int nm = 8, n1 = 12;
  auto mx = modes_1d(0.5 * pr.Lx, pr.corr_len, n1);
  auto my = modes_1d(0.5 * pr.Ly, pr.corr_len, n1);
  std::vector<std::tuple<double, int, int>> pairs;
  for (int ix = 0; ix < n1; ++ix)
    for (int iy = 0; iy < n1; ++iy) pairs.emplace_back(mx[ix].lam * my[iy].lam, ix, iy);
  std::stable_sort(pairs.begin(), pairs.end(), [](const auto& u, const auto& v) {
    if (std::get<0>(u) != std::get<0>(v)) return std::get<0>(u) > std::get<0>(v);
    return std::get<1>(u) < std::get<1>(v);
  });
  KLModes kl{};
  kl.n = std::max(pr.n_kl_phi, pr.n_kl_logK);
  for (int k = 0; k < nm; ++k) {
    const auto& [lam, ix, iy] = pairs[k];
    kl.sqrt_lam[k] = std::sqrt(lam);
    kl.wx[k] = mx[ix].w;
    kl.normx[k] = mx[ix].norm;
    kl.oddx[k] = mx[ix].odd;
    kl.wy[k] = my[iy].w;
    kl.normy[k] = my[iy].norm;
    kl.oddy[k] = my[iy].odd;
  }
  kl.xc = 0.5 * pr.Lx;
  kl.yc = -0.5 * pr.Ly;
  return kl;
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t b) {
    if (b <= bytes) return;
    if (p) HIPCHK(hipFree(p));
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, b) != hipSuccess) {
      (void)hipGetLastError();
      fail(HENRY_ENOMEM, "hipMalloc of %zu bytes failed", b);
    }
    bytes = b;
  }
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

// Thread map of a batch: blockDim = (SX, CY) with SX samples (a sample block, at most the
// batch) by CY = 256/SX cells.  sample_block 0: min(S, 64), i.e. a wavefront covers 64 samples
// of one cell; 16 or 32: a wavefront covers 2 or 4 neighbouring cells of fewer samples.
static Map make_map(int S, int ncell, int red_blocks, int sample_block = 0) {
  Map m{};
  m.S = S;
  const int sb = sample_block > 0 ? sample_block : 64;
  m.SX = S <= sb ? S : sb;
  m.CY = std::max(1, 256 / m.SX);
  m.nsb = (S + m.SX - 1) / m.SX;
  // reduction kernels: CPT cells per thread so that about `red_blocks` blocks cover the batch
  const int target = red_blocks > 0 ? std::max(64, red_blocks) : 4096;
  const int target_cb = std::max(1, target / m.nsb);
  const int rows = (ncell + m.CY - 1) / m.CY;
  m.CPT = std::max(1, (rows + target_cb - 1) / target_cb);
  m.ncb = (rows + m.CPT - 1) / m.CPT;
  return m;
}

// The multigrid stencil kernels' wide form: SP adjacent samples per thread, one 16-byte
// access per value (SP = 2 in FP64, 4 in FP32), used when the batch size is a multiple of
// SP, at least 64 SP, and some row width of SX threads (the sample block or a half or
// quarter of it) leaves no more samples idle in the last row than one sample per thread
// does; the thread geometry is that of a batch of S / SP with that SX, the sample count
// stays S.  wide_block returns that SX, 0 where there is no wide form.
static int wide_block(int S, int sp, int sample_block) {
  const int sb = sample_block > 0 ? sample_block : 64;
  if (S % sp || S < 64 * sp) return 0;
  const int sx1 = S <= sb ? S : sb;
  const int idle1 = (S + sx1 - 1) / sx1 * sx1 - S;
  for (int sx = sb; sx >= 16 && sx >= sb / 4; sx /= 2) {
    const int row = sp * sx;
    if ((S + row - 1) / row * row - S <= idle1) return sx;
  }
  return 0;
}
static int wide_samples(int S, int sp, int sample_block) { return wide_block(S, sp, sample_block) ? sp : 1; }
static Map make_map_wide(int S, int ncell, int sp, int sample_block) {
  const int sx = wide_block(S, sp, sample_block);
  if (!sx) return make_map(S, ncell, 0, sample_block);
  Map m = make_map(S / sp, ncell, 0, sx);
  m.S = S;
  return m;
}

static dim3 grid_cells(const Map& m, int ncell) {
  const long long nb = (long long)m.nsb * ((ncell + m.CY - 1) / m.CY);
  return dim3((unsigned)nb);
}
static dim3 grid_red(const Map& m) { return dim3((unsigned)((long long)m.nsb * m.ncb)); }
static dim3 block_of(const Map& m) { return dim3(m.SX, m.CY); }
// the assembly's tiles: one workgroup per (sample block, ASM_TX x ASM_TY cells)
static dim3 asm_grid(const Map& m, const Grid2& G) { return dim3((unsigned)((long long)m.nsb * asm_tiles(G.nx, G.ny))); }
static dim3 asm_block(const Map& m) { return dim3(m.SX, ASM_T); }
// Finalisation launch shape: blockDim.x = min(64, S rounded up to a power of 2) samples,
// the rest of the 64 * FIN_Y threads split each sample's partial sums.
static int fin_sx(int S) {
  int x = 1;
  while (x < S && x < 64) x <<= 1;
  return x;
}
static dim3 fin_grid(int S) { return dim3((unsigned)((S + fin_sx(S) - 1) / fin_sx(S))); }
static dim3 fin_block(int S) { return dim3(fin_sx(S), 64 * FIN_Y / fin_sx(S)); }

// LDS of the banded solve: y and x (2n each) plus CH rows of L, CH + mb rows of U, CH Dinv.
template <typename T>
static size_t band_solve_lds(int n, int mb, int CH) {
  return (size_t)(4 * n + CH * mb * 4 + (CH + mb) * mb * 4 + CH * 4) * sizeof(T);
}
template <typename T>
static int band_chunk(int n, int mb) {
  int CH = 64;
  while (CH > 1 && band_solve_lds<T>(n, mb, CH) > 64 * 1024) CH /= 2;
  return CH;
}

static Phys make_phys(const henry_problem& pr, int nx, int ny, int nsteps) {
  Phys P{};
  P.rho0 = pr.rho0;
  P.drho = pr.rho1 - pr.rho0;
  P.rho1 = pr.rho1;
  P.mu = pr.mu;
  P.g = pr.g;
  P.Dm = pr.Dm;
  P.c_left = pr.c_left;
  P.hx = pr.Lx / nx;
  P.hy = pr.Ly / ny;
  P.vol = P.hx * P.hy;
  P.tau = pr.T / nsteps;
  P.Ly = pr.Ly;
  P.Lx = pr.Lx;
  P.right_dir = pr.right_c_dirichlet;
  P.uin_fac = 1.0;
  P.qoi_xmin = pr.qoi_xmin;
  return P;
}

static FieldParams make_fp(const henry_problem& pr) {
  FieldParams fp{};
  fp.phi_mean = pr.phi_mean;
  fp.phi_amp = pr.phi_amp;
  fp.phi_min = pr.phi_min;
  fp.phi_max = pr.phi_max;
  fp.lnK_mean = std::log(pr.K_mean);
  fp.logK_amp = pr.logK_amp;
  fp.q_in = pr.q_in;
  fp.q_in_amp = pr.q_in_amp;
  fp.kappa_kc = pr.kappa_kc;
  fp.n_phi = pr.n_kl_phi;
  fp.n_logK = pr.n_kl_logK;
  fp.model = pr.field_model;
  return fp;
}

// ---------------------------------------------------------------------------
// per-shape plan: multigrid hierarchy and Krylov workspace of one batch
// ---------------------------------------------------------------------------
struct MGLevel {
  int nx, ny, ncell;
  Grid2 G;
  DevBuf J, x, b;             // MG precision
  DevBuf p, c, phi, K;        // restricted state and coefficients (FP64), levels >= 1
};

struct Plan {
  int nx, ny, S, prec, cnx, cny;
  int csolver;             // coarse solver: 0 banded LU, 1 dense LU with partial pivoting, 2 band LU with
                           // partial pivoting
  size_t N;
  Map m;
  Map mw2, mw4;            // the stencil kernels' wide forms (make_map_wide): 2 and 4 samples
  int sp2 = 1, sp4 = 1;    // per thread, where wide_samples allows them (else 1)
  Grid2 G;
  std::vector<std::unique_ptr<MGLevel>> lv;   // lv[0] = fine grid
  int nlev;
  DevBuf phi, K, uin, p, c, c_old, R, J, J32;
  DevBuf p_prev, c_prev;   // state of the previous step (initial-guess extrapolation)
  DevBuf p_prev2, c_prev2, p_prev3, c_prev3;   // and of the ones before (polynomial extrapolation)
  DevBuf vx, vr, vrh, vp, vv, vs, vt, vph, vsh;
  DevBuf LU, perm;         // coarse factors (banded or dense) and the dense solver's row permutation
  DevBuf sc, lam, ndone, status, stats, part, ctrl;
  DevBuf nhist;            // per sample: last undamped Newton update size, previous |R|^2
  size_t lu_stride;
  int mb;
  int* h_ctrl = nullptr;   // pinned mirror of ctrl
  // Compacted sub-batch for the last Newton iterations of a step: same shape and
  // capacity, used with an effective sample count Sa <= S (see Solver::compact_newton).
  std::unique_ptr<Plan> compact;
  DevBuf cidx;             // indices of the samples still iterating
  // captured BiCGStab iterations: [transposed][first iteration]
  hipGraphExec_t gexec[2][5] = {{nullptr, nullptr, nullptr, nullptr, nullptr},
                                {nullptr, nullptr, nullptr, nullptr, nullptr}};
  int gkey[2][5] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};   // per operator: nu_pre, nu_post, precision, cycle, valid
  double grtol[2] = {0.0, 0.0};
  // captured first Newton iteration of a time step (step_graphs) and what it was captured for
  hipGraphExec_t step_exec = nullptr;
  Phys step_phys{};
  henry_solver_opts step_opts{};
  int step_order = -1;
  void drop_step_graph() {
    if (step_exec) (void)hipGraphExecDestroy(step_exec);
    step_exec = nullptr;
  }
  void drop_graphs(int tr) {
    for (auto& g : gexec[tr])
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
    gkey[tr][4] = 0;
  }
  void drop_graphs() {
    drop_graphs(0);
    drop_graphs(1);
    drop_step_graph();
  }
  ~Plan() {
    drop_graphs();
    if (h_ctrl) (void)hipHostFree(h_ctrl);
  }
};

// Optional event timing of kernel classes on the context's stream.  A ring of event
// pairs per class is drained lazily (the oldest pair has normally completed), so
// timing does not serialise the host with the device.
struct Profiler {
  static constexpr int RING = 256;
  struct Slot {
    hipEvent_t a = nullptr, b = nullptr;
  };
  struct Cls {
    std::vector<Slot> ring;
    size_t head = 0, used = 0;
    long long launches = 0, units = 0;
    double ms = 0.0;
  };
  bool on = false;
  std::mutex mu;
  Cls c[HENRY_PROF_NCLASS];

  void drain_one(Cls& k, Slot& sl) {
    HIPCHK(hipEventSynchronize(sl.b));
    float e = 0.f;
    HIPCHK(hipEventElapsedTime(&e, sl.a, sl.b));
    k.ms += e;
  }
  Slot& acquire(int cls) {
    Cls& k = c[cls];
    if (k.ring.size() < RING) {
      k.ring.emplace_back();
      Slot& sl = k.ring.back();
      HIPCHK(hipEventCreate(&sl.a));
      HIPCHK(hipEventCreate(&sl.b));
      k.used++;
      return sl;
    }
    Slot& sl = k.ring[k.head];
    k.head = (k.head + 1) % RING;
    drain_one(k, sl);
    return sl;
  }
  void flush() {
    for (auto& k : c) {
      const size_t n = k.ring.size();
      if (n < RING) {
        for (size_t i = 0; i < n; ++i) drain_one(k, k.ring[i]);
      } else {
        for (size_t i = 0; i < RING; ++i) drain_one(k, k.ring[(k.head + i) % RING]);
      }
      for (auto& sl : k.ring) {
        (void)hipEventDestroy(sl.a);
        (void)hipEventDestroy(sl.b);
      }
      k.ring.clear();
      k.head = k.used = 0;
    }
  }
  void reset() {
    flush();
    for (auto& k : c) k.launches = k.units = 0, k.ms = 0.0;
  }
};

struct henry_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  // plans by (nx, ny, S, precision, coarse nx, coarse ny, reduction blocks, coarse solver,
  // sample block, instance): batches of one call that share a shape but are solved
  // concurrently get distinct instances
  std::map<std::tuple<int, int, int, int, int, int, int, int, int, int>, std::unique_ptr<Plan>> plans;
  int* h_ctrl = nullptr;   // pinned
  DevBuf mlmc_tmp;
  DevBuf adj_ck, adj_seg, adj_g;   // adjoint checkpoints, segment states, sensitivities
  DevBuf kws;                      // workspace of the kernel-level entry points
  std::atomic<long long> host_syncs{0};   // the solver's host round trips (control reads)
  std::atomic<long long> host_sync_ns{0}; // and the host time spent waiting in them
  std::vector<hipStream_t> streams; // per-grid streams of ragged solves (default priority)
  Profiler prof;
};

// Workspace of the allocation-free MLMC estimator: a file-scope device array (each device
// that runs the library holds its own copy until the process ends).  Host code never passes
// the symbol itself to a kernel or copy: it uses the device address that hipGetSymbolAddress
// returns for the current device, recorded once per device when a context is created.
static __device__ __align__(256) double scratch[HENRY_NOALLOC_SCRATCH_DOUBLES];
static constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch[MAX_DEVICES] = {};

// Record the scratch array's address on `device` (which must be current).
static hipError_t scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[device] = static_cast<double*>(ptr);
  return hipSuccess;
}

// Launch `f` on stream `st` and, when profiling (and not capturing a graph), time its
// first kernel with events of class `cls`: `f` launches through launch_timed, whose first
// call hands the events to hipExtLaunchKernelGGL, so they hold that kernel's own start and
// end timestamps (no event-record gaps around it).
static thread_local bool tl_capturing = false;
static thread_local bool tl_untimed = false;   // compacted sub-batches are not timed
static thread_local hipEvent_t tl_ev_start = nullptr, tl_ev_stop = nullptr;
template <typename K, typename... Args>
static void launch_timed(K kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t st, Args... args) {
  hipEvent_t a = tl_ev_start, b = tl_ev_stop;
  tl_ev_start = tl_ev_stop = nullptr;
  if (a) hipExtLaunchKernelGGL(kernel, grid, block, lds, st, a, b, 0, args...);
  else hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
}
template <typename F>
static void timed(henry_ctx* ctx, hipStream_t st, int cls, long long units, F&& f) {
  if (!ctx->prof.on || tl_capturing || tl_untimed) {
    f();
    return;
  }
  std::lock_guard<std::mutex> lk(ctx->prof.mu);
  auto& sl = ctx->prof.acquire(cls);
  tl_ev_start = sl.a;
  tl_ev_stop = sl.b;
  f();
  if (tl_ev_start) {
    tl_ev_start = tl_ev_stop = nullptr;
    fail(HENRY_EDEVICE, "internal: a timed launch did not go through launch_timed");
  }
  ctx->prof.c[cls].launches++;
  ctx->prof.c[cls].units += units;
}

// Capture the launches `f` makes on stream `st` (thread-local capture mode; the library's
// event timing is off meanwhile) as an instantiated graph.
template <typename F>
static hipGraphExec_t capture_graph(hipStream_t st, F&& f) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  tl_capturing = true;
  try {
    f();
  } catch (...) {
    tl_capturing = false;
    (void)hipStreamEndCapture(st, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  tl_capturing = false;
  HIPCHK(hipStreamEndCapture(st, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e);
  return ex;
}

template <typename T>
static void plan_alloc_levels(Plan& P) {
  for (int k = 0; k < P.nlev; ++k) {
    MGLevel& L = *P.lv[k];
    const size_t Nk = (size_t)L.ncell * P.S;
    if (k > 0 || P.prec == 32) {
      if (k > 0) L.J.alloc(20 * Nk * sizeof(T));
      if (k > 0) L.x.alloc(2 * Nk * sizeof(T));   // the fine cycle writes into the caller's vector
      L.b.alloc(2 * Nk * sizeof(T));
    }
    if (k > 0) {
      L.p.alloc(Nk * sizeof(double));
      L.c.alloc(Nk * sizeof(double));
      L.phi.alloc(Nk * sizeof(double));
      L.K.alloc(Nk * sizeof(double));
    }
  }
  const MGLevel& C = *P.lv[P.nlev - 1];
  P.mb = C.ny;
  if (P.csolver == 1) {
    const size_t n = 2 * (size_t)C.ncell;
    P.lu_stride = n * n;
    P.LU.alloc(P.lu_stride * P.S * sizeof(T));
    P.perm.alloc(n * P.S * sizeof(int));
  } else if (P.csolver == 2) {
    P.lu_stride = gb_stride(C.nx, C.ny);
    P.LU.alloc(P.lu_stride * P.S * sizeof(T));
    P.perm.alloc(2 * (size_t)C.ncell * P.S * sizeof(int));
  } else {
    P.lu_stride = (size_t)C.ncell * (2 * P.mb + 1) * 4;
    P.LU.alloc(P.lu_stride * P.S * sizeof(T));
  }
}

// Largest dynamic LDS one workgroup may use on the current device (the opt-in limit, which a
// launch reaches after hipFuncSetAttribute, when it is the larger).
static size_t max_lds_per_block() {
  int dev = 0, v = 0, o = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (hipDeviceGetAttribute(&o, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) {
    (void)hipGetLastError();
    o = 0;
  }
  return (size_t)std::max(v, o);
}

// The dense factorisation needs more than the default LDS limit of a launch: raise it once
// per instantiation (and device) before its first launch.
template <typename T>
static void dense_factor_prepare(size_t lds) {
  static std::mutex mu;
  static bool done[64] = {};
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if (dev >= 0 && dev < 64 && done[dev]) return;
  HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_factor<T, 16>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (dev >= 0 && dev < 64) done[dev] = true;
}

// Band LU with partial pivoting: the pivot search covers kl + 1 rows in one wavefront, and the
// factor window and the solve's staging must fit the default LDS limit of a launch.
static void check_gb_size(int nxc, int nyc, int prec) {
  const size_t f = prec == 32 ? gb_factor_lds<float>(nyc) : gb_factor_lds<double>(nyc);
  const size_t sv = prec == 32 ? gb_solve_lds<float>(nxc, nyc) : gb_solve_lds<double>(nxc, nyc);
  if (gb_kl(nyc) + 1 > 64 || gb_kl(nyc) * 2 * gb_kl(nyc) > GB_THREADS * GB_UPD || f > 64 * 1024 || sv > 64 * 1024)
    fail(HENRY_EUNSUPPORTED, "coarsest grid %dx%d too large for the pivoted band LU (ny <= 19 and the LDS limit)", nxc,
         nyc);
}

static void plan_set_wide(Plan& Q, int sample_block) {
  Q.sp2 = wide_samples(Q.S, 2, sample_block);
  Q.sp4 = wide_samples(Q.S, 4, sample_block);
  Q.mw2 = make_map_wide(Q.S, Q.nx * Q.ny, Q.sp2, sample_block);
  Q.mw4 = make_map_wide(Q.S, Q.nx * Q.ny, Q.sp4, sample_block);
}

static std::unique_ptr<Plan> make_plan(int nx, int ny, int S, const henry_solver_opts& o) {
  const int cnx = std::min(o.coarse_nx, nx), cny = std::min(o.coarse_ny, ny);
  auto P = std::make_unique<Plan>();
  P->nx = nx;
  P->ny = ny;
  P->S = S;
  P->prec = o.mg_precision;
  P->cnx = cnx;
  P->cny = cny;
  P->csolver = o.coarse_solver;
  P->G = Grid2{nx, ny, nx * ny};
  P->N = (size_t)nx * ny * S;
  P->m = make_map(S, nx * ny, o.red_blocks, o.sample_block);
  plan_set_wide(*P, o.sample_block);
  // hierarchy: halve while above the coarse size and even
  int gx = nx, gy = ny;
  while (true) {
    auto L = std::make_unique<MGLevel>();
    L->nx = gx;
    L->ny = gy;
    L->ncell = gx * gy;
    L->G = Grid2{gx, gy, gx * gy};
    P->lv.push_back(std::move(L));
    if (gx <= cnx || gy <= cny || (gx & 1) || (gy & 1)) break;
    gx /= 2;
    gy /= 2;
  }
  P->nlev = (int)P->lv.size();
  if (o.coarse_solver == 1) {
    const int n = 2 * P->lv.back()->ncell;
    const size_t need = o.mg_precision == 32 ? dense_factor_lds<float>(n, 16) : dense_factor_lds<double>(n, 16);
    if (n % 16) fail(HENRY_EUNSUPPORTED, "coarsest grid %dx%d: the dense LU needs 2 * cells divisible by 16", gx, gy);
    if (need > max_lds_per_block())
      fail(HENRY_EUNSUPPORTED, "coarsest grid %dx%d too large for the dense LU's LDS panel (%zu bytes)", gx, gy, need);
  } else if (o.coarse_solver == 2) {
    check_gb_size(gx, gy, o.mg_precision);
  } else {
    if (P->lv.back()->ny > 44) fail(HENRY_EUNSUPPORTED, "coarsest grid %dx%d: band width %d exceeds 44", gx, gy, gy);
    const int n = P->lv.back()->ncell, mb = P->lv.back()->ny;
    const size_t need = o.mg_precision == 32 ? band_solve_lds<float>(n, mb, 1) : band_solve_lds<double>(n, mb, 1);
    if (need > 64 * 1024) fail(HENRY_EUNSUPPORTED, "coarsest grid %dx%d too large for the LDS banded solve", gx, gy);
  }
  for (int k = 0; k + 1 < P->nlev; ++k)
    if (P->lv[k]->nx & 1) fail(HENRY_EUNSUPPORTED, "multigrid level %d has odd nx", k);
  const size_t N = P->N;
  P->phi.alloc(N * 8);
  P->K.alloc(N * 8);
  P->uin.alloc(S * 8);
  P->p.alloc(N * 8);
  P->c.alloc(N * 8);
  P->c_old.alloc(N * 8);
  P->p_prev.alloc(N * 8);
  P->c_prev.alloc(N * 8);
  P->p_prev2.alloc(N * 8);
  P->c_prev2.alloc(N * 8);
  P->p_prev3.alloc(N * 8);
  P->c_prev3.alloc(N * 8);
  P->R.alloc(2 * N * 8);
  P->J.alloc(20 * N * 8);
  if (o.mg_precision == 32) P->J32.alloc(20 * N * 4);
  for (DevBuf* v : {&P->vx, &P->vr, &P->vrh, &P->vp, &P->vv, &P->vs, &P->vt, &P->vph, &P->vsh}) v->alloc(2 * N * 8);
  if (o.mg_precision == 32) plan_alloc_levels<float>(*P);
  else plan_alloc_levels<double>(*P);
  P->sc.alloc((size_t)SC_NSLOT * S * 8);
  P->lam.alloc(S * 8);
  P->ndone.alloc(S * 4);
  P->nhist.alloc((size_t)S * 2 * 8);
  P->status.alloc(S * 4);
  P->stats.alloc((size_t)S * 4 * 8);
  P->part.alloc((size_t)NSERIES * P->m.ncb * S * 8);   // widest reduction: the series
  P->ctrl.alloc(64);
  HIPCHK(hipHostMalloc((void**)&P->h_ctrl, 16 * sizeof(int), hipHostMallocDefault));
  P->cidx.alloc((size_t)S * sizeof(int));
  return P;
}

using PlanKey = std::tuple<int, int, int, int, int, int, int, int, int, int>;

static PlanKey plan_key(int nx, int ny, int S, const henry_solver_opts& o, int inst) {
  return PlanKey(nx, ny, S, o.mg_precision, std::min(o.coarse_nx, nx), std::min(o.coarse_ny, ny), o.red_blocks,
                 o.coarse_solver, o.sample_block, inst);
}

// Widest per-sample reduction buffer any effective batch size Sa <= S needs.
static size_t part_bytes_max(int nx, int ny, int S, int red_blocks, int sample_block) {
  size_t mx = 0;
  for (int Sa = 1; Sa <= S; ++Sa)
    mx = std::max(mx, (size_t)NSERIES * make_map(Sa, nx * ny, red_blocks, sample_block).ncb * Sa * 8);
  return mx;
}

// The plan of a batch shape, with its compacted sub-plan (see Solver::compact_newton) created
// and sized for every effective batch size up front: the solve itself then allocates and frees
// no device or pinned memory, so concurrent solves on worker threads never call the allocator
// while another thread captures or synchronises a stream.
static Plan* get_plan(henry_ctx* ctx, int nx, int ny, int S, const henry_solver_opts& o, int inst = 0) {
  const PlanKey key = plan_key(nx, ny, S, o, inst);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) return it->second.get();
  auto P = make_plan(nx, ny, S, o);
  P->compact = make_plan(nx, ny, S, o);
  P->compact->part.alloc(part_bytes_max(nx, ny, S, o.red_blocks, o.sample_block));
  Plan* raw = P.get();
  ctx->plans[key] = std::move(P);
  return raw;
}

// Use plan Q (capacity >= Sa samples) for an effective batch of Sa samples.  Allocates
// nothing: get_plan sized the reduction buffer for every Sa.
static void plan_set_samples(Plan& Q, int Sa, int red_blocks, int sample_block) {
  Q.S = Sa;
  Q.N = (size_t)Q.nx * Q.ny * Sa;
  Q.m = make_map(Sa, Q.nx * Q.ny, red_blocks, sample_block);
  plan_set_wide(Q, sample_block);
  if ((size_t)NSERIES * Q.m.ncb * Sa * 8 > Q.part.bytes) fail(HENRY_EDEVICE, "internal: compact plan undersized");
  Q.drop_graphs();
}

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------
struct Solver {
  henry_ctx* ctx;
  const henry_problem& pr;
  const henry_solver_opts& o;
  Plan& P;
  hipStream_t st;
  Phys phys;       // fine grid
  KLModes kl;
  FieldParams fp;

  Solver(henry_ctx* c, const henry_problem& p, const henry_solver_opts& op, Plan& pl, int nsteps, hipStream_t stream)
      : ctx(c), pr(p), o(op), P(pl), st(stream) {
    phys = make_phys(pr, P.nx, P.ny, nsteps);
    kl = make_kl(pr);
    fp = make_fp(pr);
  }

  Phys phys_level(int k) const {
    Phys q = phys;
    q.hx = pr.Lx / P.lv[k]->nx;
    q.hy = pr.Ly / P.lv[k]->ny;
    q.vol = q.hx * q.hy;
    return q;
  }

  void zero_ctrl() { hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, P.ctrl.as<int>(), 16); }
  int read_ctrl(int i) {
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipMemcpyAsync(P.h_ctrl, P.ctrl.as<int>(), 16 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->host_syncs++;
    ctx->host_sync_ns += std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
    return P.h_ctrl[i];
  }

  void fields(const double* theta) {
    const Map& m = P.m;
    hipLaunchKernelGGL(k_fields, grid_cells(m, P.G.ncell), block_of(m), 0, st, m, P.G, phys, kl, fp, theta,
                       P.phi.as<double>(), P.K.as<double>(), P.uin.as<double>());
    for (int k = 1; k < P.nlev; ++k) {
      MGLevel& F = *P.lv[k - 1];
      MGLevel& C = *P.lv[k];
      const double* fphi = k == 1 ? P.phi.as<double>() : F.phi.as<double>();
      const double* fK = k == 1 ? P.K.as<double>() : F.K.as<double>();
      hipLaunchKernelGGL(k_restrict_coef, grid_cells(m, C.ncell), block_of(m), 0, st, m, F.G, C.G, fphi, fK,
                         C.phi.as<double>(), C.K.as<double>());
    }
  }

  // Residual only: the Jacobian hierarchy and the coarse factors of an earlier iterate are kept.
  void assemble_residual() {
    const Map& m = P.m;
    hipLaunchKernelGGL((k_assemble<true, double, false, false>), asm_grid(m, P.G), asm_block(m), asm_lds(m.SX), st, m, P.G,
                       phys, P.p.as<double>(), P.c.as<double>(), P.c_old.as<double>(), P.phi.as<double>(),
                       P.K.as<double>(), P.uin.as<double>(), P.R.as<double>(), (double*)nullptr, (float*)nullptr);
  }

  // fine-grid residual/Jacobian, rediscretised coarse Jacobians, coarse factorisation
  template <typename T>
  void assemble_all() {
    const Map& m = P.m;
    timed(ctx, st, HENRY_PROF_ASSEMBLE, (long long)P.N, [&] {
      if (spmv32())   // only the FP32 Jacobian: the multigrid and the Krylov products read it
        launch_timed((k_assemble<true, float, false>), asm_grid(m, P.G), asm_block(m), asm_lds(m.SX), st, m, P.G,
                           phys, P.p.as<double>(), P.c.as<double>(), P.c_old.as<double>(), P.phi.as<double>(),
                           P.K.as<double>(), P.uin.as<double>(), P.R.as<double>(), P.J32.as<float>(), (float*)nullptr);
      else if (P.prec == 32)
        launch_timed((k_assemble<true, double, true>), asm_grid(m, P.G), asm_block(m), asm_lds(m.SX), st, m, P.G,
                           phys, P.p.as<double>(), P.c.as<double>(), P.c_old.as<double>(), P.phi.as<double>(),
                           P.K.as<double>(), P.uin.as<double>(), P.R.as<double>(), P.J.as<double>(), P.J32.as<float>());
      else
        launch_timed((k_assemble<true, double, false>), asm_grid(m, P.G), asm_block(m), asm_lds(m.SX), st, m, P.G,
                           phys, P.p.as<double>(), P.c.as<double>(), P.c_old.as<double>(), P.phi.as<double>(),
                           P.K.as<double>(), P.uin.as<double>(), P.R.as<double>(), P.J.as<double>(), (float*)nullptr);
    });
    for (int k = 1; k < P.nlev; ++k) {
      MGLevel& F = *P.lv[k - 1];
      MGLevel& C = *P.lv[k];
      const double* fp_ = k == 1 ? P.p.as<double>() : F.p.as<double>();
      const double* fc_ = k == 1 ? P.c.as<double>() : F.c.as<double>();
      hipLaunchKernelGGL(k_restrict_state, grid_cells(m, C.ncell), block_of(m), 0, st, m, F.G, C.G, fp_, fc_,
                         C.p.as<double>(), C.c.as<double>());
      hipLaunchKernelGGL((k_assemble<false, T, false>), asm_grid(m, C.G), asm_block(m), asm_lds(m.SX), st, m, C.G,
                         phys_level(k), C.p.as<double>(), C.c.as<double>(), (const double*)nullptr,
                         C.phi.as<double>(), C.K.as<double>(), P.uin.as<double>(), (double*)nullptr, C.J.as<T>(),
                         (float*)nullptr);
    }
    coarse_factor<T>();
  }

  // factors of the coarsest operator: banded LU, or the dense matrix and its pivoted LU
  template <typename T>
  void coarse_factor() {
    const MGLevel& Cc = *P.lv[P.nlev - 1];
    if (P.csolver == 1) {
      const int n = 2 * Cc.ncell;
      const size_t lds = dense_factor_lds<T>(n, 16);
      dense_factor_prepare<T>(lds);
      hipLaunchKernelGGL((k_dense_build<T>), dim3(n, P.S), dim3(256), 0, st, P.S, Cc.nx, Cc.ny,
                         level_J<T>(P.nlev - 1), P.LU.as<T>());
      timed(ctx, st, HENRY_PROF_DENSE_FACTOR, (long long)P.S, [&] {
        launch_timed((k_dense_factor<T, 16>), dim3(P.S), dim3(DENSE_THREADS), lds, st, n, P.LU.as<T>(),
                           P.perm.as<int>());
      });
      return;
    }
    if (P.csolver == 2) {
      timed(ctx, st, HENRY_PROF_BAND_FACTOR, (long long)Cc.ncell * P.S, [&] {
        launch_timed((k_gb_factor<T>), dim3(P.S), dim3(GB_THREADS), gb_factor_lds<T>(Cc.ny), st, P.S, Cc.nx,
                           Cc.ny, level_J<T>(P.nlev - 1), P.LU.as<T>(), P.perm.as<int>());
      });
      return;
    }
    const size_t lds = (size_t)(P.mb + 1) * (P.mb + 1) * 4 * sizeof(T);
    timed(ctx, st, HENRY_PROF_BAND_FACTOR, (long long)Cc.ncell * P.S, [&] {
      launch_timed((k_band_factor<T>), dim3(P.S), dim3(64), lds, st, P.S, Cc.nx, Cc.ny, level_J<T>(P.nlev - 1),
                         P.LU.as<T>());
    });
  }

  template <typename T>
  const T* level_J(int k) const {
    if (k > 0) return P.lv[k]->J.as<T>();
    if (P.prec == 32) return (const T*)P.J32.as<float>();
    return (const T*)P.J.as<double>();
  }

  // One multigrid cycle x = M^{-1} b on level k (TR: the same cycle built from transposed
  // operators, a preconditioner for J^T): a V-cycle, or a W-cycle (mg_cycle 2: the coarse
  // problem gets two cycles, the second from the first's result).  zero: x starts at 0.
  template <typename T, bool TR = false>
  void vcycle(int k, const T* b, T* x, bool zero = true) {
    const Map& m = P.m;
    MGLevel& L = *P.lv[k];
    // the stencil kernels' launch width: 4 samples per thread in FP32, 2 in FP64, where the
    // batch allows it (16-byte accesses); f(integral_constant<int, SP>)
    auto wide = [&](auto&& f) {
      if constexpr (sizeof(T) == 4) {
        if (P.sp4 == 4) return f(std::integral_constant<int, 4>{});
      }
      if (P.sp2 == 2) return f(std::integral_constant<int, 2>{});
      return f(std::integral_constant<int, 1>{});
    };
    auto wide_map = [&](int sp) -> const Map& { return sp == 4 ? P.mw4 : sp == 2 ? P.mw2 : m; };
    if (k == P.nlev - 1 && P.csolver == 1) {
      timed(ctx, st, HENRY_PROF_DENSE_SOLVE, (long long)P.S, [&] {
        launch_timed((k_dense_solve<T, TR>), dim3(P.S), dim3(DENSE_SOLVE_THREADS), dense_solve_lds<T>(2 * L.ncell), st,
                           P.S, L.ncell, P.LU.as<T>(), (const int*)P.perm.as<int>(), b, x);
      });
      return;
    }
    if (k == P.nlev - 1 && P.csolver == 2) {
      timed(ctx, st, HENRY_PROF_BAND_SOLVE, (long long)L.ncell * P.S, [&] {
        launch_timed((k_gb_solve<T, TR>), dim3(P.S), dim3(64), gb_solve_lds<T>(L.nx, L.ny), st, P.S, L.nx, L.ny,
                           (const T*)P.LU.as<T>(), (const int*)P.perm.as<int>(), b, x);
      });
      return;
    }
    if (k == P.nlev - 1) {
      const int CH = band_chunk<T>(L.ncell, P.mb);
      const size_t lds = band_solve_lds<T>(L.ncell, P.mb, CH);
      timed(ctx, st, HENRY_PROF_BAND_SOLVE, (long long)L.ncell * P.S, [&] {
        if (TR)
          launch_timed((k_band_solve_T<T>), dim3(P.S), dim3(64), lds, st, P.S, L.nx, L.ny, CH, P.LU.as<T>(), b,
                             x);
        else
          launch_timed((k_band_solve<T>), dim3(P.S), dim3(64), lds, st, P.S, L.nx, L.ny, CH, P.LU.as<T>(), b, x);
      });
      return;
    }
    const T* J = level_J<T>(k);
    const int half = (L.nx + 1) / 2;
    // fine-grid smoother passes that read neighbours are timed as one class
    const long long half_units = (long long)L.ny * half * P.S;
    MGLevel& C = *P.lv[k + 1];
    auto gs_launch = [&](auto sp_tag, int colour, int mode) {
      constexpr int SP = decltype(sp_tag)::value;
      const Map& mg = wide_map(SP);
      const dim3 gg = grid_cells(mg, L.ny * half), bb = block_of(mg);
      if (mode == 1)
        launch_timed((k_gs_colour<T, TR, 1, SP>), gg, bb, 0, st, mg, L.G, C.G, colour, J, b, x, (const T*)nullptr);
      else if (mode == 2)
        launch_timed((k_gs_colour<T, TR, 2, SP>), gg, bb, 0, st, mg, L.G, C.G, colour, J, b, x,
                     (const T*)C.x.as<T>());
      else if (mode == 3)
        launch_timed((k_gs_colour<T, TR, 3, SP>), gg, bb, 0, st, mg, L.G, C.G, colour, J, b, x, (const T*)nullptr);
      else
        launch_timed((k_gs_colour<T, TR, 0, SP>), gg, bb, 0, st, mg, L.G, C.G, colour, J, b, x, (const T*)nullptr);
    };
    auto gs = [&](int colour, int mode) {
      auto f = [&] { wide([&](auto sp_tag) { gs_launch(sp_tag, colour, mode); }); };
      if (k == 0 && mode == 0) timed(ctx, st, HENRY_PROF_GS, half_units, f);
      else f();
    };
    // One pre-smoothing sweep followed by post-smoothing: the red half of the sweep is
    // never stored (its values are D^{-1} b, formed where they are read, and the first
    // post-smoothing pass recomputes red without them).
    const bool implicit_red = zero && o.nu_pre == 1 && o.nu_post >= 1;
    if (implicit_red) {
      gs(1, 3);
    } else {
      for (int sw = 0; sw < o.nu_pre; ++sw) {
        gs(0, sw == 0 && zero ? 1 : 0);
        gs(1, 0);
      }
    }
    auto rr = [&] {
      wide([&](auto sp_tag) {
        constexpr int SP = decltype(sp_tag)::value;
        const Map& mg = wide_map(SP);
        launch_timed((k_residual_restrict<T, TR, SP>), grid_cells(mg, C.ncell), block_of(mg), 0, st, mg, L.G, C.G,
                     implicit_red ? 2 : 1, J, b, x, C.b.as<T>());
      });
    };
    if (k == 0) timed(ctx, st, HENRY_PROF_RESTRICT, (long long)L.ncell * P.S, rr);
    else rr();
    const int visits = k + 2 < P.nlev ? o.mg_cycle : 1;   // the coarsest level is solved exactly
    for (int v = 0; v < visits; ++v) vcycle<T, TR>(k + 1, C.b.as<T>(), C.x.as<T>(), v == 0);
    if (o.nu_post == 0 || !o.fuse_prolong) {
      // separate prolongation and correction of every cell, then plain post-smoothing passes
      // (the red pass overwrites red x from the black neighbours alone)
      auto pc = [&] {
        wide([&](auto sp_tag) {
          constexpr int SP = decltype(sp_tag)::value;
          const Map& mg = wide_map(SP);
          launch_timed((k_prolong_correct<T, SP>), grid_cells(mg, L.ncell), block_of(mg), 0, st, mg, L.G, C.G,
                       C.x.as<T>(), x);
        });
      };
      if (k == 0) timed(ctx, st, HENRY_PROF_PROLONG, (long long)L.ncell * P.S, pc);
      else pc();
      for (int sw = 0; sw < o.nu_post; ++sw) {
        gs(0, 0);
        gs(1, 0);
      }
      return;
    }
    // the coarse-grid correction is folded into the first post-smoothing pass
    auto g2 = [&] { gs(0, 2); };
    if (k == 0) timed(ctx, st, HENRY_PROF_PROLONG, half_units, g2);
    else g2();
    gs(1, 0);
    for (int sw = 1; sw < o.nu_post; ++sw) {
      gs(0, 0);
      gs(1, 0);
    }
  }

  // out = M^{-1} in.  FP64 mode: out holds FP64 values.  FP32 mode: the FP64 input is rounded
  // to FP32 and the FP32 cycle writes its result straight into out's memory as FP32 values,
  // which the SpMV and the x update read (widening them there is exact, so no FP64 copy).
  template <typename T, bool TR = false>
  void precond(const double* in, double* out) {
    if (P.prec == 32) {
      MGLevel& L = *P.lv[0];
      const size_t n = 2 * P.N;
      const dim3 g((unsigned)((n + 255) / 256));
      hipLaunchKernelGGL((k_convert<double, float>), g, dim3(256), 0, st, n, in, L.b.as<float>());
      vcycle<float, TR>(0, L.b.as<float>(), reinterpret_cast<float*>(out));
    } else {
      vcycle<double, TR>(0, in, out);
    }
  }

  // One BiCGStab iteration comes in three parts, each a fixed kernel sequence with no host
  // decision inside.  A: p update, M^{-1} p, v = A p-hat, alpha, s = r - alpha v and the
  // half-step test.  B: M^{-1} s, t = A s-hat, omega (a sample that met the tolerance at the
  // half step keeps omega = 0, so B changes nothing for it).  C: x, r updates and the
  // convergence test.  rh: shadow residual; black_exact: the SpMV after a cycle multiplies out
  // red rows only (see bicgstab).
  template <typename T, bool TR>
  void kry_partA(int first, const double* rh, bool black_exact, double rtol2) {
    const Map& m = P.m;
    double* sc = P.sc.as<double>();
    const dim3 rg = grid_red(m), bl = block_of(m), cg = grid_cells(m, P.G.ncell);
    const dim3 fg = fin_grid(P.S), fb = fin_block(P.S);
    if (!first)   // p0 = r0 was written by the initialisation
      hipLaunchKernelGGL(k_bicg_p, cg, bl, 0, st, m, P.G.ncell, 0, sc, P.vr.as<double>(), P.vv.as<double>(),
                         P.vp.as<double>());
    precond<T, TR>(P.vp.as<double>(), P.vph.as<double>());
    timed(ctx, st, HENRY_PROF_SPMV, (long long)P.N, [&] {
      spmv_pre<1, TR>(P.vph.as<double>(), P.vv.as<double>(), rh,
                      black_exact ? (const double*)P.vp.as<double>() : nullptr);
    });
    hipLaunchKernelGGL(k_fin_alpha, fg, fb, 0, st, m, P.part.as<double>(), sc, o.krylov_breakdown,
                       P.status.as<int>());
    // r0 is held in p (unchanged until the second iteration's p update)
    hipLaunchKernelGGL(k_bicg_s, rg, bl, 0, st, m, P.G.ncell, sc, first ? P.vp.as<double>() : P.vr.as<double>(),
                       P.vv.as<double>(), P.vs.as<double>(), P.part.as<double>());
    zero_ctrl();
    hipLaunchKernelGGL(k_fin_half, fg, fb, 0, st, m, P.part.as<double>(), sc, rtol2, P.ctrl.as<int>());
  }

  template <typename T, bool TR>
  void kry_partB(bool black_exact) {
    const Map& m = P.m;
    precond<T, TR>(P.vs.as<double>(), P.vsh.as<double>());
    timed(ctx, st, HENRY_PROF_SPMV, (long long)P.N, [&] {
      spmv_pre<2, TR>(P.vsh.as<double>(), P.vt.as<double>(), P.vs.as<double>(),
                      black_exact ? (const double*)P.vs.as<double>() : nullptr);
    });
    hipLaunchKernelGGL(k_fin_omega, fin_grid(P.S), fin_block(P.S), 0, st, m, P.part.as<double>(), P.sc.as<double>());
  }

  void kry_partC(int first, const double* rh, double rtol2) {
    const Map& m = P.m;
    if (P.prec == 32)
      hipLaunchKernelGGL(k_bicg_xr<float>, grid_red(m), block_of(m), 0, st, m, P.G.ncell, first, P.sc.as<double>(),
                         reinterpret_cast<const float*>(P.vph.p), reinterpret_cast<const float*>(P.vsh.p),
                         P.vs.as<double>(), P.vt.as<double>(), rh, P.vx.as<double>(), P.vr.as<double>(),
                         P.part.as<double>());
    else
      hipLaunchKernelGGL(k_bicg_xr<double>, grid_red(m), block_of(m), 0, st, m, P.G.ncell, first, P.sc.as<double>(),
                         P.vph.as<double>(), P.vsh.as<double>(), P.vs.as<double>(), P.vt.as<double>(), rh,
                         P.vx.as<double>(), P.vr.as<double>(), P.part.as<double>());
    zero_ctrl();
    hipLaunchKernelGGL(k_fin_rho, fin_grid(P.S), fin_block(P.S), 0, st, m, P.part.as<double>(), P.sc.as<double>(),
                       rtol2, P.status.as<int>(), P.ctrl.as<int>());
  }

  // Start of a solve: r0 = sign * rhs (- A x0 when warm), p0 = r0, per-sample norms, the
  // active flags and, for Newton systems, the predictive convergence test (ctrl[0]: active
  // samples, ctrl[1]: Newton samples still iterating).
  template <bool TR>
  void kry_init(const double* rhs, double sign, int* mask, bool warm, bool newton, double rtol2, bool alias_rhat) {
    const Map& m = P.m;
    const dim3 rg = grid_red(m), bl = block_of(m);
    if (warm) spmv<1, TR, double>(P.vx.as<double>(), P.vv.as<double>(), P.vx.as<double>(), nullptr);
    hipLaunchKernelGGL(k_bicg_init, rg, bl, 0, st, m, P.G.ncell, rhs, sign, warm ? (const double*)P.vv.as<double>() : nullptr,
                       mask, alias_rhat ? (double*)nullptr : P.vrh.as<double>(), P.vp.as<double>(), P.part.as<double>());
    zero_ctrl();
    hipLaunchKernelGGL(k_fin_init, fin_grid(P.S), fin_block(P.S), 0, st, m, P.part.as<double>(), P.sc.as<double>(),
                       P.ctrl.as<int>(), newton ? P.nhist.as<double>() : (double*)nullptr, mask,
                       o.newton_tol * o.newton_predict, rtol2, alias_rhat ? sign : 1.0);
  }

  // Cycles ending in a black pass (or the exact coarse solve) leave A M^{-1} b = b on black
  // rows, so the SpMVs after them multiply out the red rows only.  With the FP32 cycle the
  // identity holds for the FP32 Jacobian, i.e. up to about 1e-7 relative: used only when the
  // tolerance is far above that (the Newton systems; their residual is always FP64).
  bool black_exact(double rtol) const { return o.nu_post >= 1 && (P.prec == 64 || rtol >= 1e-5); }

  // The forward solves of the FP32-multigrid path keep only the FP32 Jacobian: the Newton
  // systems need the operator only to the forcing term (5e-2 relative), far above FP32
  // rounding, while Newton's residual stays FP64, so the fixed point is that of the FP64
  // equations.  The adjoint's transposed solves (tolerance 1e-8) use the FP64 Jacobian.
  bool fwd_fp32_jacobian = true;
  bool spmv32() const { return P.prec == 32 && fwd_fp32_jacobian; }

  // y = J x (J^T x) with per-sample dots (k_spmv_dot) on the fine grid, in the Jacobian's
  // storage precision for these solves; x in precision TX
  template <int NDOT, bool TR, typename TX>
  void spmv(const TX* x, double* y, const double* d0, const double* yb) {
    const Map& m = P.m;
    if (spmv32())
      launch_timed((k_spmv_dot<NDOT, TR, float, TX>), grid_red(m), block_of(m), 0, st, m, P.G,
                         (const float*)P.J32.as<float>(), x, y, d0, P.part.as<double>(), yb);
    else
      launch_timed((k_spmv_dot<NDOT, TR, double, TX>), grid_red(m), block_of(m), 0, st, m, P.G,
                         (const double*)P.J.as<double>(), x, y, d0, P.part.as<double>(), yb);
  }
  // y = J M^{-1}-output: the preconditioned vector is FP32 in the FP32-multigrid path
  template <int NDOT, bool TR>
  void spmv_pre(const double* xbuf, double* y, const double* d0, const double* yb) {
    if (P.prec == 32) spmv<NDOT, TR, float>(reinterpret_cast<const float*>(xbuf), y, d0, yb);
    else spmv<NDOT, TR, double>(xbuf, y, d0, yb);
  }

  // Right-preconditioned BiCGStab, per sample: A x = sign * rhs, x in vx, with A = J
  // (or J^T when TR).  Samples with mask[s] != 0 get a zero right-hand side.  For a
  // Newton system (newton = true, mask = ndone) the initial residual norms also drive the
  // predictive convergence test; when that leaves at most `stop_at` samples iterating,
  // the solve is not started and their count is returned (else -1), so that the caller
  // can move them to a compacted batch first.
  // warm: start from the x already in vx (r0 = b - A x0); otherwise from x0 = 0.  The
  // tolerance is relative to |b| either way.
  template <typename T, bool TR = false>
  int bicgstab(const double* rhs, double sign, int* mask, double rtol, bool newton = false, int stop_at = -1,
               bool warm = false) {
    const int S = P.S;
    const bool bx = black_exact(rtol);
    const double rtol2 = rtol * rtol;
    // Newton systems (the residual buffer, cold start): the shadow residual is R itself,
    // i.e. sign * r0 (BiCGStab only uses it in ratios of dot products).  Otherwise it is a
    // stored copy of r0.  The captured graphs hold this pointer, so it is fixed per TR.
    const bool alias_rhat = !TR;
    if (alias_rhat && (rhs != P.R.as<double>() || warm || (sign != 1.0 && sign != -1.0)))
      fail(HENRY_EDEVICE, "internal: untransposed solves take the Newton residual, cold");
    const double* rh = alias_rhat ? rhs : P.vrh.as<double>();
    kry_init<TR>(rhs, sign, mask, warm, newton, rtol2, alias_rhat);
    if (read_ctrl(0) == 0) {
      // nothing to solve: x = 0, or x0 already within the tolerance
      if (!warm) HIPCHK(hipMemsetAsync(P.vx.p, 0, 2 * P.N * sizeof(double), st));
      return -1;
    }
    if (newton && P.h_ctrl[1] <= stop_at) return P.h_ctrl[1];
    const bool graphs = o.use_graphs && allow_graphs && !ctx->prof.on;
    if (graphs) {
      const int key[5] = {o.nu_pre, o.nu_post, P.prec, o.mg_cycle, 1};
      if (std::memcmp(key, P.gkey[TR], sizeof key) != 0 || P.grtol[TR] != rtol2) {
        P.drop_graphs(TR);
        std::memcpy(P.gkey[TR], key, sizeof key);
        P.grtol[TR] = rtol2;
      }
      for (int part = 0; part < 5; ++part) {
        if (P.gexec[TR][part]) continue;
        // parts 0/1: A of later/first iterations, 2: B, 3/4: C of later/first iterations
        P.gexec[TR][part] = capture([&] {
          if (part < 2) kry_partA<T, TR>(part, rh, bx, rtol2);
          else if (part == 2) kry_partB<T, TR>(bx);
          else kry_partC(part - 3, rh, rtol2);
        });
      }
    }
    for (int it = 0; it < o.krylov_maxit; ++it) {
      const int first = it == 0 ? 1 : 0;
      const int first_x = first && !warm;   // x = update (x0 = 0) rather than x += update
      if (graphs) HIPCHK(hipGraphLaunch(P.gexec[TR][first], st));
      else kry_partA<T, TR>(first, rh, bx, rtol2);
      if (read_ctrl(0) > 0) {
        if (graphs) HIPCHK(hipGraphLaunch(P.gexec[TR][2], st));
        else kry_partB<T, TR>(bx);
      }
      if (graphs) HIPCHK(hipGraphLaunch(P.gexec[TR][3 + first_x], st));
      else kry_partC(first_x, rh, rtol2);
      if (read_ctrl(0) == 0) break;
    }
    hipLaunchKernelGGL(k_accum_its, dim3((S + 255) / 256), dim3(256), 0, st, S, P.sc.as<double>(), P.stats.as<double>());
    return -1;
  }

  // Capture the launches `f` makes on this solver's stream as an instantiated graph.
  template <typename F>
  hipGraphExec_t capture(F&& f) {
    return capture_graph(st, std::forward<F>(f));
  }

  // fields, coarse coefficients, initial state, cleared status/stats
  void init(const double* theta) {
    const Map& m = P.m;
    fields(theta);
    hipLaunchKernelGGL(k_init_state, grid_cells(m, P.G.ncell), block_of(m), 0, st, m, P.G, phys, P.p.as<double>(),
                       P.c.as<double>());
    HIPCHK(hipMemsetAsync(P.status.p, 0, P.S * sizeof(int), st));
    HIPCHK(hipMemsetAsync(P.stats.p, 0, (size_t)P.S * 4 * sizeof(double), st));
  }

  // Extrapolation order of the first Newton guess at step n (-1: the inflow-aware rule of a
  // periodic recharge); constant once enough history exists.
  int guess_order(int n) const {
    if (!o.newton_extrapolate) return 0;
    if (o.newton_extrapolate >= 2 && pr.recharge_omega != 0.0) return -1;
    if (o.newton_extrapolate >= 3) return std::min(n, o.newton_extrapolate - 1);
    return n == 0 ? 0 : 1;
  }

  // Start of step n: c_old = c, Newton flags cleared, first guess extrapolated.  Inside a
  // captured graph the flags are cleared by a fill kernel, not a memset node.
  void step_prologue(int n, bool in_graph) {
    const int S = P.S;
    HIPCHK(hipMemcpyAsync(P.c_old.p, P.c.p, P.N * 8, hipMemcpyDeviceToDevice, st));
    if (in_graph) {
      hipLaunchKernelGGL(k_zero_i32, dim3((S + 255) / 256), dim3(256), 0, st, (size_t)S, P.ndone.as<int>());
      hipLaunchKernelGGL(k_zero_f64, dim3((2 * S + 255) / 256), dim3(256), 0, st, (size_t)2 * S, P.nhist.as<double>());
    } else {
      HIPCHK(hipMemsetAsync(P.ndone.p, 0, S * sizeof(int), st));
      HIPCHK(hipMemsetAsync(P.nhist.p, 0, (size_t)S * 2 * sizeof(double), st));
    }
    if (!o.newton_extrapolate) return;
    // Newton starts from a polynomial extrapolation of the last steps (u^0 itself on the
    // first step); the fixed point of the step does not depend on the guess
    const size_t n2 = P.N;
    const dim3 g((unsigned)((n2 + 255) / 256));
    const int order = guess_order(n);
    if (order >= 0 && o.newton_extrapolate >= 3) {
      const bool h3 = o.newton_extrapolate == 4;
      hipLaunchKernelGGL(k_extrapolate_poly, g, dim3(256), 0, st, n2, order, P.p.as<double>(), P.p_prev.as<double>(),
                         P.p_prev2.as<double>(), h3 ? P.p_prev3.as<double>() : nullptr);
      hipLaunchKernelGGL(k_extrapolate_poly, g, dim3(256), 0, st, n2, order, P.c.as<double>(), P.c_prev.as<double>(),
                         P.c_prev2.as<double>(), h3 ? P.c_prev3.as<double>() : nullptr);
      return;
    }
    double gp = n == 0 ? 0.0 : 1.0, gc = gp;
    if (n > 0 && order < 0) {
      // pressure follows the inflow almost instantly: scale its last increment by the
      // change of the inflow factor (linear in the forcing), bounded
      auto f = [&](int k) { return 1.0 + std::sin(pr.recharge_omega * k * phys.tau); };
      const double d0 = f(n) - f(n - 1), d1 = f(n + 1) - f(n);
      gp = std::fabs(d0) > 1e-3 ? std::max(-3.0, std::min(3.0, d1 / d0)) : 1.0;
      gc = 0.0;   // c starts from c^n: its increments do not follow the inflow factor
    }
    hipLaunchKernelGGL(k_extrapolate, g, dim3(256), 0, st, n2, gp, P.p.as<double>(), P.p_prev.as<double>());
    hipLaunchKernelGGL(k_extrapolate, g, dim3(256), 0, st, n2, gc, P.c.as<double>(), P.c_prev.as<double>());
  }

  // Newton update from vx: per-sample damping, convergence flags and statistics (ctrl[1]:
  // samples still iterating, ctrl[2]: samples that want a fresh Jacobian), then u += lam dx.
  void newton_update() {
    const Map& m = P.m;
    const int S = P.S;
    hipLaunchKernelGGL(k_delta_max, grid_red(m), block_of(m), 0, st, m, P.G.ncell, P.vx.as<double>(),
                       P.part.as<double>());
    zero_ctrl();
    hipLaunchKernelGGL(k_fin_newton, fin_grid(S), fin_block(S), 0, st, m, P.part.as<double>(),
                       pr.rho0 * pr.g * pr.Ly, o.newton_tol, o.newton_dc_max, P.lam.as<double>(), P.ndone.as<int>(),
                       P.status.as<int>(), P.stats.as<double>(), P.ctrl.as<int>(), P.nhist.as<double>(),
                       o.newton_jac_reuse);
    hipLaunchKernelGGL(k_newton_update, grid_cells(m, P.G.ncell), block_of(m), 0, st, m, P.G.ncell,
                       P.lam.as<double>(), P.vx.as<double>(), P.p.as<double>(), P.c.as<double>());
  }

  // The first Newton iteration of a step as a fixed kernel sequence with every decision on
  // the device: full assembly, exactly one BiCGStab iteration with both halves (per-sample
  // active flags and omega = 0 after a half-step exit mask the samples that are done), the
  // damped update and the convergence flags.  No prediction can stop a sample before its
  // first solve (the history was cleared), so nothing needs compacting before it.
  template <typename T>
  void newton_first_fixed() {
    assemble_all<T>();
    const double rtol2 = o.krylov_rtol * o.krylov_rtol;
    const bool bx = black_exact(o.krylov_rtol);
    const double* rh = P.R.as<double>();
    kry_init<false>(rh, -1.0, P.ndone.as<int>(), false, true, rtol2, true);
    kry_partA<T, false>(1, rh, bx, rtol2);
    kry_partB<T, false>(bx);
    kry_partC(1, rh, rtol2);
    hipLaunchKernelGGL(k_accum_its, dim3((P.S + 255) / 256), dim3(256), 0, st, P.S, P.sc.as<double>(),
                       P.stats.as<double>());
    newton_update();
  }

  static bool same_phys(const Phys& a, const Phys& b) {
    return a.rho0 == b.rho0 && a.drho == b.drho && a.rho1 == b.rho1 && a.mu == b.mu && a.g == b.g && a.Dm == b.Dm &&
           a.c_left == b.c_left && a.hx == b.hx && a.hy == b.hy && a.vol == b.vol && a.tau == b.tau && a.Ly == b.Ly &&
           a.Lx == b.Lx && a.uin_fac == b.uin_fac && a.qoi_xmin == b.qoi_xmin && a.right_dir == b.right_dir;
  }

  // Replay (capturing first when the plan has none for these settings) the step graph:
  // prologue + newton_first_fixed.  Returns after the launch; nothing is read back.
  template <typename T>
  void launch_step_graph(int n) {
    const int order = guess_order(n);
    if (!P.step_exec || !same_phys(P.step_phys, phys) || std::memcmp(&P.step_opts, &o, sizeof o) != 0 ||
        P.step_order != order) {
      P.drop_step_graph();
      P.step_exec = capture([&] {
        step_prologue(n, true);
        newton_first_fixed<T>();
      });
      P.step_phys = phys;
      P.step_opts = o;
      P.step_order = order;
    }
    HIPCHK(hipGraphLaunch(P.step_exec, st));
  }

  // one implicit-Euler step n -> n+1: damped Newton with multigrid-preconditioned BiCGStab
  template <typename T>
  void time_step(int n, int nsteps) {
    const Map& m = P.m;
    const int S = P.S;
    const dim3 bl = block_of(m);
    const Range range("henry step %d/%d %dx%d S=%d fp%d", n + 1, nsteps, P.nx, P.ny, S, P.prec);
    if (progress_every && (n % progress_every == 0 || n == nsteps - 1)) {
      std::fprintf(stderr, "[henry] %dx%d S=%d fp%d step %d/%d\n", P.nx, P.ny, S, P.prec, n + 1, nsteps);
      std::fflush(stderr);
    }
    // implicit Euler: boundary data at the end of the step, t = (n + 1) tau
    phys.uin_fac = 1.0 + std::sin(pr.recharge_omega * (n + 1) * phys.tau);
    // The whole first Newton iteration replayed as one graph, with one host read after it, once
    // the step's kernel arguments no longer change: constant inflow and a settled extrapolation
    // order (the first steps have less history).
    const int order = guess_order(n);
    const bool settled = order >= 0 && order == guess_order(n + 1);
    if (o.step_graphs && allow_graphs && !ctx->prof.on && pr.recharge_omega == 0.0 && settled &&
        o.newton_maxit > 1) {
      launch_step_graph<T>(n);
      const int remaining = read_ctrl(1);
      const bool fresh = P.h_ctrl[2] > 0;
      if (remaining > 0) {
        if (allow_compact && 4 * remaining <= 3 * S) compact_newton<T>(remaining, 1);
        else newton_loop<T>(1, fresh);
      }
    } else {
      step_prologue(n, false);
      newton_loop<T>(0);
    }
    hipLaunchKernelGGL(k_balance, grid_red(m), bl, 0, st, m, P.G, phys, P.p.as<double>(), P.c.as<double>(),
                       P.c_old.as<double>(), P.phi.as<double>(), P.K.as<double>(), P.uin.as<double>(),
                       P.part.as<double>());
    hipLaunchKernelGGL(k_fin_balance, fin_grid(S), fin_block(S), 0, st, m, phys, P.part.as<double>(),
                       P.uin.as<double>(), o.c_range_tol, P.stats.as<double>(), P.status.as<int>());
  }

  // Newton iterations it0.. of the current step on this plan's batch.  Once at most
  // 3/4 of the samples are still iterating, the rest of the step runs on a compacted
  // copy of those samples (compact_newton), so converged samples cost no bandwidth.
  // fresh0: the first of these iterations assembles J (else it keeps the Jacobian of the
  // previous iteration: a chord step).
  template <typename T>
  void newton_loop(int it0, bool fresh0 = true) {
    const int S = P.S;
    int remaining = S;
    bool fresh = fresh0;
    for (int it = it0; it < o.newton_maxit && remaining > 0; ++it) {
      if (fresh) assemble_all<T>();
      else assemble_residual();
      // predictive stops can leave few samples iterating before the solve: compact first
      const bool can_compact = allow_compact && o.newton_predict > 0.0 && it + 1 < o.newton_maxit;
      const int left = bicgstab<T, false>(P.R.as<double>(), -1.0, P.ndone.as<int>(), o.krylov_rtol, true,
                                          can_compact ? (3 * S) / 4 : -1);
      if (left >= 0) {
        if (left > 0) compact_newton<T>(left, it);
        return;
      }
      newton_update();
      remaining = read_ctrl(1);
      // chord iteration next (same J) while every iterating sample's update was small
      fresh = P.h_ctrl[2] > 0;
      if (allow_compact && remaining > 0 && 4 * remaining <= 3 * S && it + 1 < o.newton_maxit) {
        compact_newton<T>(remaining, it + 1);
        return;
      }
    }
    if (remaining > 0)
      hipLaunchKernelGGL(k_mark_unconverged, dim3((S + 255) / 256), dim3(256), 0, st, S, P.ndone.as<int>(),
                         P.status.as<int>());
  }

  bool allow_compact = true;

  // Gather the Sa samples still iterating into the compact sub-plan, finish their Newton
  // iterations there and scatter state, status and statistics back.
  template <typename T>
  void compact_newton(int Sa, int it0) {
    const int S = P.S;
    if (!P.compact) fail(HENRY_EDEVICE, "internal: plan without a compact sub-plan");
    Plan& Q = *P.compact;
    plan_set_samples(Q, Sa, o.red_blocks, o.sample_block);
    int* idx = P.cidx.as<int>();
    hipLaunchKernelGGL(k_compact_index, dim3(1), dim3(COMPACT_THREADS), 0, st, S, P.ndone.as<int>(), idx);
    auto gather = [&](const double* src, double* dst, size_t rows) {
      const size_t n = rows * Sa;
      hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows, S, Sa, idx, src, dst);
    };
    auto scatter = [&](const double* src, double* dst, size_t rows) {
      const size_t n = rows * Sa;
      hipLaunchKernelGGL(k_scatter_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows, S, Sa, idx, src, dst);
    };
    const size_t nc = (size_t)P.G.ncell;
    gather(P.p.as<double>(), Q.p.as<double>(), nc);
    gather(P.c.as<double>(), Q.c.as<double>(), nc);
    gather(P.c_old.as<double>(), Q.c_old.as<double>(), nc);
    gather(P.phi.as<double>(), Q.phi.as<double>(), nc);
    gather(P.K.as<double>(), Q.K.as<double>(), nc);
    gather(P.uin.as<double>(), Q.uin.as<double>(), 1);
    for (int k = 1; k < P.nlev; ++k) {
      gather(P.lv[k]->phi.as<double>(), Q.lv[k]->phi.as<double>(), P.lv[k]->ncell);
      gather(P.lv[k]->K.as<double>(), Q.lv[k]->K.as<double>(), P.lv[k]->ncell);
    }
    hipLaunchKernelGGL(k_gather_sample_info, dim3((Sa + 255) / 256), dim3(256), 0, st, Sa, idx, P.status.as<int>(),
                       P.stats.as<double>(), P.nhist.as<double>(), Q.status.as<int>(), Q.stats.as<double>(),
                       Q.nhist.as<double>());
    HIPCHK(hipMemsetAsync(Q.ndone.p, 0, Sa * sizeof(int), st));
    Solver sq(ctx, pr, o, Q, 1, st);
    sq.phys = phys;
    sq.allow_compact = false;
    sq.allow_graphs = false;
    sq.fwd_fp32_jacobian = fwd_fp32_jacobian;
    tl_untimed = true;
    try {
      sq.newton_loop<T>(it0);
    } catch (...) {
      tl_untimed = false;
      throw;
    }
    tl_untimed = false;
    scatter(Q.p.as<double>(), P.p.as<double>(), nc);
    scatter(Q.c.as<double>(), P.c.as<double>(), nc);
    hipLaunchKernelGGL(k_scatter_sample_info, dim3((Sa + 255) / 256), dim3(256), 0, st, Sa, idx, Q.status.as<int>(),
                       Q.stats.as<double>(), Q.ndone.as<int>(), Q.nhist.as<double>(), P.status.as<int>(),
                       P.stats.as<double>(), P.ndone.as<int>(), P.nhist.as<double>());
  }

  void qoi(double* out) {
    const Map& m = P.m;
    hipLaunchKernelGGL(k_qoi, grid_red(m), block_of(m), 0, st, m, P.G, phys, P.c.as<double>(), P.part.as<double>());
    hipLaunchKernelGGL(k_fin_sum, fin_grid(P.S), fin_block(P.S), 0, st, m, P.part.as<double>(), phys.vol, out);
  }

  int progress_every = 0;
  bool allow_graphs = true;

  template <typename T>
  void run(const henry_batch& B) {
    const char* pe = std::getenv("HENRY_PROGRESS");
    progress_every = pe ? std::max(1, std::atoi(pe)) : 0;
    init(B.theta);
    const int S = P.S;
    for (int n = 0; n < B.grid.nsteps; ++n) {
      time_step<T>(n, B.grid.nsteps);
      if (B.series) {
        hipLaunchKernelGGL(k_series, grid_red(P.m), block_of(P.m), 0, st, P.m, P.G, phys, P.c.as<double>(),
                           P.part.as<double>());
        hipLaunchKernelGGL(k_fin_series, fin_grid(S), fin_block(S), 0, st, P.m, P.part.as<double>(),
                           B.series + (size_t)n * NSERIES * S);
      }
    }
    if (B.qoi) qoi(B.qoi);
    if (B.c_T) HIPCHK(hipMemcpyAsync(B.c_T, P.c.p, P.N * 8, hipMemcpyDeviceToDevice, st));
    if (B.p_T) HIPCHK(hipMemcpyAsync(B.p_T, P.p.p, P.N * 8, hipMemcpyDeviceToDevice, st));
    if (B.status) HIPCHK(hipMemcpyAsync(B.status, P.status.p, S * sizeof(int), hipMemcpyDeviceToDevice, st));
    if (B.stats) HIPCHK(hipMemcpyAsync(B.stats, P.stats.p, (size_t)S * 4 * 8, hipMemcpyDeviceToDevice, st));
  }

  // Discrete adjoint: forward with checkpoints every C steps, then a reverse sweep that
  // recomputes each segment and solves J_n^T lam_n = rhs_n step by step.
  template <typename T>
  void adjoint(const double* theta, int nsteps, int C, double* qoi_out, double* grad, int* status_out) {
    fwd_fp32_jacobian = false;   // forward, recomputed and transposed solves all use the FP64 Jacobian
    const char* pe = std::getenv("HENRY_PROGRESS");
    progress_every = pe ? std::max(1, std::atoi(pe)) : 0;
    const Map& m = P.m;
    const int S = P.S;
    const size_t N = P.N, st2 = 2 * N * sizeof(double);
    const int ncp = nsteps / C + 1;
    ctx->adj_ck.alloc((size_t)ncp * 4 * st2);   // (p, c) and the three previous steps' (p, c)
    ctx->adj_seg.alloc((size_t)(C + 1) * st2);
    const int guess = o.adjoint_guess;
    ctx->adj_g.alloc((2 * N + 2 * N + S + (guess > 0 ? 2 * N : 0) + (guess > 1 ? 2 * N : 0)) * sizeof(double));
    double* ck = ctx->adj_ck.as<double>();
    double* seg = ctx->adj_seg.as<double>();
    double* gphi = ctx->adj_g.as<double>();
    double* gK = gphi + N;
    double* rhs = gK + N;            // 2N
    double* guin = rhs + 2 * N;      // S
    double* lam1 = guess > 0 ? guin + S : nullptr;          // lambda of the step solved last
    double* lam2 = guess > 1 ? lam1 + 2 * N : nullptr;      // and of the one before
    auto save = [&](double* dst) {
      HIPCHK(hipMemcpyAsync(dst, P.p.p, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(dst + N, P.c.p, N * 8, hipMemcpyDeviceToDevice, st));
    };
    auto load = [&](const double* src) {
      HIPCHK(hipMemcpyAsync(P.p.p, src, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(P.c.p, src + N, N * 8, hipMemcpyDeviceToDevice, st));
    };
    auto save_ck = [&](double* dst) {
      save(dst);
      HIPCHK(hipMemcpyAsync(dst + 2 * N, P.p_prev.p, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(dst + 3 * N, P.c_prev.p, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(dst + 4 * N, P.p_prev2.p, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(dst + 5 * N, P.c_prev2.p, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(dst + 6 * N, P.p_prev3.p, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(dst + 7 * N, P.c_prev3.p, N * 8, hipMemcpyDeviceToDevice, st));
    };
    auto load_ck = [&](const double* src) {
      load(src);
      HIPCHK(hipMemcpyAsync(P.p_prev.p, src + 2 * N, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(P.c_prev.p, src + 3 * N, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(P.p_prev2.p, src + 4 * N, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(P.c_prev2.p, src + 5 * N, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(P.p_prev3.p, src + 6 * N, N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(P.c_prev3.p, src + 7 * N, N * 8, hipMemcpyDeviceToDevice, st));
    };
    init(theta);
    save_ck(ck);
    for (int n = 0; n < nsteps; ++n) {
      time_step<T>(n, nsteps);
      if ((n + 1) % C == 0) save_ck(ck + (size_t)((n + 1) / C) * 8 * N);
    }
    if (qoi_out) qoi(qoi_out);
    const dim3 cg = grid_cells(m, P.G.ncell), bl = block_of(m), rg = grid_red(m);
    const size_t nz = 2 * N + S;
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((2 * N + 255) / 256)), dim3(256), 0, st, 2 * N, gphi);
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, st, (size_t)S, guin);
    (void)nz;
    hipLaunchKernelGGL(k_adj_rhs_final, cg, bl, 0, st, m, P.G, phys, P.c.as<double>(), rhs);
    const int nseg = (nsteps + C - 1) / C;
    const dim3 g2((unsigned)((2 * N + 255) / 256));
    int solved = 0;   // reverse steps solved so far
    for (int sg = nseg - 1; sg >= 0; --sg) {
      const int n0 = sg * C, n1 = std::min(n0 + C, nsteps);
      load_ck(ck + (size_t)sg * 8 * N);
      save(seg);
      for (int n = n0; n < n1; ++n) {
        time_step<T>(n, nsteps);
        save(seg + (size_t)(n + 1 - n0) * 2 * N);
      }
      for (int n = n1; n > n0; --n) {
        const Range range("henry adjoint step %d/%d %dx%d S=%d", n, nsteps, P.nx, P.ny, S);
        const double* un = seg + (size_t)(n - n0) * 2 * N;
        const double* um = seg + (size_t)(n - 1 - n0) * 2 * N;
        load(un);
        HIPCHK(hipMemcpyAsync(P.c_old.p, um + N, N * 8, hipMemcpyDeviceToDevice, st));
        assemble_all<T>();
        // first guess: lambda of the step after (guess 1) or its linear extrapolation
        // 2 lambda^{n+1} - lambda^{n+2} (guess 2); the tolerance stays relative to |rhs|
        const int gmode = std::min(guess, solved);
        if (gmode == 1)
          HIPCHK(hipMemcpyAsync(P.vx.p, lam1, 2 * N * sizeof(double), hipMemcpyDeviceToDevice, st));
        else if (gmode == 2)
          hipLaunchKernelGGL(k_axpby, g2, dim3(256), 0, st, 2 * N, 2.0, lam1, -1.0, lam2, P.vx.as<double>());
        bicgstab<T, true>(rhs, 1.0, nullptr, o.krylov_rtol_adjoint, false, -1, gmode > 0);   // every sample
        // step n ends at t = n tau: its inflow factor weights the sensitivity to the base inflow
        phys.uin_fac = 1.0 + std::sin(pr.recharge_omega * n * phys.tau);
        if (lam2) std::swap(lam1, lam2);
        if (lam1) HIPCHK(hipMemcpyAsync(lam1, P.vx.p, 2 * N * sizeof(double), hipMemcpyDeviceToDevice, st));
        ++solved;
        hipLaunchKernelGGL(k_adj_param, rg, bl, 0, st, m, P.G, phys, P.p.as<double>(), P.c.as<double>(),
                           P.c_old.as<double>(), P.phi.as<double>(), P.K.as<double>(), P.vx.as<double>(), gphi, gK,
                           P.part.as<double>());
        hipLaunchKernelGGL(k_fin_accum, fin_grid(S), fin_block(S), 0, st, m, P.part.as<double>(), guin);
        if (n > 1)
          hipLaunchKernelGGL(k_adj_rhs_prev, cg, bl, 0, st, m, P.G, phys, P.c_old.as<double>(), P.phi.as<double>(),
                             P.vx.as<double>(), rhs);
      }
    }
    hipLaunchKernelGGL(k_adj_theta, rg, bl, 0, st, m, P.G, phys, kl, fp, theta, P.K.as<double>(), gphi, gK,
                       P.part.as<double>());
    hipLaunchKernelGGL(k_fin_theta, fin_grid(S), fin_block(S), 0, st, m, P.part.as<double>(), guin,
                       pr.q_in * pr.q_in_amp, grad);
    if (status_out) HIPCHK(hipMemcpyAsync(status_out, P.status.p, S * sizeof(int), hipMemcpyDeviceToDevice, st));
  }

  int count_failed() {
    zero_ctrl();
    hipLaunchKernelGGL(k_count_nonzero, dim3((P.S + 255) / 256), dim3(256), 0, st, P.S, P.status.as<int>(),
                       P.ctrl.as<int>() + 2);
    return read_ctrl(2);
  }
};

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------
static void check_problem(const henry_problem* pr) {
  if (!pr) fail(HENRY_EINVAL, "problem is NULL");
  const double v[] = {pr->Lx, pr->Ly, pr->T, pr->rho0, pr->rho1, pr->mu, pr->g, pr->Dm, pr->K_mean, pr->corr_len};
  for (double x : v)
    if (!(std::isfinite(x) && x > 0)) fail(HENRY_EINVAL, "problem constants must be positive and finite");
  if (pr->n_kl_phi < 0 || pr->n_kl_phi > 4 || pr->n_kl_logK < 0 || pr->n_kl_logK > 8)
    fail(HENRY_EINVAL, "n_kl_phi must be in [0,4] and n_kl_logK in [0,8]");
  if (pr->field_model != 0 && pr->field_model != 1) fail(HENRY_EINVAL, "field_model must be 0 or 1");
  if (pr->field_model == 1 && !(std::isfinite(pr->kappa_kc) && pr->kappa_kc > 0))
    fail(HENRY_EINVAL, "kappa_kc must be positive and finite");
  if (!std::isfinite(pr->recharge_omega)) fail(HENRY_EINVAL, "recharge_omega must be finite");
  if (!std::isfinite(pr->qoi_xmin)) fail(HENRY_EINVAL, "qoi_xmin must be finite");
}

static void check_grid(const henry_problem& pr, henry_grid g) {
  if (g.nx < 2 || g.ny < 2 || g.nsteps < 1) fail(HENRY_EINVAL, "grid %dx%d, %d steps is invalid", g.nx, g.ny, g.nsteps);
  if (std::fabs(pr.Lx / g.nx - pr.Ly / g.ny) > 1e-12 * pr.Lx / g.nx)
    fail(HENRY_EINVAL, "cells must be square: Lx/nx = %g, Ly/ny = %g", pr.Lx / g.nx, pr.Ly / g.ny);
  if ((long long)g.nx * g.ny > (1LL << 26)) fail(HENRY_EINVAL, "grid too large");
}

static void check_opts(const henry_solver_opts& o) {
  if (o.mg_precision != 32 && o.mg_precision != 64) fail(HENRY_EINVAL, "mg_precision must be 32 or 64");
  if (o.nu_pre < 1 || o.nu_post < 0 || o.nu_pre > 8 || o.nu_post > 8) fail(HENRY_EINVAL, "nu_pre in [1,8], nu_post in [0,8]");
  if (o.coarse_nx < 1 || o.coarse_ny < 1) fail(HENRY_EINVAL, "coarse grid must be positive");
  if (!(o.newton_tol > 0) || !(o.krylov_rtol > 0) || !(o.newton_dc_max > 0) || !(o.krylov_rtol_adjoint > 0))
    fail(HENRY_EINVAL, "tolerances must be positive");
  if (o.newton_maxit < 1 || o.krylov_maxit < 1) fail(HENRY_EINVAL, "iteration limits must be positive");
  if (o.red_blocks < 0) fail(HENRY_EINVAL, "red_blocks must be >= 0");
  if (!(o.newton_predict >= 0.0 && o.newton_predict <= 1.0)) fail(HENRY_EINVAL, "newton_predict must be in [0, 1]");
  if (!(o.newton_jac_reuse >= 0.0)) fail(HENRY_EINVAL, "newton_jac_reuse must be >= 0");
  if (o.newton_extrapolate < 0 || o.newton_extrapolate > 4) fail(HENRY_EINVAL, "newton_extrapolate must be 0..4");
  if (o.adjoint_guess < 0 || o.adjoint_guess > 2) fail(HENRY_EINVAL, "adjoint_guess must be 0, 1 or 2");
  if (o.mg_cycle != 1 && o.mg_cycle != 2) fail(HENRY_EINVAL, "mg_cycle must be 1 (V) or 2 (W)");
  if (o.coarse_solver < 0 || o.coarse_solver > 2)
    fail(HENRY_EINVAL, "coarse_solver must be 0 (banded), 1 (dense) or 2 (pivoted band)");
  if (o.step_graphs != 0 && o.step_graphs != 1) fail(HENRY_EINVAL, "step_graphs must be 0 or 1");
  if (o.ragged_threads != 0 && o.ragged_threads != 1) fail(HENRY_EINVAL, "ragged_threads must be 0 or 1");
  if (o.sample_block != 0 && o.sample_block != 16 && o.sample_block != 32 && o.sample_block != 64)
    fail(HENRY_EINVAL, "sample_block must be 0, 16, 32 or 64");
  if (o.fuse_prolong != 0 && o.fuse_prolong != 1) fail(HENRY_EINVAL, "fuse_prolong must be 0 or 1");
  if (!(o.krylov_breakdown >= 0.0) || !std::isfinite(o.krylov_breakdown))
    fail(HENRY_EINVAL, "krylov_breakdown must be finite and >= 0");
}

static int theta_check(henry_ctx* ctx, const double* theta, int S) {
  DevBuf flag;
  flag.alloc(sizeof(int));
  HIPCHK(hipMemsetAsync(flag.p, 0, sizeof(int), ctx->stream));
  hipLaunchKernelGGL(k_check_finite, dim3((S * 13 + 255) / 256), dim3(256), 0, ctx->stream, (size_t)S * 13, theta,
                     flag.as<int>());
  int h = 0;
  HIPCHK(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return h;
}

template <typename F>
static int guarded(henry_ctx* ctx, F&& f) {
  if (!ctx) return HENRY_EINVAL;
  try {
    HIPCHK(hipSetDevice(ctx->device));
    int r = f();
    ctx->err.clear();
    return r;
  } catch (const HenryError& e) {
    ctx->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return HENRY_ENOMEM;
  } catch (const std::exception& e) {   // e.g. a host thread that could not start
    ctx->err = std::string("host runtime error: ") + e.what();
    return HENRY_EDEVICE;
  }
}

// ---------------------------------------------------------------------------
// ragged batches: merge batches that share a grid, run each grid on its own stream
// ---------------------------------------------------------------------------
struct Group {
  henry_grid grid{};
  int S = 0;
  std::vector<int> members, offs;
  DevBuf theta, c, p, qoi, status, stats, series;   // merged groups only
  hipStream_t stream = nullptr;
  int failed = 0;
  bool ok = true;
  HenryError err{0, ""};
};

static hipStream_t ctx_stream(henry_ctx* ctx, size_t k) {
  while (ctx->streams.size() <= k) {
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));   // default priority
    ctx->streams.push_back(s);
  }
  return ctx->streams[k];
}

static int solve_ragged(henry_ctx* ctx, const henry_problem& pr, const henry_solver_opts& o, henry_batch* batches,
                        int nb) {
  if (nb == 0) return 0;
  std::vector<std::unique_ptr<Group>> groups;
  for (int b = 0; b < nb; ++b) {
    const henry_grid& g = batches[b].grid;
    Group* G = nullptr;
    for (auto& q : groups)
      if (q->grid.nx == g.nx && q->grid.ny == g.ny && q->grid.nsteps == g.nsteps) G = q.get();
    if (!G) {
      groups.push_back(std::make_unique<Group>());
      G = groups.back().get();
      G->grid = g;
    }
    G->members.push_back(b);
    G->offs.push_back(G->S);
    G->S += batches[b].nsamples;
  }
  // most expensive first, so the longest dependency chain starts first
  std::stable_sort(groups.begin(), groups.end(), [](const auto& a, const auto& b) {
    return (double)a->grid.nx * a->grid.ny * a->grid.nsteps * a->S > (double)b->grid.nx * b->grid.ny * b->grid.nsteps * b->S;
  });
  // Work runs on the context's own streams (capturable, unlike the legacy default
  // stream), ordered after the caller's stream and joined back to it at the end.
  const bool multi = groups.size() > 1;
  hipEvent_t start = nullptr;
  HIPCHK(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  HIPCHK(hipEventRecord(start, ctx->stream));
  std::vector<Plan*> plans;
  std::vector<henry_batch> gb(groups.size());
  std::map<PlanKey, int> used;   // groups that share a plan shape (e.g. the same grid with other step counts)
  for (size_t k = 0; k < groups.size(); ++k) {
    Group& G = *groups[k];
    G.stream = ctx_stream(ctx, k);
    HIPCHK(hipStreamWaitEvent(G.stream, start, 0));
    const int inst = used[plan_key(G.grid.nx, G.grid.ny, G.S, o, 0)]++;
    plans.push_back(get_plan(ctx, G.grid.nx, G.grid.ny, G.S, o, inst));
    henry_batch& B = gb[k];
    B.grid = G.grid;
    B.nsamples = G.S;
    if (G.members.size() == 1) {
      B = batches[G.members[0]];
      continue;
    }
    const size_t N = (size_t)G.grid.nx * G.grid.ny * G.S;
    G.theta.alloc((size_t)G.S * 13 * 8);
    for (size_t i = 0; i < G.members.size(); ++i) {
      const henry_batch& M = batches[G.members[i]];
      HIPCHK(hipMemcpyAsync(G.theta.as<double>() + (size_t)G.offs[i] * 13, M.theta, (size_t)M.nsamples * 13 * 8,
                            hipMemcpyDeviceToDevice, G.stream));
    }
    G.c.alloc(N * 8);
    G.p.alloc(N * 8);
    G.qoi.alloc(G.S * 8);
    G.status.alloc(G.S * 4);
    G.stats.alloc((size_t)G.S * 4 * 8);
    bool want_series = false;
    for (int b : G.members) want_series = want_series || batches[b].series;
    if (want_series) G.series.alloc((size_t)G.grid.nsteps * NSERIES * G.S * 8);
    B.series = want_series ? G.series.as<double>() : nullptr;
    B.theta = G.theta.as<double>();
    B.c_T = G.c.as<double>();
    B.p_T = G.p.as<double>();
    B.qoi = G.qoi.as<double>();
    B.status = G.status.as<int>();
    B.stats = G.stats.as<double>();
  }
  auto work = [&](size_t k) {
    Group& G = *groups[k];
    const Range range("henry grid %dx%d S=%d steps=%d", G.grid.nx, G.grid.ny, G.S, G.grid.nsteps);
    try {
      HIPCHK(hipSetDevice(ctx->device));
      Solver sv(ctx, pr, o, *plans[k], G.grid.nsteps, G.stream);
      if (o.mg_precision == 32) sv.run<float>(gb[k]);
      else sv.run<double>(gb[k]);
      HIPCHK(hipGetLastError());
      G.failed = sv.count_failed();
    } catch (const HenryError& e) {
      G.ok = false;
      G.err = e;
    } catch (const std::bad_alloc&) {
      G.ok = false;
      G.err = HenryError{HENRY_ENOMEM, "host allocation failed"};
    } catch (const std::exception& e) {
      G.ok = false;
      G.err = HenryError{HENRY_EDEVICE, std::string("host runtime error: ") + e.what()};
    } catch (...) {
      G.ok = false;
      G.err = HenryError{HENRY_EDEVICE, "unknown host exception"};
    }
  };
  if (!multi || o.ragged_threads == 1) {
    for (size_t k = 0; k < groups.size(); ++k) work(k);
  } else {
    std::vector<std::thread> th;
    for (size_t k = 0; k < groups.size(); ++k) th.emplace_back(work, k);
    for (auto& t : th) t.join();
  }
  int failed = 0;
  for (auto& gp : groups) {
    Group& G = *gp;
    if (!G.ok) throw G.err;
    failed += G.failed;
    if (G.members.size() > 1) {
      const size_t nc = (size_t)G.grid.nx * G.grid.ny;
      for (size_t i = 0; i < G.members.size(); ++i) {
        const henry_batch& M = batches[G.members[i]];
        const size_t off = G.offs[i], Sb = M.nsamples, S = G.S;
        if (M.c_T)
          HIPCHK(hipMemcpy2DAsync(M.c_T, Sb * 8, G.c.as<double>() + off, S * 8, Sb * 8, nc, hipMemcpyDeviceToDevice,
                                  G.stream));
        if (M.p_T)
          HIPCHK(hipMemcpy2DAsync(M.p_T, Sb * 8, G.p.as<double>() + off, S * 8, Sb * 8, nc, hipMemcpyDeviceToDevice,
                                  G.stream));
        if (M.qoi) HIPCHK(hipMemcpyAsync(M.qoi, G.qoi.as<double>() + off, Sb * 8, hipMemcpyDeviceToDevice, G.stream));
        if (M.status)
          HIPCHK(hipMemcpyAsync(M.status, G.status.as<int>() + off, Sb * 4, hipMemcpyDeviceToDevice, G.stream));
        if (M.stats)
          HIPCHK(hipMemcpyAsync(M.stats, G.stats.as<double>() + off * 4, Sb * 4 * 8, hipMemcpyDeviceToDevice, G.stream));
        if (M.series)
          HIPCHK(hipMemcpy2DAsync(M.series, Sb * 8, G.series.as<double>() + off, S * 8, Sb * 8,
                                  (size_t)G.grid.nsteps * NSERIES, hipMemcpyDeviceToDevice, G.stream));
      }
    }
    hipEvent_t done = nullptr;
    HIPCHK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    HIPCHK(hipEventRecord(done, G.stream));
    HIPCHK(hipStreamWaitEvent(ctx->stream, done, 0));
    HIPCHK(hipEventDestroy(done));
  }
  // merged buffers are released only after the copies above have run
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipEventDestroy(start));
  return failed;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void henry_problem_default(henry_problem* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->Lx = 2.0;
  p->Ly = 1.0;
  p->T = 36000.0;
  p->rho0 = 1000.0;
  p->rho1 = 1025.0;
  p->mu = 1e-3;
  p->g = 9.81;
  p->Dm = 1.88571e-5;
  p->phi_mean = 0.35;
  p->phi_amp = 0.2;
  p->phi_min = 0.2;
  p->phi_max = 0.5;
  p->K_mean = 1.020408e-9;
  p->logK_amp = 0.5;
  p->corr_len = 0.5;
  p->q_in = 6.6e-5;
  p->q_in_amp = 0.1;
  p->n_kl_phi = 4;
  p->n_kl_logK = 8;
  p->right_c_dirichlet = 0;
  p->c_left = 0.0;
  p->field_model = 0;
  p->kappa_kc = 2.088415e-8;
  p->recharge_omega = 0.0;
  p->qoi_xmin = 1.0;
}

void henry_solver_opts_default(henry_solver_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->mg_precision = 64;
  o->coarse_nx = 8;
  o->coarse_ny = 4;
  o->nu_pre = 1;
  o->nu_post = 2;
  o->newton_tol = 1e-9;
  o->newton_dc_max = 2.0;
  o->newton_maxit = 200;
  o->krylov_rtol = 5e-2;
  o->krylov_maxit = 60;
  o->c_range_tol = 1e-8;
  o->use_graphs = 0;
  o->red_blocks = 4096;
  o->krylov_rtol_adjoint = 1e-8;
  o->mg_cycle = 1;
  o->adjoint_guess = 2;
  o->coarse_solver = 0;
  o->step_graphs = 1;
  o->ragged_threads = 0;
  o->sample_block = 0;
  o->fuse_prolong = 1;
  o->krylov_breakdown = 0.0;
  o->newton_extrapolate = 4;
  o->newton_predict = 1.0;
  o->newton_jac_reuse = 1e-3;
}

int henry_ctx_create(henry_ctx** out, int device, void* stream) {
  if (!out) return HENRY_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return HENRY_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return HENRY_EDEVICE;
  auto* c = new (std::nothrow) henry_ctx;
  if (!c) return HENRY_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  if (scratch_init(device) != hipSuccess) {
    delete c;
    return HENRY_EDEVICE;
  }
  if (hipHostMalloc((void**)&c->h_ctrl, 16 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return HENRY_EDEVICE;
  }
  *out = c;
  return HENRY_OK;
}

void henry_ctx_destroy(henry_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  try {
    c->prof.flush();
  } catch (const HenryError&) {
  }
  for (auto s : c->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  c->plans.clear();
  if (c->h_ctrl) (void)hipHostFree(c->h_ctrl);
  delete c;
}

const char* henry_last_error(const henry_ctx* c) { return c ? c->err.c_str() : "null context"; }

int henry_sample_fields(henry_ctx* ctx, const henry_problem* prob, henry_grid grid, int S, const double* theta,
                        double* phi, double* K, double* q_in) {
  return guarded(ctx, [&]() -> int {
    check_problem(prob);
    check_grid(*prob, grid);
    if (S < 1 || !theta) fail(HENRY_EINVAL, "S must be >= 1 and theta non-NULL");
    if (theta_check(ctx, theta, S)) fail(HENRY_EINVAL, "theta contains non-finite values");
    const Map m = make_map(S, grid.nx * grid.ny, 0);
    const Grid2 G{grid.nx, grid.ny, grid.nx * grid.ny};
    const Phys P = make_phys(*prob, grid.nx, grid.ny, grid.nsteps);
    const KLModes kl = make_kl(*prob);
    const FieldParams fp = make_fp(*prob);
    hipLaunchKernelGGL(k_fields, grid_cells(m, G.ncell), block_of(m), 0, ctx->stream, m, G, P, kl, fp, theta, phi, K,
                       q_in);
    HIPCHK(hipGetLastError());
    return HENRY_OK;
  });
}

int henry_solve_batch(henry_ctx* ctx, const henry_problem* prob, const henry_solver_opts* opts, henry_batch* batches,
                      int nbatches) {
  return guarded(ctx, [&]() -> int {
    check_problem(prob);
    henry_solver_opts o;
    if (opts) o = *opts;
    else henry_solver_opts_default(&o);
    check_opts(o);
    if (nbatches < 0 || (nbatches > 0 && !batches)) fail(HENRY_EINVAL, "batches");
    for (int b = 0; b < nbatches; ++b) {
      check_grid(*prob, batches[b].grid);
      if (batches[b].nsamples < 1 || !batches[b].theta) fail(HENRY_EINVAL, "batch %d: nsamples < 1 or theta NULL", b);
      if (theta_check(ctx, batches[b].theta, batches[b].nsamples)) fail(HENRY_EINVAL, "batch %d: non-finite theta", b);
    }
    const Range range("henry_solve_batch %d batches", nbatches);
    return solve_ragged(ctx, *prob, o, batches, nbatches);
  });
}

int henry_adjoint_batch(henry_ctx* ctx, const henry_problem* prob, const henry_solver_opts* opts, henry_grid grid,
                        int S, const double* theta, int checkpoint_every, double* qoi, double* dqoi_dtheta,
                        int* status) {
  return guarded(ctx, [&]() -> int {
    check_problem(prob);
    henry_solver_opts o;
    if (opts) o = *opts;
    else henry_solver_opts_default(&o);
    check_opts(o);
    check_grid(*prob, grid);
    if (S < 1 || !theta || !dqoi_dtheta) fail(HENRY_EINVAL, "S < 1, theta or dqoi_dtheta NULL");
    if (checkpoint_every < 1) fail(HENRY_EINVAL, "checkpoint_every must be >= 1");
    if (theta_check(ctx, theta, S)) fail(HENRY_EINVAL, "theta contains non-finite values");
    Plan* P = get_plan(ctx, grid.nx, grid.ny, S, o);
    const Range range("henry_adjoint_batch %dx%d S=%d steps=%d", grid.nx, grid.ny, S, grid.nsteps);
    hipStream_t st = ctx_stream(ctx, 0);
    hipEvent_t ev = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, ctx->stream));
    HIPCHK(hipStreamWaitEvent(st, ev, 0));
    Solver sv(ctx, *prob, o, *P, grid.nsteps, st);
    if (o.mg_precision == 32) sv.adjoint<float>(theta, grid.nsteps, checkpoint_every, qoi, dqoi_dtheta, status);
    else sv.adjoint<double>(theta, grid.nsteps, checkpoint_every, qoi, dqoi_dtheta, status);
    HIPCHK(hipGetLastError());
    const int nf = sv.count_failed();
    HIPCHK(hipEventRecord(ev, st));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ev, 0));
    HIPCHK(hipEventDestroy(ev));
    return nf;
  });
}

}  // extern "C"

// Shared body of mlmc_estimate and mlmc_estimate_noalloc.  `work` (device, `work_doubles`
// long) holds the per-level moments and the per-cell field moments; NULL: the context's own
// buffer, grown as needed.  Host bookkeeping uses fixed arrays (no host allocation either).
static int mlmc_estimate_impl(henry_ctx* ctx, int L, const int* m, const henry_grid* grids,
                              const double* const* g_fine, const double* const* g_coarse,
                              const double* const* c_fine, const double* const* c_coarse, double alpha, double* mean,
                              double* var_of_estimator, double* rmse, double* V_l, double* mean_field,
                              double* var_field, double* work, size_t work_doubles) {
  if (L < 0 || !m || !g_fine) fail(HENRY_EINVAL, "L, m or g_fine invalid");
  if (L + 1 > FieldLevels::MAXL) fail(HENRY_EUNSUPPORTED, "at most %d levels", FieldLevels::MAXL);
  for (int l = 0; l <= L; ++l) {
    if (m[l] < 1 || !g_fine[l]) fail(HENRY_EINVAL, "level %d: m < 1 or g_fine NULL", l);
    if (l > 0 && (!g_coarse || !g_coarse[l])) fail(HENRY_EINVAL, "level %d: g_coarse NULL", l);
  }
  const bool fields = c_fine && (mean_field || var_field);
  // workspace: [L+1][2] level moments, then per level [mean_f, var_f, mean_c, var_c] fields
  size_t off[FieldLevels::MAXL] = {};
  size_t need = 2 * (size_t)(L + 1);
  if (fields) {
    if (!grids) fail(HENRY_EINVAL, "grids required for field moments");
    for (int l = 0; l <= L; ++l) {
      if (!c_fine[l]) fail(HENRY_EINVAL, "level %d: c_fine NULL", l);
      if (l > 0 && (!c_coarse || !c_coarse[l])) fail(HENRY_EINVAL, "level %d: c_coarse NULL", l);
      if (grids[l].nx < 1 || grids[l].ny < 1) fail(HENRY_EINVAL, "level %d: empty grid", l);
      if (l > 0 && (grids[l].nx != 2 * grids[l - 1].nx || grids[l].ny != 2 * grids[l - 1].ny))
        fail(HENRY_EINVAL, "level %d grid is not a 2x refinement of level %d", l, l - 1);
      off[l] = need;
      need += 2 * (size_t)grids[l].nx * grids[l].ny + (l > 0 ? 2 * (size_t)grids[l - 1].nx * grids[l - 1].ny : 0);
    }
  }
  if (!work) {
    ctx->mlmc_tmp.alloc(need * sizeof(double));
    work = ctx->mlmc_tmp.as<double>();
  } else if (need > work_doubles) {
    fail(HENRY_EINVAL, "estimator workspace of %zu doubles exceeds the %zu available", need, work_doubles);
  }
  hipStream_t st = ctx->stream;
  // scalar estimator: per level mean and unbiased variance of Y_l (two-pass, fixed order)
  for (int l = 0; l <= L; ++l)
    hipLaunchKernelGGL(k_level_moments, dim3(1), dim3(256), 0, st, m[l], g_fine[l], l > 0 ? g_coarse[l] : nullptr,
                       work + 2 * l);
  if (fields) {
    const int nxL = grids[L].nx, nyL = grids[L].ny, ncL = nxL * nyL;
    for (int l = 0; l <= L; ++l) {
      const int nc = grids[l].nx * grids[l].ny;
      double* t = work + off[l];
      hipLaunchKernelGGL(k_cell_moments, dim3((nc + 255) / 256), dim3(256), 0, st, nc, m[l], c_fine[l], t, t + nc);
      if (l > 0) {
        const int ncc = grids[l - 1].nx * grids[l - 1].ny;
        hipLaunchKernelGGL(k_cell_moments, dim3((ncc + 255) / 256), dim3(256), 0, st, ncc, m[l], c_coarse[l],
                           t + 2 * nc, t + 2 * nc + ncc);
      }
    }
    FieldLevels fl{};
    fl.L = L;
    for (int l = 0; l <= L; ++l) {
      fl.nx[l] = grids[l].nx;
      fl.off[l] = (long long)off[l];
    }
    hipLaunchKernelGGL(k_field_accumulate, dim3((ncL + 255) / 256), dim3(256), 0, st, fl, nxL, nyL, work, mean_field,
                       var_field);
  }
  HIPCHK(hipGetLastError());
  double h[2 * FieldLevels::MAXL];
  HIPCHK(hipMemcpyAsync(h, work, 2 * (size_t)(L + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double mu = 0.0, var = 0.0;
  for (int l = 0; l <= L; ++l) {
    mu += h[2 * l];
    var += h[2 * l + 1] / m[l];
    if (V_l) V_l[l] = h[2 * l + 1];
  }
  const double bias = L > 0 ? std::fabs(h[2 * L]) / (std::pow(2.0, alpha) - 1.0) : 0.0;
  if (mean) *mean = mu;
  if (var_of_estimator) *var_of_estimator = var;
  if (rmse) *rmse = std::sqrt(var + bias * bias);
  return HENRY_OK;
}

extern "C" {

int mlmc_estimate(henry_ctx* ctx, int L, const int* m, const henry_grid* grids, const double* const* g_fine,
                  const double* const* g_coarse, const double* const* c_fine, const double* const* c_coarse,
                  double alpha, double* mean, double* var_of_estimator, double* rmse, double* V_l, double* mean_field,
                  double* var_field) {
  return guarded(ctx, [&]() -> int {
    return mlmc_estimate_impl(ctx, L, m, grids, g_fine, g_coarse, c_fine, c_coarse, alpha, mean, var_of_estimator,
                              rmse, V_l, mean_field, var_field, nullptr, 0);
  });
}

int mlmc_estimate_noalloc(henry_ctx* ctx, int L, const int* m, const henry_grid* grids, const double* const* g_fine,
                          const double* const* g_coarse, const double* const* c_fine, const double* const* c_coarse,
                          double alpha, double* mean, double* var_of_estimator, double* rmse, double* V_l,
                          double* mean_field, double* var_field) {
  return guarded(ctx, [&]() -> int {
    double* ws = (ctx->device >= 0 && ctx->device < MAX_DEVICES) ? g_scratch[ctx->device] : nullptr;
    if (!ws) fail(HENRY_EDEVICE, "estimator scratch address not recorded for device %d", ctx->device);
    return mlmc_estimate_impl(ctx, L, m, grids, g_fine, g_coarse, c_fine, c_coarse, alpha, mean, var_of_estimator,
                              rmse, V_l, mean_field, var_field, ws, (size_t)HENRY_NOALLOC_SCRATCH_DOUBLES);
  });
}

int mlmc_estimate_series(henry_ctx* ctx, int L, const int* m, const henry_grid* grids, int nq,
                         const double* const* s_fine, const double* const* s_coarse, double* mean,
                         double* var_of_estimator, double* Ymean_l, double* V_l) {
  return guarded(ctx, [&]() -> int {
    if (L < 0 || !m || !grids || !s_fine || nq < 1) fail(HENRY_EINVAL, "L, m, grids, s_fine or nq invalid");
    if (L + 1 > SeriesLevels::MAXL) fail(HENRY_EUNSUPPORTED, "at most %d levels", SeriesLevels::MAXL);
    SeriesLevels sl{};
    sl.L = L;
    sl.nq = nq;
    sl.r0 = grids[0].nsteps;
    if (sl.r0 < 1) fail(HENRY_EINVAL, "grids[0].nsteps must be >= 1");
    for (int l = 0; l <= L; ++l) {
      if (m[l] < 1 || !s_fine[l]) fail(HENRY_EINVAL, "level %d: m < 1 or s_fine NULL", l);
      if (grids[l].nsteps % sl.r0) fail(HENRY_EINVAL, "level %d: nsteps is not a multiple of level 0's", l);
      sl.m[l] = m[l];
      sl.f[l] = s_fine[l];
      sl.df[l] = grids[l].nsteps / sl.r0;
      if (l > 0) {
        if (!s_coarse || !s_coarse[l]) fail(HENRY_EINVAL, "level %d: s_coarse NULL", l);
        sl.c[l] = s_coarse[l];
        sl.dc[l] = grids[l - 1].nsteps / sl.r0;
      }
    }
    hipStream_t st = ctx->stream;
    const size_t n = (size_t)sl.r0 * nq;
    DevBuf tmp;
    double* ym = Ymean_l;
    double* vv = V_l;
    if (!ym || !vv) tmp.alloc(2 * (L + 1) * n * sizeof(double));
    if (!ym) ym = tmp.as<double>();
    if (!vv) vv = tmp.as<double>() + (L + 1) * n;
    hipLaunchKernelGGL(k_series_moments, dim3((unsigned)n, (unsigned)(L + 1)), dim3(256), 0, st, sl, ym, vv);
    hipLaunchKernelGGL(k_series_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sl, ym, vv, mean,
                       var_of_estimator);
    HIPCHK(hipGetLastError());
    if (tmp.p) HIPCHK(hipStreamSynchronize(st));   // tmp is freed on return
    return HENRY_OK;
  });
}

// least-squares fit of log2(v_l) = a + b l over the given levels; returns (b, 2^a)
static std::pair<double, double> fit_log2(const std::vector<int>& lv, const std::vector<double>& v) {
  const int n = (int)lv.size();
  double xm = 0.0, ym = 0.0;
  for (int i = 0; i < n; ++i) {
    xm += lv[i];
    ym += std::log2(v[i]);
  }
  xm /= n;
  ym /= n;
  double sxy = 0.0, sxx = 0.0;
  for (int i = 0; i < n; ++i) {
    sxy += (lv[i] - xm) * (std::log2(v[i]) - ym);
    sxx += (lv[i] - xm) * (lv[i] - xm);
  }
  const double b = sxy / sxx;
  return {b, std::exp2(ym - b * xm)};
}

int mlmc_plan(int Lp, const double* Ymean_abs, const double* V_l, const double* s_l, double eps, double E0,
              int max_level, long long* m_l, double* cost, double* rates) {
  if (Lp < 2 || !Ymean_abs || !V_l || !s_l || !m_l || !(eps > 0) || !(E0 > 0) || max_level < 1) return HENRY_EINVAL;
  for (int l = 0; l <= Lp; ++l)
    if (!(s_l[l] > 0) || !(V_l[l] > 0) || !(Ymean_abs[l] > 0) || !std::isfinite(Ymean_abs[l])) return HENRY_EINVAL;
  std::vector<int> lv;
  std::vector<double> ym, vv, ss;
  for (int l = 1; l <= Lp; ++l) {
    lv.push_back(l);
    ym.push_back(Ymean_abs[l]);
    vv.push_back(V_l[l]);
  }
  const auto fa = fit_log2(lv, ym), fb = fit_log2(lv, vv);
  const double alpha = -fa.first, c1 = fa.second, beta = -fb.first, c2 = fb.second;
  std::vector<int> lc;
  for (int l = 0; l <= Lp; ++l) {
    lc.push_back(l);
    ss.push_back(s_l[l]);
  }
  const auto fg = fit_log2(lc, ss);
  const double gamma = fg.first, c3 = fg.second;
  if (!(alpha > 0)) return HENRY_EINVAL;   // no weak convergence: no level count can meet the bias
  int L = max_level;
  for (int l = 1; l <= max_level; ++l)
    if (c1 * std::exp2(-alpha * l) / (std::exp2(alpha) - 1.0) <= eps * E0 / std::sqrt(2.0)) {
      L = l;
      break;
    }
  std::vector<double> V(L + 1), s(L + 1);
  for (int l = 0; l <= L; ++l) {
    V[l] = l <= Lp ? V_l[l] : c2 * std::exp2(-beta * l);
    s[l] = l <= Lp ? s_l[l] : c3 * std::exp2(gamma * l);
  }
  const int rc = mlmc_optimal_samples(L, V.data(), s.data(), eps * E0, m_l, cost);
  if (rc != HENRY_OK) return rc;
  if (rates) {
    rates[0] = alpha;
    rates[1] = beta;
    rates[2] = gamma;
    rates[3] = c1;
    rates[4] = c2;
    rates[5] = c3;
    // plain Monte Carlo at level L for the same accuracy (section 5, Test B4): Var g_0 of
    // the pilot stands in for Var g_L
    rates[6] = 2.0 / ((eps * E0) * (eps * E0)) * s[L] * V_l[0];
  }
  return L;
}

// ---------------------------------------------------------------------------
// kernel-level entry points (the solve's own kernels, one launch each)
// ---------------------------------------------------------------------------
int henry_assemble(henry_ctx* ctx, const henry_problem* prob, henry_grid grid, int S, const double* theta,
                   const double* p, const double* c, const double* c_old, int step, double* R, double* J) {
  return guarded(ctx, [&]() -> int {
    check_problem(prob);
    check_grid(*prob, grid);
    if (S < 1 || !theta || !p || !c || !c_old || !R || !J) fail(HENRY_EINVAL, "S < 1 or a NULL array");
    if (step < 0 || step >= grid.nsteps) fail(HENRY_EINVAL, "step %d outside 0..%d", step, grid.nsteps - 1);
    if (theta_check(ctx, theta, S)) fail(HENRY_EINVAL, "theta contains non-finite values");
    const Map m = make_map(S, grid.nx * grid.ny, 0);
    const Grid2 G{grid.nx, grid.ny, grid.nx * grid.ny};
    Phys P = make_phys(*prob, grid.nx, grid.ny, grid.nsteps);
    P.uin_fac = 1.0 + std::sin(prob->recharge_omega * (step + 1) * P.tau);   // the step ends at (step + 1) tau
    const size_t N = (size_t)G.ncell * S;
    ctx->kws.alloc((2 * N + S) * sizeof(double));
    double* phi = ctx->kws.as<double>();
    double* K = phi + N;
    double* uin = K + N;
    hipLaunchKernelGGL(k_fields, grid_cells(m, G.ncell), block_of(m), 0, ctx->stream, m, G, P, make_kl(*prob),
                       make_fp(*prob), theta, phi, K, uin);
    hipLaunchKernelGGL((k_assemble<true, double, false, true>), asm_grid(m, G), asm_block(m), asm_lds(m.SX), ctx->stream, m,
                       G, P, p, c, c_old, (const double*)phi, (const double*)K, (const double*)uin, R, J,
                       (float*)nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));   // the workspace may be regrown by the next call
    return HENRY_OK;
  });
}

int henry_jacobian_apply(henry_ctx* ctx, henry_grid grid, int S, const double* J, const double* x, double* y,
                         int transpose) {
  return guarded(ctx, [&]() -> int {
    if (grid.nx < 1 || grid.ny < 1 || S < 1 || !J || !x || !y) fail(HENRY_EINVAL, "grid, S or a NULL array");
    const Map m = make_map(S, grid.nx * grid.ny, 0);
    const Grid2 G{grid.nx, grid.ny, grid.nx * grid.ny};
    ctx->kws.alloc((size_t)m.ncb * S * sizeof(double));
    double* part = ctx->kws.as<double>();
    if (transpose)
      hipLaunchKernelGGL((k_spmv_dot<1, true>), grid_red(m), block_of(m), 0, ctx->stream, m, G, J, x, y, x, part,
                         (const double*)nullptr);
    else
      hipLaunchKernelGGL((k_spmv_dot<1, false>), grid_red(m), block_of(m), 0, ctx->stream, m, G, J, x, y, x, part,
                         (const double*)nullptr);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return HENRY_OK;
  });
}

int henry_gs_pass(henry_ctx* ctx, henry_grid grid, int S, const double* J, const double* b, double* x, int colour,
                  int transpose) {
  return guarded(ctx, [&]() -> int {
    if (grid.nx < 1 || grid.ny < 1 || S < 1 || !J || !b || !x) fail(HENRY_EINVAL, "grid, S or a NULL array");
    if (colour != 0 && colour != 1) fail(HENRY_EINVAL, "colour must be 0 (red) or 1 (black)");
    const Map m = make_map(S, grid.nx * grid.ny, 0);
    const Grid2 G{grid.nx, grid.ny, grid.nx * grid.ny};
    const dim3 gg = grid_cells(m, grid.ny * ((grid.nx + 1) / 2));
    if (transpose)
      hipLaunchKernelGGL((k_gs_colour<double, true, 0>), gg, block_of(m), 0, ctx->stream, m, G, G, colour, J, b, x,
                         (const double*)nullptr);
    else
      hipLaunchKernelGGL((k_gs_colour<double, false, 0>), gg, block_of(m), 0, ctx->stream, m, G, G, colour, J, b, x,
                         (const double*)nullptr);
    HIPCHK(hipGetLastError());
    return HENRY_OK;
  });
}

}  // extern "C"

template <typename T>
static void coarse_solve_t(henry_ctx* ctx, int solver, henry_grid g, int S, const T* J, const T* b, T* x, int tr,
                           void* ws) {
  const int nc = g.nx * g.ny, n = 2 * nc;
  hipStream_t st = ctx->stream;
  T* LU = static_cast<T*>(ws);
  if (solver == 1) {
    int* perm = reinterpret_cast<int*>(LU + (size_t)n * n * S);
    const size_t lds = dense_factor_lds<T>(n, 16);
    dense_factor_prepare<T>(lds);
    hipLaunchKernelGGL((k_dense_build<T>), dim3(n, S), dim3(256), 0, st, S, g.nx, g.ny, J, LU);
    hipLaunchKernelGGL((k_dense_factor<T, 16>), dim3(S), dim3(DENSE_THREADS), lds, st, n, LU, perm);
    if (tr)
      hipLaunchKernelGGL((k_dense_solve<T, true>), dim3(S), dim3(DENSE_SOLVE_THREADS), dense_solve_lds<T>(n), st, S, nc, LU,
                         (const int*)perm, b, x);
    else
      hipLaunchKernelGGL((k_dense_solve<T, false>), dim3(S), dim3(DENSE_SOLVE_THREADS), dense_solve_lds<T>(n), st, S, nc,
                         LU, (const int*)perm, b, x);
    return;
  }
  if (solver == 2) {
    int* piv = reinterpret_cast<int*>(LU + gb_stride(g.nx, g.ny) * S);
    hipLaunchKernelGGL((k_gb_factor<T>), dim3(S), dim3(GB_THREADS), gb_factor_lds<T>(g.ny), st, S, g.nx, g.ny, J, LU,
                       piv);
    if (tr)
      hipLaunchKernelGGL((k_gb_solve<T, true>), dim3(S), dim3(64), gb_solve_lds<T>(g.nx, g.ny), st, S, g.nx, g.ny,
                         (const T*)LU, (const int*)piv, b, x);
    else
      hipLaunchKernelGGL((k_gb_solve<T, false>), dim3(S), dim3(64), gb_solve_lds<T>(g.nx, g.ny), st, S, g.nx, g.ny,
                         (const T*)LU, (const int*)piv, b, x);
    return;
  }
  const int mb = g.ny;
  hipLaunchKernelGGL((k_band_factor<T>), dim3(S), dim3(64), (size_t)(mb + 1) * (mb + 1) * 4 * sizeof(T), st, S, g.nx,
                     g.ny, J, LU);
  const int CH = band_chunk<T>(nc, mb);
  if (tr)
    hipLaunchKernelGGL((k_band_solve_T<T>), dim3(S), dim3(64), band_solve_lds<T>(nc, mb, CH), st, S, g.nx, g.ny, CH,
                       (const T*)LU, b, x);
  else
    hipLaunchKernelGGL((k_band_solve<T>), dim3(S), dim3(64), band_solve_lds<T>(nc, mb, CH), st, S, g.nx, g.ny, CH,
                       (const T*)LU, b, x);
}

extern "C" {

int henry_coarse_solve(henry_ctx* ctx, int solver, int precision, henry_grid coarse, int S, const double* J,
                       const double* b, double* x, int transpose) {
  return guarded(ctx, [&]() -> int {
    if (coarse.nx < 1 || coarse.ny < 1 || S < 1 || !J || !b || !x) fail(HENRY_EINVAL, "grid, S or a NULL array");
    if (solver < 0 || solver > 2) fail(HENRY_EINVAL, "solver must be 0 (banded), 1 (dense) or 2 (pivoted band)");
    if (precision != 64 && precision != 32) fail(HENRY_EINVAL, "precision must be 64 or 32");
    const int nc = coarse.nx * coarse.ny, n = 2 * nc;
    const size_t N = (size_t)nc * S;
    const size_t tsz = precision == 64 ? 8 : 4;
    if (solver == 1) {
      const size_t need = precision == 64 ? dense_factor_lds<double>(n, 16) : dense_factor_lds<float>(n, 16);
      if (n % 16 || need > max_lds_per_block()) fail(HENRY_EUNSUPPORTED, "grid %dx%d: no dense LU", coarse.nx, coarse.ny);
    } else if (solver == 2) {
      check_gb_size(coarse.nx, coarse.ny, precision);
    } else {
      if (coarse.ny > 44 || band_solve_lds<double>(nc, coarse.ny, 1) > 64 * 1024)
        fail(HENRY_EUNSUPPORTED, "grid %dx%d: no banded LU", coarse.nx, coarse.ny);
    }
    const size_t fac = solver == 1   ? (size_t)n * n * S * tsz + (size_t)n * S * sizeof(int)
                       : solver == 2 ? gb_stride(coarse.nx, coarse.ny) * S * tsz + (size_t)n * S * sizeof(int)
                                     : (size_t)nc * (2 * coarse.ny + 1) * 4 * S * tsz;
    const size_t conv = precision == 32 ? (20 * N + 4 * N) * sizeof(float) : 0;   // FP32 copies of J, b and x
    ctx->kws.alloc(conv + fac);
    hipStream_t st = ctx->stream;
    if (precision == 64) {
      coarse_solve_t<double>(ctx, solver, coarse, S, J, b, x, transpose, ctx->kws.p);
    } else {
      float* J32 = ctx->kws.as<float>();
      float* b32 = J32 + 20 * N;
      float* x32 = b32 + 2 * N;
      hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)((20 * N + 255) / 256)), dim3(256), 0, st, 20 * N,
                         J, J32);
      hipLaunchKernelGGL((k_convert<double, float>), dim3((unsigned)((2 * N + 255) / 256)), dim3(256), 0, st, 2 * N, b,
                         b32);
      coarse_solve_t<float>(ctx, solver, coarse, S, J32, b32, x32, transpose, static_cast<char*>(ctx->kws.p) + conv);
      hipLaunchKernelGGL((k_convert<float, double>), dim3((unsigned)((2 * N + 255) / 256)), dim3(256), 0, st, 2 * N,
                         x32, x);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return HENRY_OK;
  });
}

int henry_autotune(henry_ctx* ctx, const henry_problem* prob, henry_solver_opts* opts, henry_grid grid, int S,
                   const double* theta, double* best_ms) {
  return guarded(ctx, [&]() -> int {
    check_problem(prob);
    if (!opts) fail(HENRY_EINVAL, "opts is NULL");
    check_opts(*opts);
    check_grid(*prob, grid);
    if (S < 1 || !theta) fail(HENRY_EINVAL, "S < 1 or theta NULL");
    if (theta_check(ctx, theta, S)) fail(HENRY_EINVAL, "theta contains non-finite values");
    hipStream_t st = ctx_stream(ctx, 0);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    HIPCHK(hipEventRecord(ev0, ctx->stream));
    HIPCHK(hipStreamWaitEvent(st, ev0, 0));
    const bool prof = ctx->prof.on;
    ctx->prof.on = false;
    std::vector<PlanKey> used;
    // time of one implicit-Euler step of the caller's batch: the first step (damped start) and
    // a repetition run untimed, so one-time costs (allocation, graph capture) are excluded and
    // a weaker but cheaper preconditioner is charged for its extra Newton iterations
    const int nsteps = std::max(4, grid.nsteps);
    auto time_of = [&](const henry_solver_opts& c) -> double {
      Plan* P = get_plan(ctx, grid.nx, grid.ny, S, c);
      used.push_back(plan_key(grid.nx, grid.ny, S, c, 0));
      Solver sv(ctx, *prob, c, *P, nsteps, st);
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        sv.init(theta);
        if (c.mg_precision == 32) sv.time_step<float>(0, nsteps);
        else sv.time_step<double>(0, nsteps);
        HIPCHK(hipEventRecord(ev0, st));
        if (c.mg_precision == 32) sv.time_step<float>(1, nsteps);
        else sv.time_step<double>(1, nsteps);
        HIPCHK(hipEventRecord(ev1, st));
        HIPCHK(hipEventSynchronize(ev1));
        HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
      }
      return ms;
    };
    // coordinate descent from the caller's options: one setting at a time over its candidates,
    // keeping the fastest (coarsest grid, smoother sweeps, thread map, prolongation fusion,
    // reduction blocks, hipGraphs)
    henry_solver_opts win = *opts;
    double best = time_of(win);
    auto sweep = [&](auto apply, const std::vector<std::array<int, 2>>& vals) {
      for (const auto& v : vals) {
        henry_solver_opts c = win;
        apply(c, v);
        if (std::memcmp(&c, &win, sizeof c) == 0) continue;
        const double t = time_of(c);
        if (t < best) {
          best = t;
          win = c;
        }
      }
    };
    sweep([](henry_solver_opts& c, std::array<int, 2> v) { c.coarse_nx = v[0]; c.coarse_ny = v[1]; },
          {{8, 4}, {16, 8}});
    sweep([](henry_solver_opts& c, std::array<int, 2> v) { c.nu_pre = v[0]; c.nu_post = v[1]; },
          {{1, 1}, {1, 2}, {2, 2}});
    sweep([](henry_solver_opts& c, std::array<int, 2> v) { c.sample_block = v[0]; }, {{0, 0}, {32, 0}, {16, 0}});
    sweep([](henry_solver_opts& c, std::array<int, 2> v) { c.fuse_prolong = v[0]; }, {{1, 0}, {0, 0}});
    sweep([](henry_solver_opts& c, std::array<int, 2> v) { c.red_blocks = v[0]; }, {{4096, 0}, {16384, 0}});
    sweep([](henry_solver_opts& c, std::array<int, 2> v) { c.use_graphs = v[0]; }, {{0, 0}, {1, 0}});
    // keep only the winner's plan
    const PlanKey keep = plan_key(grid.nx, grid.ny, S, win, 0);
    HIPCHK(hipStreamSynchronize(st));
    for (const auto& k : used)
      if (k != keep) ctx->plans.erase(k);
    ctx->prof.on = prof;
    *opts = win;
    if (best_ms) *best_ms = best;
    HIPCHK(hipEventRecord(ev0, st));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ev0, 0));
    HIPCHK(hipEventDestroy(ev0));
    HIPCHK(hipEventDestroy(ev1));
    return HENRY_OK;
  });
}

int henry_profile(henry_ctx* ctx, int enable) {
  return guarded(ctx, [&]() -> int {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (enable) {
      ctx->prof.reset();
      ctx->prof.on = true;
      ctx->host_syncs = 0;
      ctx->host_sync_ns = 0;
    } else {
      ctx->prof.on = false;
    }
    return HENRY_OK;
  });
}

int henry_profile_read(henry_ctx* ctx, int cls, long long* launches, long long* units, double* total_ms) {
  return guarded(ctx, [&]() -> int {
    if (cls < 0 || cls >= HENRY_PROF_NCLASS) fail(HENRY_EINVAL, "profile class %d", cls);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (cls == HENRY_PROF_HOST_SYNC) {
      if (launches) *launches = ctx->host_syncs.load();
      if (units) *units = 0;
      if (total_ms) *total_ms = ctx->host_sync_ns.load() * 1e-6;
      return HENRY_OK;
    }
    auto& k = ctx->prof.c[cls];
    // drain completed pairs without dropping the class's accumulated totals
    const size_t n = k.ring.size();
    for (size_t i = 0; i < n; ++i) {
      auto& sl = k.ring[(k.head + i) % n];
      ctx->prof.drain_one(k, sl);
      (void)hipEventDestroy(sl.a);
      (void)hipEventDestroy(sl.b);
    }
    k.ring.clear();
    k.head = k.used = 0;
    if (launches) *launches = k.launches;
    if (units) *units = k.units;
    if (total_ms) *total_ms = k.ms;
    return HENRY_OK;
  });
}

int mlmc_optimal_samples(int L, const double* V_l, const double* s_l, double eps, long long* m_l, double* cost) {
  if (L < 0 || !V_l || !s_l || !(eps > 0)) return HENRY_EINVAL;
  double tot = 0.0;
  for (int l = 0; l <= L; ++l) {
    if (!(V_l[l] >= 0) || !(s_l[l] > 0)) return HENRY_EINVAL;
    tot += std::sqrt(V_l[l] * s_l[l]);
  }
  double c = 0.0;
  for (int l = 0; l <= L; ++l) {
    const double mr = 2.0 / (eps * eps) * std::sqrt(V_l[l] / s_l[l]) * tot;
    const long long mi = (long long)std::ceil(mr);
    if (m_l) m_l[l] = mi;
    c += (double)mi * s_l[l];
  }
  if (cost) *cost = c;
  return HENRY_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// The paper's vertex-centred discretisation (section 2.3): batched time loop with damped
// Newton and right-preconditioned BiCGStab, the preconditioner symmetric four-colour block
// Gauss-Seidel sweeps from zero (the same arithmetic for every sample; per-sample decisions
// on the device, one host read per Krylov iteration and per Newton iteration).
// ---------------------------------------------------------------------------
namespace {

// The coarsest vertex grid is factored with partial pivoting in one workgroup per sample; its
// dense matrix may need more LDS than a launch gets by default: raise the limit once per device.
template <typename K>
static void vc_lds_prepare(K* kernel, size_t bytes) {
  static std::mutex mu;
  static bool done[64] = {};
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if (dev >= 0 && dev < 64 && done[dev]) return;
  HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes));
  if (dev >= 0 && dev < 64) done[dev] = true;
}
static size_t vc_dense_lds(int n, size_t tsz) { return (size_t)n * n * tsz + (size_t)n * sizeof(double) + 16; }

// one coarse level of the vertex-grid multigrid (the finest level is the solver's own data)
struct VCLevel {
  int nx, ny, nv, ne;
  Map m, me;
  Grid2 E;
  Phys P;
  DevBuf phi, K, p, c, co, Rs, J, b, x, r;
};

struct VCSolver {
  henry_ctx* ctx;
  const henry_problem& pr;
  const henry_solver_opts& o;
  int nx, ny, nsteps, S, nv, ne;
  hipStream_t st;
  Map m, me;
  Grid2 E;
  Phys P;
  size_t NV;
  DevBuf phi, K, uin, p, c, c_old, R, J, x, r, rh, pv, ph, v, sv, sh, t, part, sc, ctrl, status, mgr, LUc, pivc;
  // multigrid precision (mg_precision): 64, or 32 with the Jacobian stored in FP32 for the
  // cycle and the Krylov products, and the cycle's input and output rounded at its ends (mb, mx)
  int prec;
  size_t tsz;
  DevBuf mb, mx;
  DevBuf hp1, hp2, hp3, hc1, hc2, hc3;   // states of the last steps (first Newton guess)
  int* h_ctrl = nullptr;
  std::vector<std::unique_ptr<VCLevel>> lv;   // coarse levels 1.. of the multigrid preconditioner
  hipGraphExec_t gbody = nullptr;             // one BiCGStab iteration (use_graphs)

  VCSolver(henry_ctx* c_, const henry_problem& pr_, const henry_solver_opts& o_, henry_grid g, int S_,
           hipStream_t stream)
      : ctx(c_), pr(pr_), o(o_), nx(g.nx), ny(g.ny), nsteps(g.nsteps), S(S_), prec(o_.mg_precision),
        tsz(o_.mg_precision == 32 ? 4 : 8) {
    st = stream;
    nv = (nx + 1) * (ny + 1);
    ne = nx * ny;
    m = make_map(S, nv, o.red_blocks);
    me = make_map(S, ne, 0);
    E = Grid2{nx, ny, ne};
    P = make_phys(pr, nx, ny, nsteps);
    NV = (size_t)nv * S;
    phi.alloc((size_t)ne * S * 8);
    K.alloc((size_t)ne * S * 8);
    uin.alloc((size_t)S * 8);
    for (DevBuf* b : {&p, &c, &c_old, &hp1, &hp2, &hp3, &hc1, &hc2, &hc3}) b->alloc(NV * 8);
    for (DevBuf* b : {&R, &x, &r, &rh, &pv, &ph, &v, &sv, &sh, &t}) b->alloc(2 * NV * 8);
    J.alloc(36 * NV * tsz);
    part.alloc((size_t)3 * m.ncb * S * 8);
    sc.alloc((size_t)VC_NSC * S * 8);
    ctrl.alloc(sizeof(int));
    status.alloc((size_t)S * sizeof(int));
    HIPCHK(hipHostMalloc((void**)&h_ctrl, sizeof(int), hipHostMallocDefault));
    // halve while both element counts are even and stay at or above the coarse grid
    int gx = nx, gy = ny;
    while (gx % 2 == 0 && gy % 2 == 0 && gx / 2 >= o.coarse_nx && gy / 2 >= o.coarse_ny) {
      gx /= 2;
      gy /= 2;
      auto L = std::make_unique<VCLevel>();
      L->nx = gx;
      L->ny = gy;
      L->nv = (gx + 1) * (gy + 1);
      L->ne = gx * gy;
      L->m = make_map(S, L->nv, o.red_blocks);
      L->me = make_map(S, L->ne, 0);
      L->E = Grid2{gx, gy, L->ne};
      L->P = make_phys(pr, gx, gy, nsteps);
      const size_t n = (size_t)L->nv * S;
      L->phi.alloc((size_t)L->ne * S * 8);
      L->K.alloc((size_t)L->ne * S * 8);
      for (DevBuf* b : {&L->p, &L->c, &L->co}) b->alloc(n * 8);
      L->Rs.alloc(2 * n * 8);
      for (DevBuf* b : {&L->b, &L->x, &L->r}) b->alloc(2 * n * tsz);
      L->J.alloc(36 * n * tsz);
      lv.push_back(std::move(L));
    }
    // the coarsest grid's dense matrix must fit the LDS of one workgroup
    if (!lv.empty() && 2 * lv.back()->nv > VC_DENSE_MAX) lv.clear();
    if (!lv.empty()) {
      const int n = 2 * lv.back()->nv;
      mgr.alloc(2 * NV * tsz);
      LUc.alloc((size_t)n * n * S * tsz);
      pivc.alloc((size_t)n * S * sizeof(int));
      if (prec == 32) {
        vc_lds_prepare(&k_vc_dense_factor<float>, vc_dense_lds(VC_DENSE_MAX, 4));
        vc_lds_prepare(&k_vc_dense_solve<float>, vc_dense_lds(VC_DENSE_MAX, 4));
      } else {
        vc_lds_prepare(&k_vc_dense_factor<double>, vc_dense_lds(VC_DENSE_MAX, 8));
        vc_lds_prepare(&k_vc_dense_solve<double>, vc_dense_lds(VC_DENSE_MAX, 8));
      }
    }
    if (prec == 32) {
      mb.alloc(2 * NV * 4);
      mx.alloc(2 * NV * 4);
    }
  }
  ~VCSolver() {
    if (gbody) (void)hipGraphExecDestroy(gbody);
    if (h_ctrl) (void)hipHostFree(h_ctrl);
  }

  void fields(const double* theta) {
    hipLaunchKernelGGL(k_fields, grid_cells(me, ne), block_of(me), 0, st, me, E, P, make_kl(pr), make_fp(pr), theta,
                       phi.as<double>(), K.as<double>(), uin.as<double>());
    const double* pf = phi.as<double>();
    const double* kf = K.as<double>();
    Grid2 Ef = E;
    for (auto& L : lv) {
      hipLaunchKernelGGL(k_vc_coarse_fields, grid_cells(L->me, L->ne), block_of(L->me), 0, st, L->me, L->E, Ef, pf, kf,
                         L->phi.as<double>(), L->K.as<double>());
      pf = L->phi.as<double>();
      kf = L->K.as<double>();
      Ef = L->E;
    }
  }
  // Coarse operators at the injected state.  The coarsest grid's operator serves only its LU
  // factors, which are refreshed at the first Newton iteration of each step (refresh_coarsest)
  // and kept for the step's later iterations: the preconditioner changes, not the fixed point.
  void coarse_assemble(bool refresh_coarsest) {
    if (prec == 32) coarse_assemble_t<float>(refresh_coarsest);
    else coarse_assemble_t<double>(refresh_coarsest);
  }
  template <typename T>
  void coarse_assemble_t(bool refresh_coarsest) {
    const double *pf = p.as<double>(), *cf = c.as<double>(), *cof = c_old.as<double>();
    Grid2 Ef = E;
    for (auto& L : lv) {
      if (L == lv.back() && !refresh_coarsest) return;
      hipLaunchKernelGGL(k_vc_inject, grid_cells(L->m, L->nv), block_of(L->m), 0, st, L->m, L->E, Ef, pf, cf, cof,
                         L->p.as<double>(), L->c.as<double>(), L->co.as<double>());
      Phys Pl = L->P;
      Pl.uin_fac = P.uin_fac;
      hipLaunchKernelGGL((k_vc_assemble<true, T>), grid_cells(L->m, L->nv), block_of(L->m), 0, st, L->m, L->E, Pl,
                         (const double*)L->phi.as<double>(), (const double*)L->K.as<double>(),
                         (const double*)uin.as<double>(), (const double*)L->p.as<double>(),
                         (const double*)L->c.as<double>(), (const double*)L->co.as<double>(), L->Rs.as<double>(),
                         L->J.as<T>());
      pf = L->p.as<double>();
      cf = L->c.as<double>();
      cof = L->co.as<double>();
      Ef = L->E;
    }
    if (!lv.empty()) {
      const VCLevel& Lc = *lv.back();
      hipLaunchKernelGGL(k_vc_dense_factor<T>, dim3(S), dim3(256), vc_dense_lds(2 * Lc.nv, sizeof(T)), st, S, Lc.E,
                         (const T*)Lc.J.as<T>(), LUc.as<T>(), pivc.as<int>());
    }
  }
  // one V-cycle on level k (0: the fine grid) for J_k x = b from x = 0, in precision T
  template <typename T>
  void vcycle(int k, const T* b, T* xo) {
    const VCLevel* L = k > 0 ? lv[k - 1].get() : nullptr;
    const Map& mk = k > 0 ? L->m : m;
    const Grid2& Ek = k > 0 ? L->E : E;
    const int nvk = k > 0 ? L->nv : nv;
    const T* Jk = k > 0 ? L->J.as<T>() : J.as<T>();
    if (k == (int)lv.size()) {   // coarsest: the direct solve with this step's factors
      hipLaunchKernelGGL(k_vc_dense_solve<T>, dim3(S), dim3(64), vc_dense_lds(2 * nvk, sizeof(T)), st, S, Ek,
                         (const T*)LUc.as<T>(), (const int*)pivc.as<int>(), b, xo);
      return;
    }
    // x starts at zero: the first forward sweep skips the colours not yet swept, so x is not
    // cleared; the last colour swept (3) has a zero residual
    for (int sw = 0; sw < std::max(1, o.nu_pre); ++sw)
      for (int col = 0; col < 4; ++col) gs_pass<T>(k, mk, Ek, col, Jk, b, xo, sw == 0);
    T* rk = k > 0 ? L->r.as<T>() : mgr.as<T>();
    hipLaunchKernelGGL(k_vc_resid<T>, grid_cells(mk, nvk), block_of(mk), 0, st, mk, Ek, 3, Jk, b, (const T*)xo, rk);
    VCLevel* C = lv[k].get();
    hipLaunchKernelGGL(k_vc_restrict<T>, grid_cells(C->m, C->nv), block_of(C->m), 0, st, C->m, C->E, Ek, (const T*)rk,
                       C->b.as<T>());
    vcycle<T>(k + 1, C->b.as<T>(), C->x.as<T>());
    hipLaunchKernelGGL(k_vc_prolong_add<T>, grid_cells(mk, nvk), block_of(mk), 0, st, mk, Ek, C->E,
                       (const T*)C->x.as<T>(), xo);
    for (int sw = 0; sw < std::max(1, o.nu_post); ++sw)
      for (int col = 3; col >= 0; --col) gs_pass<T>(k, mk, Ek, col, Jk, b, xo);
  }
  // one colour pass on level k (first: of the first forward sweep from x = 0); the fine
  // grid's full passes are timed as HENRY_PROF_GS (units: the colour's vertex-samples)
  template <typename T>
  void gs_pass(int k, const Map& mk, const Grid2& Ek, int col, const T* Jk, const T* b, T* xo, bool first = false) {
    const dim3 g = grid_cells(mk, vc_colour_cells(Ek.nx, Ek.ny, 0));
    if (first) {
      hipLaunchKernelGGL((k_vc_gs<true, T>), g, block_of(mk), 0, st, mk, Ek, col, Jk, b, xo);
      return;
    }
    auto f = [&] { launch_timed(k_vc_gs<false, T>, g, block_of(mk), 0, st, mk, Ek, col, Jk, b, xo); };
    if (k == 0) timed(ctx, st, HENRY_PROF_GS, (long long)vc_colour_cells(Ek.nx, Ek.ny, col) * S, f);
    else f();
  }
  // residual R and, with_j, the Jacobian JJ (stored in the multigrid precision: FP64 or FP32)
  void assemble(bool with_j, const double* pp, const double* cc, const double* co, double* RR, void* JJ) {
    if (with_j)
      timed(ctx, st, HENRY_PROF_ASSEMBLE, (long long)NV, [&] {
        if (prec == 32)
          launch_timed((k_vc_assemble<true, float>), grid_cells(m, nv), block_of(m), 0, st, m, E, P,
                       (const double*)phi.as<double>(), (const double*)K.as<double>(),
                       (const double*)uin.as<double>(), pp, cc, co, RR, static_cast<float*>(JJ));
        else
          launch_timed((k_vc_assemble<true, double>), grid_cells(m, nv), block_of(m), 0, st, m, E, P,
                       (const double*)phi.as<double>(), (const double*)K.as<double>(),
                       (const double*)uin.as<double>(), pp, cc, co, RR, static_cast<double*>(JJ));
      });
    else
      hipLaunchKernelGGL((k_vc_assemble<false, double>), grid_cells(m, nv), block_of(m), 0, st, m, E, P,
                         (const double*)phi.as<double>(), (const double*)K.as<double>(),
                         (const double*)uin.as<double>(), pp, cc, co, RR, (double*)nullptr);
  }
  int read_ctrl() {
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipMemcpyAsync(h_ctrl, ctrl.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->host_syncs++;
    ctx->host_sync_ns += std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
    return *h_ctrl;
  }
  void zero_ctrl() { hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, (size_t)1, ctrl.as<int>()); }
  template <int NQ>
  void dots(VCPairs ab) {
    hipLaunchKernelGGL((k_vc_dots<NQ>), grid_red(m), block_of(m), 0, st, m, nv, ab, part.as<double>());
  }
  dim3 g2() const { return dim3((unsigned)((2 * NV + 255) / 256)); }
  // x = M^{-1} b: a multigrid V-cycle where the grid coarsens, else symmetric four-colour sweeps;
  // with the FP32 multigrid, b is rounded to FP32 on entry and the result widened on exit
  void precond(const double* b, double* xo) {
    if (prec == 64) {
      precond_t<double>(b, xo);
      return;
    }
    const dim3 g = g2();
    hipLaunchKernelGGL((k_convert<double, float>), g, dim3(256), 0, st, 2 * NV, b, mb.as<float>());
    precond_t<float>(mb.as<float>(), mx.as<float>());
    hipLaunchKernelGGL((k_convert<float, double>), g, dim3(256), 0, st, 2 * NV, (const float*)mx.as<float>(), xo);
  }
  template <typename T>
  void precond_t(const T* b, T* xo) {
    if (!lv.empty()) {
      vcycle<T>(0, b, xo);
      return;
    }
    const int sweeps = std::max(1, o.nu_pre + o.nu_post);
    for (int k = 0; k < sweeps; ++k) {
      for (int col = 0; col < 4; ++col) gs_pass<T>(0, m, E, col, (const T*)J.as<T>(), b, xo, k == 0);
      for (int col = 3; col >= 0; --col) gs_pass<T>(0, m, E, col, (const T*)J.as<T>(), b, xo);
    }
  }
  // y = J x with the stored Jacobian (FP32 with the FP32 multigrid), accumulated in FP64
  void spmv(const double* xi, double* yo) {
    timed(ctx, st, HENRY_PROF_SPMV, (long long)NV, [&] {
      if (prec == 32)
        launch_timed(k_vc_spmv<float>, grid_cells(m, nv), block_of(m), 0, st, m, E, (const float*)J.as<float>(), xi, yo);
      else
        launch_timed(k_vc_spmv<double>, grid_cells(m, nv), block_of(m), 0, st, m, E, (const double*)J.as<double>(), xi,
                     yo);
    });
  }
  // J x = -R (masked by the Newton flags); returns the iterations run
  int bicgstab() {
    double* scp = sc.as<double>();
    const dim3 fg = fin_grid(S), fb = fin_block(S);
    hipLaunchKernelGGL(k_vc_rhs, g2(), dim3(256), 0, st, 2 * NV, NV, S, (const double*)scp, (const double*)R.as<double>(),
                       x.as<double>(), r.as<double>(), pv.as<double>(), rh.as<double>());
    dots<1>(VCPairs{{r.as<double>(), nullptr, nullptr}, {r.as<double>(), nullptr, nullptr}});
    zero_ctrl();
    hipLaunchKernelGGL(k_vc_bicg_start, fg, fb, 0, st, m, (const double*)part.as<double>(), scp, ctrl.as<int>(),
                       o.newton_tol * o.newton_predict);
    if (read_ctrl() == 0) return 0;
    // the iteration's launches use fixed buffers and constants, so with use_graphs they are
    // captured once per solver and replayed
    const bool graphs = o.use_graphs && !ctx->prof.on;
    if (graphs && !gbody) gbody = capture_graph(st, [&] { iteration(); });
    int it = 0;
    for (; it < o.krylov_maxit; ++it) {
      if (graphs) HIPCHK(hipGraphLaunch(gbody, st));
      else iteration();
      if (read_ctrl() == 0) {
        ++it;
        break;
      }
    }
    return it;
  }
  // one BiCGStab iteration for every sample still iterating; ends with the count of those
  // still iterating in ctrl
  void iteration() {
    double* scp = sc.as<double>();
    const dim3 fg = fin_grid(S), fb = fin_block(S);
    const double rtol2 = o.krylov_rtol * o.krylov_rtol;
    precond(pv.as<double>(), ph.as<double>());
    spmv(ph.as<double>(), v.as<double>());
    dots<1>(VCPairs{{rh.as<double>(), nullptr, nullptr}, {v.as<double>(), nullptr, nullptr}});
    hipLaunchKernelGGL(k_vc_bicg_alpha, fg, fb, 0, st, m, (const double*)part.as<double>(), scp, status.as<int>());
    hipLaunchKernelGGL(k_vc_axpy_s, g2(), dim3(256), 0, st, 2 * NV, NV, S, (const double*)scp,
                       (const double*)r.as<double>(), (const double*)v.as<double>(), sv.as<double>());
    precond(sv.as<double>(), sh.as<double>());
    spmv(sh.as<double>(), t.as<double>());
    dots<3>(VCPairs{{sv.as<double>(), t.as<double>(), t.as<double>()}, {sv.as<double>(), sv.as<double>(), t.as<double>()}});
    hipLaunchKernelGGL(k_vc_bicg_omega, fg, fb, 0, st, m, (const double*)part.as<double>(), scp, rtol2);
    hipLaunchKernelGGL(k_vc_update_xr, g2(), dim3(256), 0, st, 2 * NV, NV, S, (const double*)scp,
                       (const double*)ph.as<double>(), (const double*)sh.as<double>(), (const double*)sv.as<double>(),
                       (const double*)t.as<double>(), x.as<double>(), r.as<double>());
    dots<2>(VCPairs{{rh.as<double>(), r.as<double>(), nullptr}, {r.as<double>(), r.as<double>(), nullptr}});
    zero_ctrl();
    hipLaunchKernelGGL(k_vc_bicg_beta, fg, fb, 0, st, m, (const double*)part.as<double>(), scp, rtol2,
                       status.as<int>(), ctrl.as<int>());
    hipLaunchKernelGGL(k_vc_update_p, g2(), dim3(256), 0, st, 2 * NV, NV, S, (const double*)scp,
                       (const double*)r.as<double>(), (const double*)v.as<double>(), pv.as<double>());
  }
  // First Newton guess of step n, as henry_solve_batch makes it (newton_extrapolate): a
  // polynomial through the last steps, or under a periodic recharge p moved along the inflow
  // factor's change and c kept; the step's fixed point does not depend on it.
  void guess(int n) {
    if (!o.newton_extrapolate) return;
    const dim3 g((unsigned)((NV + 255) / 256));
    const bool rech = pr.recharge_omega != 0.0;
    if (o.newton_extrapolate >= 3 && !rech) {
      const int order = std::min(n, o.newton_extrapolate - 1);
      const bool h3 = o.newton_extrapolate == 4;
      hipLaunchKernelGGL(k_extrapolate_poly, g, dim3(256), 0, st, NV, order, p.as<double>(), hp1.as<double>(),
                         hp2.as<double>(), h3 ? hp3.as<double>() : nullptr);
      hipLaunchKernelGGL(k_extrapolate_poly, g, dim3(256), 0, st, NV, order, c.as<double>(), hc1.as<double>(),
                         hc2.as<double>(), h3 ? hc3.as<double>() : nullptr);
      return;
    }
    double gp = n == 0 ? 0.0 : 1.0, gc = gp;
    if (n > 0 && rech && o.newton_extrapolate >= 2) {
      auto f = [&](int k) { return 1.0 + std::sin(pr.recharge_omega * k * P.tau); };
      const double d0 = f(n) - f(n - 1), d1 = f(n + 1) - f(n);
      gp = std::fabs(d0) > 1e-3 ? std::max(-3.0, std::min(3.0, d1 / d0)) : 1.0;
      gc = 0.0;
    }
    hipLaunchKernelGGL(k_extrapolate, g, dim3(256), 0, st, NV, gp, p.as<double>(), hp1.as<double>());
    hipLaunchKernelGGL(k_extrapolate, g, dim3(256), 0, st, NV, gc, c.as<double>(), hc1.as<double>());
  }
  void run(const double* theta, double* c_T, double* p_T, double* qoi, int* status_out, double* stats) {
    fields(theta);
    hipLaunchKernelGGL(k_vc_init, grid_cells(m, nv), block_of(m), 0, st, m, E, P, p.as<double>(), c.as<double>());
    HIPCHK(hipMemsetAsync(sc.p, 0, (size_t)VC_NSC * S * 8, st));
    HIPCHK(hipMemsetAsync(status.p, 0, (size_t)S * sizeof(int), st));
    double* scp = sc.as<double>();
    const double p_ref = pr.rho0 * pr.g * pr.Ly;
    const dim3 fg = fin_grid(S), fb = fin_block(S);
    for (int n = 0; n < nsteps; ++n) {
      const Range range("henry vc step %d/%d %dx%d S=%d", n + 1, nsteps, nx, ny, S);
      P.uin_fac = 1.0 + std::sin(pr.recharge_omega * (n + 1) * P.tau);
      HIPCHK(hipMemcpyAsync(c_old.p, c.p, NV * 8, hipMemcpyDeviceToDevice, st));
      guess(n);
      hipLaunchKernelGGL(k_vc_step_start, fg, fb, 0, st, S, (const int*)status.as<int>(), scp);
      bool done = false;
      for (int it = 0; it < o.newton_maxit && !done; ++it) {
        assemble(true, p.as<double>(), c.as<double>(), c_old.as<double>(), R.as<double>(), J.p);
        coarse_assemble(it == 0);
        bicgstab();
        hipLaunchKernelGGL(k_vc_absmax, grid_red(m), block_of(m), 0, st, m, nv, (const double*)x.as<double>(),
                           part.as<double>());
        zero_ctrl();
        hipLaunchKernelGGL(k_vc_newton_fin, fg, fb, 0, st, m, (const double*)part.as<double>(), scp, o.newton_tol, p_ref,
                           o.newton_dc_max, status.as<int>(), ctrl.as<int>());
        hipLaunchKernelGGL(k_vc_newton_update, dim3((unsigned)((NV + 255) / 256)), dim3(256), 0, st, NV, S,
                           (const double*)scp, (const double*)x.as<double>(), p.as<double>(), c.as<double>());
        done = read_ctrl() == 0;
      }
      hipLaunchKernelGGL(k_vc_step_end, fg, fb, 0, st, S, status.as<int>(), (const double*)scp);
    }
    if (qoi) {
      hipLaunchKernelGGL(k_vc_qoi, grid_red(m), block_of(m), 0, st, m, E, P, (const double*)c.as<double>(),
                         part.as<double>());
      hipLaunchKernelGGL(k_fin_sum, fg, fb, 0, st, m, (const double*)part.as<double>(), 1.0, qoi);
    }
    if (c_T) HIPCHK(hipMemcpyAsync(c_T, c.p, NV * 8, hipMemcpyDeviceToDevice, st));
    if (p_T) HIPCHK(hipMemcpyAsync(p_T, p.p, NV * 8, hipMemcpyDeviceToDevice, st));
    if (status_out) HIPCHK(hipMemcpyAsync(status_out, status.p, (size_t)S * sizeof(int), hipMemcpyDeviceToDevice, st));
    if (stats)
      hipLaunchKernelGGL(k_vc_stats, fg, fb, 0, st, S, (const double*)scp, stats);
  }
};

static void check_vc_grid(const henry_problem& pr, henry_grid g) {
  if (g.nx < 2 || g.ny < 2 || g.nsteps < 1) fail(HENRY_EINVAL, "grid %dx%d, %d steps is invalid", g.nx, g.ny, g.nsteps);
  if ((long long)(g.nx + 1) * (g.ny + 1) > (1LL << 24)) fail(HENRY_EINVAL, "grid too large");
  (void)pr;
}

}  // namespace

extern "C" {

int henry_vc_assemble(henry_ctx* ctx, const henry_problem* prob, henry_grid grid, int S, const double* theta,
                      const double* p, const double* c, const double* c_old, int step, double* R, double* J) {
  return guarded(ctx, [&]() -> int {
    check_problem(prob);
    check_vc_grid(*prob, grid);
    if (S < 1 || !theta || !p || !c || !c_old || !R || !J) fail(HENRY_EINVAL, "S < 1 or a NULL array");
    if (step < 0 || step >= grid.nsteps) fail(HENRY_EINVAL, "step %d outside 0..%d", step, grid.nsteps - 1);
    if (theta_check(ctx, theta, S)) fail(HENRY_EINVAL, "theta contains non-finite values");
    henry_solver_opts o;
    henry_solver_opts_default(&o);
    VCSolver sv(ctx, *prob, o, grid, S, ctx->stream);
    sv.P.uin_fac = 1.0 + std::sin(prob->recharge_omega * (step + 1) * sv.P.tau);
    sv.fields(theta);
    sv.assemble(true, p, c, c_old, R, J);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return HENRY_OK;
  });
}

int henry_vc_solve_batch(henry_ctx* ctx, const henry_problem* prob, const henry_solver_opts* opts,
                         henry_batch* batches, int nbatches) {
  return guarded(ctx, [&]() -> int {
    check_problem(prob);
    henry_solver_opts o;
    if (opts) o = *opts;
    else henry_solver_opts_default(&o);
    check_opts(o);
    if (nbatches < 0 || (nbatches > 0 && !batches)) fail(HENRY_EINVAL, "nbatches < 0 or batches NULL");
    for (int k = 0; k < nbatches; ++k) {
      const henry_batch& B = batches[k];
      check_vc_grid(*prob, B.grid);
      if (B.nsamples < 1 || !B.theta) fail(HENRY_EINVAL, "batch %d: nsamples < 1 or theta NULL", k);
      if (B.series) fail(HENRY_EINVAL, "batch %d: the vertex-centred solve has no series output", k);
      if (theta_check(ctx, B.theta, B.nsamples)) fail(HENRY_EINVAL, "batch %d: theta contains non-finite values", k);
    }
    if (nbatches == 0) return 0;
    const Range range("henry_vc_solve_batch %d batches", nbatches);
    // one library stream per batch (created here, before any worker starts), each ordered after
    // the caller's stream; the batches run from their own host threads unless ragged_threads is 1
    std::vector<hipStream_t> streams(nbatches);
    for (int k = 0; k < nbatches; ++k) streams[k] = ctx_stream(ctx, (size_t)k);
    hipEvent_t ev = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, ctx->stream));
    for (int k = 0; k < nbatches; ++k) HIPCHK(hipStreamWaitEvent(streams[k], ev, 0));
    HIPCHK(hipEventDestroy(ev));
    // every solver's device and pinned memory is allocated here and freed after the join, so no
    // worker allocates or frees while another captures a graph or synchronises its stream
    std::vector<std::unique_ptr<VCSolver>> solvers;
    for (int k = 0; k < nbatches; ++k)
      solvers.push_back(std::make_unique<VCSolver>(ctx, *prob, o, batches[k].grid, batches[k].nsamples, streams[k]));
    std::vector<int> nfail(nbatches, 0), ok(nbatches, 1);
    std::vector<std::vector<int>> hs(nbatches);
    for (int k = 0; k < nbatches; ++k) hs[k].resize(batches[k].nsamples);
    std::vector<HenryError> err(nbatches, HenryError{0, ""});
    auto work = [&](int k) {
      try {
        HIPCHK(hipSetDevice(ctx->device));
        const henry_batch& B = batches[k];
        const Range r("henry vc grid %dx%d S=%d steps=%d", B.grid.nx, B.grid.ny, B.nsamples, B.grid.nsteps);
        VCSolver& sv = *solvers[k];
        sv.run(B.theta, B.c_T, B.p_T, B.qoi, B.status, B.stats);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(hs[k].data(), sv.status.p, (size_t)B.nsamples * sizeof(int), hipMemcpyDeviceToHost,
                              streams[k]));
        HIPCHK(hipStreamSynchronize(streams[k]));
        for (int v : hs[k]) nfail[k] += v != 0;
      } catch (const HenryError& e) {
        ok[k] = 0;
        err[k] = e;
      } catch (const std::bad_alloc&) {
        ok[k] = 0;
        err[k] = HenryError{HENRY_ENOMEM, "host allocation failed"};
      } catch (const std::exception& e) {
        ok[k] = 0;
        err[k] = HenryError{HENRY_EDEVICE, std::string("host runtime error: ") + e.what()};
      } catch (...) {
        ok[k] = 0;
        err[k] = HenryError{HENRY_EDEVICE, "unknown host exception"};
      }
    };
    if (nbatches == 1 || o.ragged_threads == 1) {
      for (int k = 0; k < nbatches; ++k) work(k);
    } else {
      std::vector<std::thread> th;
      for (int k = 0; k < nbatches; ++k) th.emplace_back(work, k);
      for (auto& t : th) t.join();
    }
    int failed = 0;
    for (int k = 0; k < nbatches; ++k) {
      if (!ok[k]) throw err[k];
      failed += nfail[k];
    }
    return failed;
  });
}

int henry_vc_solve(henry_ctx* ctx, const henry_problem* prob, const henry_solver_opts* opts, henry_grid grid, int S,
                   const double* theta, double* c_T, double* p_T, double* qoi, int* status, double* stats) {
  return guarded(ctx, [&]() -> int {
    check_problem(prob);
    henry_solver_opts o;
    if (opts) o = *opts;
    else henry_solver_opts_default(&o);
    check_opts(o);
    check_vc_grid(*prob, grid);
    if (S < 1 || !theta) fail(HENRY_EINVAL, "S < 1 or theta NULL");
    if (theta_check(ctx, theta, S)) fail(HENRY_EINVAL, "theta contains non-finite values");
    const Range range("henry_vc_solve %dx%d S=%d steps=%d", grid.nx, grid.ny, S, grid.nsteps);
    // the solve runs on the library's own stream (graphs cannot be captured on the legacy
    // default stream), ordered after the caller's stream and synchronised before returning
    hipStream_t st = ctx_stream(ctx, 0);
    hipEvent_t ev = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, ctx->stream));
    HIPCHK(hipStreamWaitEvent(st, ev, 0));
    HIPCHK(hipEventDestroy(ev));
    VCSolver sv(ctx, *prob, o, grid, S, st);
    sv.run(theta, c_T, p_T, qoi, status, stats);
    HIPCHK(hipGetLastError());
    int nf = 0;
    std::vector<int> hs(S);
    HIPCHK(hipMemcpyAsync(hs.data(), sv.status.p, (size_t)S * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int s = 0; s < S; ++s) nf += hs[s] != 0;
    return nf;
  });
}

}  // extern "C"
