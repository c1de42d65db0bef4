/*
 * henry.h -- C ABI of libhenry: batched stochastic Henry problem solves and the
 * multilevel Monte Carlo estimator on one AMD Instinct MI355X (gfx950).
 *
 * Method (arXiv 2403.17018):
 *   - model: fluid and salt mass balance with Darcy flow, linear density, constant
 *     viscosity, D = phi*Dm*I (section 2.1, eqs. e_cont_eq, e_tran_eq, e_Darcy_vel,
 *     e_lin_density, e_mol_diff; boundary conditions of section 2.1);
 *   - discretisation: finite volumes with upwinding and implicit Euler; Newton for the
 *     nonlinear step; BiCGStab preconditioned by a geometric multigrid V-cycle with a
 *     direct coarse-grid solve (section 2.3);
 *   - uncertainty: porosity, permeability and recharge driven by a parameter vector
 *     theta (section 2.2 and section 4 "Uncertain porosity and recharge");
 *   - MLMC telescoping estimator, variances and optimal sample numbers (section 3,
 *     eqs. EgL, A, goal_variance, M_ell, total_cost_MLMC, MSE).
 *
 * Conventions
 *   - Array arguments are DEVICE pointers owned by the caller unless marked "host".
 *     The library never frees caller memory.
 *   - Per-cell-per-sample arrays use layout [j][i][s]: sample fastest, then cell
 *     column i (x direction, nx cells), then cell row j (y direction, from the
 *     bottom y = -Ly up to y = 0).  Index = (j*nx + i)*S + s.
 *   - theta is [S][13] row-major: xi_0..3 (porosity KL coefficients, U[-1,1]),
 *     eta_0..7 (log-permeability KL coefficients, N(0,1)), zeta (recharge, U[-1,1]).
 *   - Work is enqueued on the context's HIP stream; calls that return per-sample
 *     failure counts synchronise that stream before returning.
 *   - Return codes: 0 = success; < 0 = hard error (below); > 0 = number of samples
 *     whose status is not HENRY_STATUS_OK (soft failure; outputs are still written).
 *     henry_last_error() describes the last hard error of a context.
 *   - Workspace (multigrid hierarchy, Krylov vectors, coarse factors) is allocated by
 *     the library inside the context and reused between calls of the same shape.
 */
#ifndef HENRY_H
#define HENRY_H

#if defined(__GNUC__)
#define HENRY_API __attribute__((visibility("default")))
#else
#define HENRY_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define HENRY_NTHETA 13

enum henry_error {
  HENRY_OK = 0,
  HENRY_EINVAL = -1,       /* invalid argument (shape, NULL pointer, non-finite theta) */
  HENRY_EDEVICE = -2,      /* a HIP runtime call failed */
  HENRY_ENOMEM = -3,       /* device allocation failed */
  HENRY_EUNSUPPORTED = -4  /* valid but unsupported option */
};

enum henry_sample_status {
  HENRY_STATUS_OK = 0,
  HENRY_STATUS_NEWTON = 1,     /* Newton did not converge within newton_maxit in some step */
  HENRY_STATUS_KRYLOV = 2,     /* BiCGStab breakdown (rho or omega vanished) */
  HENRY_STATUS_NONFINITE = 3,  /* a non-finite update was produced; the sample was frozen */
  HENRY_STATUS_RANGE = 4       /* c left [-c_range_tol, 1 + c_range_tol] */
};

typedef struct henry_ctx henry_ctx;

/* Physical problem.  Defaults (henry_problem_default): paper Table 1 with the
 * studied workload's g = 9.81 and rho1 = 1025; domain [0,2]x[-1,0] m; T = 36000 s. */
typedef struct {
  double Lx, Ly;          /* domain [0,Lx] x [-Ly,0], m */
  double T;               /* final time, s */
  double rho0, rho1;      /* fresh water and brine density, kg/m^3 (eq. e_lin_density) */
  double mu;              /* viscosity, Pa s */
  double g;               /* gravity, m/s^2 */
  double Dm;              /* diffusion coefficient, m^2/s (D = phi Dm I, eq. e_mol_diff) */
  double phi_mean, phi_amp, phi_min, phi_max;  /* phi = clip(phi_mean(1+phi_amp*sum sqrt(lam)xi e), min, max) */
  double K_mean, logK_amp;                     /* ln K = ln K_mean + logK_amp*sum sqrt(lam) eta e */
  double corr_len;        /* exponential covariance correlation length, m */
  double q_in, q_in_amp;  /* left inflow velocity u_in = q_in (1 + q_in_amp zeta), m/s */
  int n_kl_phi, n_kl_logK;/* KL modes used (<= 4 and <= 8) */
  int right_c_dirichlet;  /* 0: c = 1 carried by inflow on the right side only;
                             1: additionally diffusive Dirichlet c = 1 (paper section 2.1) */
  double c_left;          /* c of the left inflow and its Dirichlet value (0) */
  int field_model;        /* 0: the KL fields above [0]; 1: the paper's own model (section 4):
                             phi = phi_mean C0 C1 C2 (eq. poro_2levels) with xi_1 = theta[0],
                             xi_2 = theta[1]: C0 = 1.2(1 + 0.2 xi_1) for y < -0.8, else 1;
                             C1 = 1 + 0.15(xi_2 cos(pi x/2) - xi_2 sin(2 pi y) + xi_1 cos(2 pi x));
                             C2 = 1 + 0.2(xi_1 sin(64 pi x) + xi_2 sin(32 pi y)); K by
                             Kozeny-Carman (eq. e_perm_Kozeny_Carman); phi_amp, phi_min,
                             phi_max, K_mean, logK_amp and the KL settings are unused */
  double kappa_kc;        /* Kozeny-Carman scale: K = kappa_kc phi^3 / (1 - phi^2), m^2 [2.088415e-8] */
  double recharge_omega;  /* the left inflow of the step ending at t is u_in (1 + sin(recharge_omega t))
                             (eq. e_recharge_of_param: pi/40 rad/s); 0: constant [0] */
  double qoi_xmin;        /* the QoI is the salt mass in the cells whose centre lies in x > qoi_xmin, m [1.0] */
} henry_problem;

/* One mesh level: nx x ny square cells (h = Lx/nx = Ly/ny), nsteps implicit-Euler
 * steps of tau = T/nsteps.  MLMC level l uses 32*2^l x 16*2^l cells, 48*2^l steps. */
typedef struct {
  int nx, ny, nsteps;
} henry_grid;

/* Solver options.  Defaults (henry_solver_opts_default) in brackets. */
typedef struct {
  int mg_precision;      /* 64: FP64 multigrid; 32: FP32 multigrid preconditioner inside the
                            FP64 BiCGStab/Newton (iterative refinement) [64] */
  int coarse_nx, coarse_ny; /* coarsest multigrid grid, solved directly (coarse_solver) [8, 4] */
  int nu_pre, nu_post;   /* red-black block Gauss-Seidel sweeps [1, 2] */
  double newton_tol;     /* converged when |dc|_inf <= tol and |dp|_inf <= tol*rho0*g*Ly [1e-9] */
  double newton_dc_max;  /* each update is scaled by min(1, dc_max/|dc|_inf) [2.0] */
  int newton_maxit;      /* per time step [200] */
  double krylov_rtol;    /* BiCGStab forcing term of the Newton systems: |r|_2 <= rtol |r0|_2 per
                            sample, tested after each half step [5e-2]; Newton's own stopping
                            test fixes the accuracy */
  int krylov_maxit;      /* [60] */
  double c_range_tol;    /* status 4 when c leaves [-tol, 1+tol] after a step; a flag only, the
                            sample goes on (a negative tol narrows the range) [1e-8] */
  int use_graphs;        /* capture each Krylov iteration in a hipGraph and replay it [0] */
  int red_blocks;        /* target thread blocks of the per-sample reduction kernels [4096] */
  double krylov_rtol_adjoint; /* BiCGStab tolerance of the transposed (adjoint) systems [1e-8] */
  int newton_extrapolate;     /* first Newton guess of a step, from the states of the last steps
                                 (fewer available on the first steps: lower order).
                                 0: u^n.  1: 2u^n - u^{n-1}.  2: as 1.  3: quadratic
                                 3u^n - 3u^{n-1} + u^{n-2}.  4: cubic 4u^n - 6u^{n-1} +
                                 4u^{n-2} - u^{n-3}.  2..4 under a periodic recharge
                                 (recharge_omega != 0): p^n + g (p^n - p^{n-1}) with g the
                                 ratio of the next to the last change of the inflow factor
                                 (bounded to [-3, 3]) and c^n [4] */
  double newton_predict;      /* > 0: a sample is also converged, without another linear solve, when
                                 its predicted update |dc_{k-1}| |R_k| / |R_{k-1}| (after an undamped
                                 update) is <= newton_predict * newton_tol; 0 disables [1] */
  double newton_jac_reuse;    /* > 0: after a Newton update whose size (as for newton_tol) is
                                 <= newton_jac_reuse for every sample still iterating, the next
                                 iteration keeps the Jacobian, the multigrid hierarchy and the
                                 coarse factors (a chord step; only R is reassembled).  The first
                                 iteration of each step always assembles.  0 disables [1e-3] */
  int mg_cycle;               /* 1: V-cycle; 2: W-cycle (two coarse cycles per level above the
                                 coarsest) [1] */
  int adjoint_guess;          /* first guess of each transposed solve of the reverse sweep.
                                 0: lambda = 0.  1: lambda^{n+1} of the step solved before.
                                 2: 2 lambda^{n+1} - lambda^{n+2}.  The tolerance
                                 krylov_rtol_adjoint stays relative to the right-hand side [2] */
  int coarse_solver;          /* direct solver of the coarsest grid (Gaussian elimination, section 2.3).
                                 0: block-banded LU without pivoting (cells ordered j fastest, block
                                 bandwidth coarse ny), one wavefront per sample [0].  1: dense LU with
                                 partial pivoting of the 2*cells x 2*cells matrix, one workgroup per
                                 sample, trailing updates on the matrix cores; needs 2*cells divisible
                                 by 16 and its 16-column panel in LDS (32x16 cells at most in FP64).
                                 2: the same elimination with partial pivoting in band storage (cells
                                 ordered i-major: kl = ku = 2 coarse_ny + 1 scalar diagonals; the
                                 dense LU's pivots and factors without its work on the zeros outside
                                 the band), one workgroup per sample; needs coarse_ny <= 19 */
  int step_graphs;            /* 1: once a step's kernel arguments are settled (constant inflow, full
                                 extrapolation history), its first Newton iteration -- the step's
                                 start, assembly, one BiCGStab iteration with both halves and the
                                 damped update, every decision taken per sample on the device -- is
                                 replayed from one captured hipGraph, followed by one host read; only
                                 samples that still iterate continue as usual.  Changes the iteration
                                 path, not the discrete solution [1] */
  int ragged_threads;         /* ragged calls with several grids: 0: one host thread (and stream) per
                                 grid, run concurrently [0]; 1: the grids one after another from the
                                 calling thread (for tools that cannot follow several threads) */
  int sample_block;           /* threads per thread-block row (the kernels' tile): 0: min(S, 64), a
                                 wavefront reads 64 samples of one cell [0]; 16 or 32: a wavefront
                                 covers 4 or 2 neighbouring cells of 16 or 32 samples.  The
                                 multigrid's smoother, restriction and prolongation take 2 (FP64)
                                 or 4 (FP32) adjacent samples per thread when S is a multiple of
                                 that width, at least 64 times it, and a row of this many threads
                                 (or a half or quarter of it) leaves no more samples idle */
  int fuse_prolong;           /* 1: the coarse-grid correction is prolonged inside the first
                                 post-smoothing pass and never stored [1]; 0: a separate prolongation
                                 and correction of every cell, then plain passes */
  double krylov_breakdown;    /* near-breakdown guard of BiCGStab: a sample stops with status 2 when
                                 |(r-hat, A M^-1 p)| <= krylov_breakdown * |rho|, i.e. when the step
                                 length |alpha| would reach 1 / krylov_breakdown; the exact zeros
                                 (rho, omega or (r-hat, A M^-1 p) vanishing, or a non-finite value)
                                 stop it whatever the value.  >= 0 [0] */
} henry_solver_opts;

/* One batch of S independent samples on one grid (ragged batches: several per call). */
typedef struct {
  henry_grid grid;
  int nsamples;
  const double* theta;   /* device [S][13] */
  double* c_T;           /* device [ny][nx][S] concentration at t = T, or NULL */
  double* p_T;           /* device [ny][nx][S] pressure at t = T, or NULL */
  double* qoi;           /* device [S] salt mass in x > qoi_xmin at t = T: sum c rho(c) h^2 over the
                            cells whose centre lies there (section 5, eq. integral_s), or NULL */
  int* status;           /* device [S] henry_sample_status, or NULL */
  double* stats;         /* device [S][4]: Newton iterations, BiCGStab iterations (summed over the
                            run), max relative fluid and salt mass-balance defect; or NULL */
  double* series;        /* device [nsteps][HENRY_NSERIES][S] or NULL: after every step the
                            time-resolved QoIs of section 5, integrating the cell-wise constant c
                            exactly: [0] Q_S = sum c rho(c) |cell| (eq. integral_s, kg/m);
                            [1] Q_FW = area with c <= 0.012178 (eq. integral_fw, m^2);
                            [2 + b] salt mass sum c rho(c) |cell n Delta_b| in the square Delta_b
                            of half-width 0.1 around point b of eq. 12points (eq. integral_box):
                            x = 0.90, 1.15, 1.40, 1.65, 1.90 for b % 5, y = -0.95, -0.75, -0.50
                            for b / 5 */
} henry_batch;

#define HENRY_NSERIES 17

HENRY_API void henry_problem_default(henry_problem* p);
HENRY_API void henry_solver_opts_default(henry_solver_opts* o);

/* Create a context on HIP device `device` whose work is issued on `stream`
 * (a hipStream_t; NULL = the default stream).  Returns HENRY_OK or an error. */
HENRY_API int henry_ctx_create(henry_ctx** ctx, int device, void* stream);
HENRY_API void henry_ctx_destroy(henry_ctx* ctx);
/* Message of the last hard error on this context ("" if none).  Owned by ctx. */
HENRY_API const char* henry_last_error(const henry_ctx* ctx);

/* Random input fields at cell centres (paper section 4: the fields are evaluated at
 * the integration points of each grid, not interpolated from rasters).
 * KL eigenpairs of the separable exponential covariance with correlation length
 * corr_len on [0,Lx]x[-Ly,0], modes sorted by eigenvalue.
 *   theta: device [S][13]; phi, K: device [ny][nx][S]; q_in: device [S] (u_in).
 * Any output may be NULL. */
HENRY_API int henry_sample_fields(henry_ctx* ctx, const henry_problem* prob, henry_grid grid, int S,
                        const double* theta, double* phi, double* K, double* q_in);

/* Solve every batch over its full time horizon: c(0) = 0, implicit Euler, Newton with
 * multigrid-preconditioned BiCGStab (section 2.3).  Batches may differ in grid and
 * sample count (ragged MLMC levels); they are solved concurrently.  With the environment
 * variable HENRY_PROGRESS=k set, every k-th time step is reported on stderr.
 * Returns 0, a hard error, or the total number of samples with non-zero status. */
HENRY_API int henry_solve_batch(henry_ctx* ctx, const henry_problem* prob, const henry_solver_opts* opts,
                      henry_batch* batches, int nbatches);

/* Discrete adjoint of the converged time-stepped solve: dQ/dtheta for
 * Q = salt mass in x > qoi_xmin at t = T.  KL fields (field_model 0): xi_1..4, eta_1..8 and
 * zeta; the paper's model (field_model 1, section 4): xi_1 = theta[0] and xi_2 = theta[1]
 * through the porosity and the Kozeny-Carman permeability, the other KL slots 0; theta[12]
 * through the inflow, each step's sensitivity weighted by its recharge factor
 * 1 + sin(recharge_omega t) at the end of the step.  Reverse sweep of transposed, multigrid-
 * preconditioned BiCGStab solves, states recomputed from checkpoints taken every
 * `checkpoint_every` steps.
 *   theta: device [S][13]; qoi: device [S] or NULL; dqoi_dtheta: device [S][13];
 *   status: device [S] or NULL. */
HENRY_API int henry_adjoint_batch(henry_ctx* ctx, const henry_problem* prob, const henry_solver_opts* opts,
                        henry_grid grid, int S, const double* theta, int checkpoint_every,
                        double* qoi, double* dqoi_dtheta, int* status);

/* MLMC estimator over levels 0..L (section 3, eqs. A, goal_variance, MSE):
 *   Y_l = g_fine[l] - g_coarse[l] sample by sample (g_coarse[0] = NULL, i.e. g_{-1} = 0);
 *   mean = sum_l mean(Y_l); V_l = unbiased sample variance of Y_l;
 *   var_of_estimator = sum_l V_l/m_l; bias = |mean(Y_L)|/(2^alpha - 1) (0 when L = 0);
 *   rmse = sqrt(var_of_estimator + bias^2).
 * Field moments (optional: c_fine may be NULL) on the finest grid, coarse fields
 * injected piecewise-constantly into 2x2 children:
 *   mean_field = sum_l I_{l->L}[mean(c_fine[l]) - I mean(c_coarse[l])]
 *   var_field  = sum_l I_{l->L}[S2(c_fine[l]) - I S2(c_coarse[l])]   (S2 unbiased)
 * All sums run on the device in FP64 in a fixed order.
 *   m, grids: host [L+1]; g_fine, g_coarse, c_fine, c_coarse: host arrays of device
 *   pointers (QoIs [m_l]; fields [ny_l][nx_l][m_l] with coarse fields on grid l-1);
 *   mean, var_of_estimator, rmse, V_l (host [L+1]) may be NULL;
 *   mean_field, var_field: device [ny_L][nx_L] or NULL. */
HENRY_API int mlmc_estimate(henry_ctx* ctx, int L, const int* m, const henry_grid* grids,
                  const double* const* g_fine, const double* const* g_coarse,
                  const double* const* c_fine, const double* const* c_coarse, double alpha,
                  double* mean, double* var_of_estimator, double* rmse, double* V_l,
                  double* mean_field, double* var_field);

/* Allocation-free variant of mlmc_estimate, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, outputs, kernels and summation order as mlmc_estimate (results are
 * bitwise equal).  Its workspace -- 2 (L+1) doubles of level moments plus, with fields,
 * sum_l 2 (n_l + n_{l-1}) doubles of cell moments (n_l = nx_l ny_l cells, n_{-1} = 0) -- lives
 * in a file-scope device array of HENRY_NOALLOC_SCRATCH_DOUBLES doubles (8 MiB) that each
 * device holds until the process ends; its address is recorded when a context is created on
 * that device.  A larger workspace is refused with HENRY_EINVAL before any work is enqueued
 * (levels 0..4 of 32x16 .. 512x256 cells need 436 234 doubles).  The call allocates no device
 * or host memory; like mlmc_estimate it synchronises the context's stream to return the host
 * scalars.  All calls on one device share the array: calls that overlap on one device (other
 * contexts or threads) race and must be serialised by the caller. */
#define HENRY_NOALLOC_SCRATCH_DOUBLES (1 << 20)
HENRY_API int mlmc_estimate_noalloc(henry_ctx* ctx, int L, const int* m, const henry_grid* grids,
                                    const double* const* g_fine, const double* const* g_coarse,
                                    const double* const* c_fine, const double* const* c_coarse, double alpha,
                                    double* mean, double* var_of_estimator, double* rmse, double* V_l,
                                    double* mean_field, double* var_field);

/* MLMC estimate of time-resolved QoIs (section 3 applied at every time point, eq. A) at
 * the common times t_k = (k + 1) T / r_0, k < r_0 = grids[0].nsteps, where level l's entry is
 * its step (k + 1) r_l / r_0 - 1 (every r_l a multiple of r_0) and its coarse partner's the
 * step (k + 1) r_{l-1} / r_0 - 1 of the partner's own series:
 *   Y_l = s_fine[l] - s_coarse[l] per sample (s_coarse[0] = NULL, i.e. g_{-1} = 0);
 *   mean = sum_l mean(Y_l), var_of_estimator = sum_l V_l / m_l, V_l unbiased.
 *   m, grids, s_fine, s_coarse: host [L+1]; s_fine[l]: device [r_l][nq][m_l] (the layout of
 *   henry_batch.series with nq = HENRY_NSERIES), s_coarse[l]: device [r_{l-1}][nq][m_l];
 *   mean, var_of_estimator: device [r_0][nq] or NULL; Ymean_l, V_l: device [L+1][r_0][nq]
 *   or NULL.  A scalar QoI is the case r_l = 1, nq = 1. */
HENRY_API int mlmc_estimate_series(henry_ctx* ctx, int L, const int* m, const henry_grid* grids, int nq,
                         const double* const* s_fine, const double* const* s_coarse, double* mean,
                         double* var_of_estimator, double* Ymean_l, double* V_l);

/* Adaptive MLMC plan (section 3: eqs. num_levels and scaled_m_l_S, here with refinement
 * factor 2 per level) from pilot statistics on levels 0..Lp (Lp >= 2, host arrays):
 * |mean Y_l| (Ymean_abs), V_l and the cost per sample s_l.  Least-squares fits in log2 give
 * |E Y_l| = c1 2^(-alpha l) and V_l = c2 2^(-beta l) over l = 1..Lp and s_l = c3 2^(gamma l)
 * over l = 0..Lp.  L is the smallest level in [1, max_level] whose bias estimate
 * c1 2^(-alpha L) / (2^alpha - 1) is <= eps E0 / sqrt(2) (max_level if none), and
 * m_l = ceil(2 eps^-2 E0^-2 sqrt(V_l/s_l) sum_i sqrt(V_i s_i)) for l <= L, with the pilot V_l
 * and s_l up to Lp and the fitted models beyond; eps is relative to E0 = |E g_0|.
 * m_l: host [max_level + 1]; cost: host, model cost sum m_l s_l (may be NULL);
 * rates: host [7] = alpha, beta, gamma, c1, c2, c3 and the cost of plain Monte Carlo at level
 * L for the same accuracy, 2 eps^-2 E0^-2 s_L V_0 (section 5, Test B4, with the pilot's
 * variance of g_0 for that of g_L) (may be NULL).
 * Returns L, or HENRY_EINVAL (also when the fitted alpha is not positive). */
HENRY_API int mlmc_plan(int Lp, const double* Ymean_abs, const double* V_l, const double* s_l, double eps,
                        double E0, int max_level, long long* m_l, double* cost, double* rates);

/* eq. M_ell and eq. total_cost_MLMC: m_l = ceil(2 eps^-2 sqrt(V_l/s_l) sum_i sqrt(V_i s_i)),
 * cost = sum m_l s_l.  Host arrays; returns HENRY_OK or HENRY_EINVAL. */
HENRY_API int mlmc_optimal_samples(int L, const double* V_l, const double* s_l, double eps,
                         long long* m_l, double* cost);

/* Autotuner for one batch shape (ragged-batching support).  Coordinate descent from *opts:
 * one setting at a time over its candidates -- coarsest grid {8x4, 16x8}, smoother sweeps
 * {1+1, 1+2, 2+2}, sample block (tile) {64, 32, 16}, prolongation fusion {on, off},
 * reduction blocks {4096, 16384}, hipGraphs {off, on} -- keeping the fastest.  Each candidate
 * runs the first implicit-Euler step of the caller's samples untimed and times the second
 * (twice; the second timing counts), so a weaker but cheaper preconditioner is charged for any
 * extra Newton iterations; writes the fastest into *opts (other fields unchanged) and its step
 * time into *best_ms (host, may be NULL).  All candidates converge to the same discrete
 * solution; only speed differs.  theta: device [S][13]. */
HENRY_API int henry_autotune(henry_ctx* ctx, const henry_problem* prob, henry_solver_opts* opts, henry_grid grid,
                             int S, const double* theta, double* best_ms);

/* Kernel-level entry points: single launches of the solve's own kernels, for tests and
 * diagnostics.  Work runs on the context's stream; henry_assemble, henry_jacobian_apply and
 * henry_coarse_solve synchronise it before returning (their workspace is the context's).
 *
 * henry_assemble: the residual and analytic Jacobian of the implicit-Euler step `step`
 * (0-based; the step ends at t = (step + 1) T / nsteps, where the recharge factor is taken) at
 * the state (p, c), previous state c_old, fields from theta (section 2.1 balance laws,
 * eqs. e_cont_eq, e_tran_eq, e_Darcy_vel, e_lin_density, e_mol_diff with the boundary
 * conditions of section 2.1; finite volumes and implicit Euler of section 2.3).
 *   theta: device [S][13]; p, c, c_old: device [ny][nx][S];
 *   R: device [2][ny][nx][S] (fluid, salt mass residual, kg/m per step as the solve uses it);
 *   J: device [20][ny][nx][S]: 2x2 blocks d R^a_P / d u^b_Q stored at [blk*4 + a*2 + b] with
 *   blk = 0 centre (Q = P), 1 west, 2 east, 3 south, 4 north neighbour (0 where it does not
 *   exist); a, b = 0 pressure, 1 concentration. */
HENRY_API int henry_assemble(henry_ctx* ctx, const henry_problem* prob, henry_grid grid, int S, const double* theta,
                             const double* p, const double* c, const double* c_old, int step, double* R, double* J);

/* y = J x (transpose = 0) or J^T x (transpose = 1) for the block operator J in the layout of
 * henry_assemble: the Newton systems of section 2.3 and their transposes (discrete adjoint).
 * x, y: device [2][ny][nx][S], distinct. */
HENRY_API int henry_jacobian_apply(henry_ctx* ctx, henry_grid grid, int S, const double* J, const double* x, double* y,
                                   int transpose);

/* One colour of a red-black 2x2-block Gauss-Seidel sweep (the multigrid smoother): for every
 * cell with (i + j) % 2 == colour, x_P = D_P^{-1} (b_P - sum over neighbours A_PQ x_Q), with
 * J^T's blocks when transpose = 1.  J as in henry_assemble; b, x: device [2][ny][nx][S]. */
HENRY_API int henry_gs_pass(henry_ctx* ctx, henry_grid grid, int S, const double* J, const double* b, double* x,
                            int colour, int transpose);

/* Direct solve of a block operator on a coarse grid (Gaussian elimination, section 2.3):
 * x = J^{-1} b (or J^{-T} b) with solver 0 (block-banded LU without pivoting), 1 (dense LU
 * with partial pivoting) or 2 (LU with partial pivoting in band storage), factored and solved
 * in `precision` 64 or 32 (J and b are rounded to
 * FP32 first in the latter).  J: device FP64 [20][ny][nx][S] as in henry_assemble; b, x:
 * device FP64 [2][ny][nx][S].  HENRY_EUNSUPPORTED when the grid does not fit the solver. */
HENRY_API int henry_coarse_solve(henry_ctx* ctx, int solver, int precision, henry_grid coarse, int S, const double* J,
                                 const double* b, double* x, int transpose);

/* The paper's own discretisation (section 2.3): vertex-centred finite volumes on a grid of
 * grid.nx x grid.ny rectangular elements (grid.nsteps implicit-Euler steps over prob->T), with
 * p and c at the (nx + 1)(ny + 1) vertices, each vertex's box made of its quarter-elements,
 * fluxes through the box faces inside each element evaluated at the face midpoints with the
 * bilinear gradients of p and c and the interpolated density (eqs. e_cont_eq, e_tran_eq,
 * e_Darcy_vel, e_lin_density), partial upwind for the convective salt flux (the upwind fraction
 * w = max(0, 1 - 2 D_f / |F|) of each face, D_f = rho phi D_m |face| / h: central where the
 * face Peclet number is at most 2), and the boundary data of section 2.1: Dirichlet
 * p = -rho1 g y, c = 1 at the vertices on x = Lx, Dirichlet c = c_left and the inflow mass flux
 * rho(c_left) u_in on x = 0, closed top and bottom.  phi and K are constant per element (the
 * fields of henry_sample_fields at element centres).  Vectors are [ny+1][nx+1][S]; vertex
 * (i, j) sits at x = i Lx/nx, y = -Ly + j Ly/ny.  Any element aspect ratio is allowed.
 *
 * henry_vc_solve: the whole run per sample from c = 0 (c = 1 on x = Lx), damped Newton as in
 * henry_solve_batch (newton_tol, newton_dc_max, newton_maxit, the first guess by
 * newton_extrapolate, the predictive stop by newton_predict), each Newton system solved by right-preconditioned BiCGStab (krylov_rtol,
 * krylov_maxit).  The preconditioner is a geometric multigrid V-cycle (section 2.3) on vertex
 * grids halved while both element counts are even and at least coarse_nx x coarse_ny:
 * nu_pre forward and nu_post backward four-colour block Gauss-Seidel sweeps, full-weighting
 * restriction and bilinear prolongation, operators rediscretised at the injected state, and
 * Gaussian elimination with partial pivoting on the coarsest grid (at most 70 vertices; its
 * factors are refreshed at the first Newton iteration of each step).  A grid that does not
 * coarsen that far uses nu_pre + nu_post symmetric sweeps instead.
 *   theta: device [S][13]; c_T, p_T: device [ny+1][nx+1][S] or NULL; qoi: device [S] salt mass
 *   sum c rho(c) |box n {x > qoi_xmin}| or NULL; status: device [S] (1 Newton, 2 Krylov
 *   breakdown, 3 non-finite) or NULL; stats: device [S][2] Newton and BiCGStab iterations or NULL.
 *   Returns the number of samples with a non-zero status, or a negative error.
 * henry_vc_solve_batch: several batches (grids and sample counts may differ: the levels and
 *   coarse partners of an MLMC estimate over Table 2's hierarchy) in one call, each on its own
 *   library stream from its own host thread (one after another with ragged_threads = 1), all
 *   ordered after the context's stream and finished on return.  Each henry_batch holds the
 *   outputs of henry_vc_solve with its shapes (c_T, p_T [ny+1][nx+1][S], stats [S][2]); series
 *   must be NULL.  Returns the total number of samples with a non-zero status, or the first
 *   batch's error.
 * henry_vc_assemble: residual R [2][ny+1][nx+1][S] and Jacobian J [36][ny+1][nx+1][S] of step
 *   `step` at (p, c) with previous state c_old; J holds the 2x2 blocks d R^a_v / d u^k_q for the
 *   3 x 3 vertices q = v + (di, dj) around v at [((dj+1) * 3 + di+1) * 4 + a * 2 + k] (0 where q
 *   does not exist).  A Dirichlet unknown's row is u - u_D.  Synchronises the stream. */
HENRY_API int henry_vc_solve(henry_ctx* ctx, const henry_problem* prob, const henry_solver_opts* opts, henry_grid grid,
                             int S, const double* theta, double* c_T, double* p_T, double* qoi, int* status,
                             double* stats);
HENRY_API int henry_vc_solve_batch(henry_ctx* ctx, const henry_problem* prob, const henry_solver_opts* opts,
                                   henry_batch* batches, int nbatches);
HENRY_API int henry_vc_assemble(henry_ctx* ctx, const henry_problem* prob, henry_grid grid, int S, const double* theta,
                                const double* p, const double* c, const double* c_old, int step, double* R, double* J);

/* Kernel-class timing on the context's stream (instrumentation for benchmarks).
 * henry_profile(ctx, 1) resets the counters and brackets every later launch of the
 * classes below with HIP events (launches on whole batches only: the compacted
 * sub-batches that finish a time step's last Newton iterations are not timed);
 * henry_profile(ctx, 0) stops.  henry_profile_read()
 * returns, for one class: launches, units processed (cell-samples; for the smoother,
 * cells of the swept colour x samples) and the summed event time in ms.  Both calls
 * synchronise the stream. */
enum henry_prof_class {
  HENRY_PROF_ASSEMBLE = 0,    /* fine-grid residual + Jacobian assembly (henry_vc_solve: its
                                 vertex-centred assembly, units vertex-samples) */
  HENRY_PROF_GS = 1,          /* fine-grid red-black GS passes that read neighbours (henry_vc_solve:
                                 each four-colour pass, units the colour's vertex-samples) */
  HENRY_PROF_SPMV = 2,        /* fine-grid FP64 block SpMV with fused dots (henry_vc_solve: the
                                 nine-point SpMV, units vertex-samples) */
  HENRY_PROF_RESTRICT = 3,    /* fine-grid fused residual + restriction */
  HENRY_PROF_PROLONG = 4,     /* prolongation + correction onto the fine grid */
  HENRY_PROF_BAND_FACTOR = 5, /* coarse banded LU factorisation */
  HENRY_PROF_BAND_SOLVE = 6,  /* coarse banded triangular solves */
  HENRY_PROF_DENSE_FACTOR = 7,/* dense coarse LU: the pivoted factorisation (units: samples) */
  HENRY_PROF_DENSE_SOLVE = 8, /* dense coarse triangular solves (units: samples) */
  HENRY_PROF_HOST_SYNC = 9,   /* the solver's host round trips (control reads): launches = their
                                 number, units = 0, total_ms = host time spent waiting in them;
                                 counted whether or not event timing is enabled */
  HENRY_PROF_NCLASS = 10
};
HENRY_API int henry_profile(henry_ctx* ctx, int enable);
HENRY_API int henry_profile_read(henry_ctx* ctx, int cls, long long* launches, long long* units, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* HENRY_H */
