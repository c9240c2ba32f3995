/*
 * stmlmc.h -- C interface of the space-time multilevel Monte Carlo library
 * for the monodomain equation on AMD Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem ("Space-time
 * multilevel Monte Carlo methods and their application to cardiac
 * electrophysiology"): for every value of the random input, solve the
 * nonlinear space-time system C u + r(u) = f (Sec. 3.3, eq. mono_disc) whose
 * conductivity is a truncated Karhunen-Loeve expansion (Sec. 2.2,
 * eq. KL-expansion), and combine the samples with the MC / MLMC estimators of
 * Sec. 3.1.2 (eqs. MC-estimator, MLMC-estimator).
 *
 * Conventions shared by every call
 *  - All bulk arrays are DEVICE pointers on the device that was current at
 *    stm_create; the caller owns them; the library never frees caller memory.
 *    Host pointers are named *_host or documented as host.
 *  - Arrays are dense, row-major, float64 unless stated, with the layouts
 *    given per argument.  Nodes are numbered x fastest, then y, then z;
 *    elements likewise.  A space-time array u[s][k][i] stores time levels
 *    k = 1..m (index k-1); the initial state is not stored.
 *  - Work is enqueued on the stream given at stm_create.  Calls that return
 *    host-side results (stats, counts, scalars) synchronise that stream.
 *  - Every call returns an stm_status; none aborts or exits.  Argument errors
 *    are detected before any work is enqueued (STM_E_INVALID).  HIP runtime
 *    errors return STM_E_DEVICE.  The message of the last error of a context is
 *    available from stm_last_error().
 *  - One context per host thread; calls on one context are not thread safe.
 */
#ifndef STMLMC_H
#define STMLMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STM_OK = 0,
  STM_E_INVALID = -1,        /* bad argument, shape or pointer */
  STM_E_NOMEM = -2,          /* device workspace could not be allocated */
  STM_E_DEVICE = -3,         /* HIP runtime error */
  STM_E_NOT_CONVERGED = -4,  /* a Newton iteration hit its limit; results hold the last iterate */
  STM_E_NONFINITE = -5,      /* NaN/Inf met in an input or a residual */
  STM_E_UNSUPPORTED = -6     /* valid request this build does not handle */
} stm_status;

typedef enum {
  STM_PREC_FP64 = 0,   /* every floating-point step in float64 */
  STM_PREC_MIXED = 1   /* float32 Krylov/multigrid and split-fp16 KL GEMM inside float64 Newton refinement */
} stm_precision;

typedef enum {
  STM_FIBER_DIAG2D = 0,  /* theta = pi/4 + 0.5 y */
  STM_FIBER_ROT3D = 1,   /* theta = -pi/3 + (2 pi/3) z / lz */
  STM_FIBER_X = 2,       /* theta = 0 */
  STM_FIBER_DIAG = 3     /* theta = pi/4 */
} stm_fiber_law;

typedef enum {
  STM_FIELD_LOGNORMAL = 0,  /* sigma = sigma_f0 exp(g) */
  STM_FIELD_ADDITIVE = 1    /* sigma = sigma_f0 (1 + g): the paper's expansion G_0 + s sum sqrt(lambda_k)
                               phi_k y_k (Sec. 2.2, eq. KL-expansion) with G_0 = sigma_f0 and the
                               factor s G_0 folded into the modes; the caller keeps 1 + g > 0 */
} stm_field_kind;

typedef enum {
  STM_QOI_ACTIVATION = 0,  /* the activation-time map on the finest grid, n_L values */
  STM_QOI_SPACETIME = 1    /* the space-time solution u itself on the finest space-time grid, time levels
                              1 .. m_L: m_L n_L values, level k at t = k dt_L (Sec. 4.1: E[u] with
                              the error measured in L^2(0, T; L^2(D))) */
} stm_qoi;

typedef enum {
  STM_IC_BALL = 0,   /* u(x, 0) = 1 in the closed ball |x - ic_center| <= ic_radius, else 0 */
  STM_IC_GAUSS = 1   /* u(x, 0) = exp(-|x - ic_center|^2 / ic_radius^2): the paper's Gaussian
                        stimulus (Sec. 4, "Parameters for the experiments"), in units of u_peak */
} stm_ic_kind;

#define STM_MAX_LEVELS 8

/* One MLMC level: nodes per axis (nz = 1 in 2D; nx >= 3, ny >= 2 in 2D (a strip of one element
 * row with y-constant data is the 1D problem), ny >= 3 and nz >= 2 in 3D) and time steps.
 * smooth_sweeps and cheb_ratio override the problem's coarse_sweeps and
 * cheb_ratio for this level (0 keeps the problem's value); a tuner measures
 * them per level, since the best smoother degree depends on the slab
 * operator's spectrum, i.e. on h and dt. */
typedef struct {
  int nx, ny, nz;
  int m;
  int smooth_sweeps;          /* Jacobi sweeps on the level's coarsest V-cycle grid, 0 .. 32 */
  double cheb_ratio;          /* Chebyshev interval ratio, 0 or > 1 */
  double team_seconds[32];    /* measured device seconds per sample with a team of g+1 workgroups
                                 (0 = unknown); the MLMC scheduler's starting cost model, refined by
                                 the measurements of every launch */
} stm_level;

/*
 * The problem: monodomain equation du/dt = div(D grad u) + f(u) on the box
 * [0,lx] x [0,ly] (x [0,lz]) with homogeneous Neumann boundaries, the theta
 * scheme in time on [0,T] (backward Euler or the paper's Crank-Nicolson, see
 * theta), Q1 elements in space (Sec. 2.1, Sec. 3.2).
 *   f(u) = k_react u (u - a_react)(1 - u)       (FitzHugh-Nagumo cubic, eq. ionic_term)
 *   D_e  = sigma_e a a^T + tau_e (I - a a^T),
 *          tau_e = transverse_ratio sigma_f0 (tau_relative = 0) or transverse_ratio sigma_e (= 1;
 *          with transverse_ratio 1 the isotropic scalar field sigma_e I of Sec. 2.1)
 *   a    = (cos theta, sin theta[, 0]), theta from fiber_law at the element centroid
 *   u(x, 0) from ic_kind (stm_ic_kind)
 * The activation map is the first time u reaches `threshold`.
 */
typedef struct {
  int dim;                    /* 2 or 3 */
  double lx, ly, lz;
  double T;
  double k_react, a_react;
  double sigma_f0, transverse_ratio;
  int fiber_law;              /* stm_fiber_law */
  double ic_center[3], ic_radius;
  double threshold;
  int n_levels;               /* 1 .. STM_MAX_LEVELS, coarse to fine, each axis refined 2:1 or kept */
  stm_level levels[STM_MAX_LEVELS];
  int n_modes;                /* KL modes M, 1 .. 256 */
  int precision;              /* stm_precision */
  /* solver controls; 0 selects the default */
  double newton_tol;          /* max-norm Newton step per slab (u is O(1)): 1e-10; a slab stops when its
                                 step or the step predicted from the observed contraction is below it */
  int newton_max;             /* Newton iterations per slab: 30 */
  double gmres_rtol;          /* relative Krylov residual: 1e-10 (fp64), 1e-5 (mixed) */
  int gmres_restart;          /* Krylov dimension of one linear solve: 16, at most 30; an unfinished
                                 solve is continued by the next Newton step */
  int mg_levels;              /* grids of the geometric-multigrid V-cycle that preconditions each slab's
                                 GMRES: 1 (default; Chebyshev-weighted sweeps on the level's grid only),
                                 2 .. 8, or -1 (as deep as the grid allows).  Coarsening halves every axis
                                 while all stay odd with >= 5 nodes in x, y (>= 3 in z).  Coarse operators
                                 are rediscretised: element conductivity the mean of its children, the
                                 coarse grid's own fibre angles, reaction weights injected from the level's
                                 grid.  Restriction is full weighting (the transpose of Q1 interpolation).
                                 A level with coarse grids is solved by one-workgroup teams */
  int smooth_steps;           /* weighted-Jacobi sweeps before and after the coarse correction: 2 */
  double smooth_omega;        /* fixed Jacobi weight (smoother 0): 0.7 */
  int coarse_sweeps;          /* weighted-Jacobi sweeps on the coarsest grid (the only grid when
                                 mg_levels = 1): 8, at most 32 */
  int smoother;               /* 0 (default): sweep weights 1/xi_s, xi_s the Chebyshev roots on
                                 [lmax/cheb_ratio, lmax] of D^-1 A, lmax by power iteration;
                                 1: the fixed weight smooth_omega */
  double cheb_ratio;          /* 10 (2D), 30 (3D) */
  int lds_kb;                 /* LDS staging budget per workgroup in KiB: 144 */
  int block_threads;          /* threads per workgroup: chosen from the grid size */
  int max_lanes;              /* workgroups per solver launch: 1024 (capped by co-residency) */
  int team_size;              /* workgroups per sample in stm_st_solve: 0 = chosen from S and the
                                 device; >1 only with mg_levels = 1 */
  double theta;               /* weight of the new time level in the diffusion term, in [1/2, 1]:
                                 1 (default; 0 selects it) backward Euler, 1/2 the paper's
                                 Crank-Nicolson (Sec. 3.2, eq. st-system: A = M + dt/2 K,
                                 B = -M + dt/2 K); the reaction is always taken at the new level
                                 (Sec. 3.3, eq. mono_disc).  Slab k solves
                                 M (u_k - u_{k-1})/dt + K (theta u_k + (1-theta) u_{k-1}) - M f(u_k) = 0 */
  int field_kind;             /* stm_field_kind of stm_kl_synthesize and stm_mlmc_estimate: 0 lognormal */
  int tau_relative;           /* 0: tau_e = transverse_ratio sigma_f0; 1: tau_e = transverse_ratio sigma_e */
  int ic_kind;                /* stm_ic_kind: 0 ball */
  int qoi;                    /* stm_qoi of stm_mlmc_estimate: 0 activation map */
  int newton_damping;         /* 0 (default) or 1: a slab's Newton step is halved (down to 1/64 of it)
                                 while the FP64 residual 2-norm it leads to exceeds the last accepted
                                 one; -1: full Newton steps */
  int st_mode;                /* 0 (default): Newton slab by slab in time order (exact block forward
                                 substitution of the space-time system, Sec. 3.2 eq. system_C);
                                 1: Newton on the whole space-time system, each linear step one GMRES
                                 over all m slabs right-preconditioned by forward substitution with
                                 the slab preconditioner (Sec. 3.2, Sec. 3.5: the paper's monolithic,
                                 parallel-in-time solve).  Mode 1 needs (restart + 4) m n inner
                                 words of workspace per concurrent sample and 256 or 512 threads
                                 per workgroup */
} stm_problem;

/* Per-sample solver statistics (host array filled by stm_st_solve). */
typedef struct {
  int status;                 /* stm_status of this sample */
  int newton_max_per_slab;    /* largest Newton count of any time slab */
  int64_t newton_iters;       /* Newton iterations summed over slabs */
  int64_t krylov_iters;       /* Krylov iterations summed over all linear solves */
  double final_step;          /* largest final max-norm Newton step over slabs */
  double device_seconds;      /* wall time of this sample on its workgroup(s) */
  double algorithmic_bytes;   /* bytes the solve's passes must move: each array a pass reads or
                                 writes counted once per pass (cache re-reads not counted) */
  double phase_seconds[8];    /* per-phase device time (residual, smoothing, Arnoldi stencil, dots,
                                 orthogonalisation, update, -, -) in libraries built with phase
                                 timers; zero otherwise */
  double model_bytes;         /* bytes of the solve by per-node word counts of the method's steps,
                                 n nodes: 4 float64 words per Newton residual; per Krylov iteration j
                                 (0-based within its linear solve) 4 words for the Jacobian product,
                                 5 per smoother sweep (on every V-cycle grid, weighted by its nodes)
                                 and 2j + 3 for the Arnoldi step, in the inner precision.  Passes the
                                 kernel fuses are counted as the separate steps they replace */
  int64_t damped_steps;       /* Newton steps halved because the residual 2-norm grew (each halving
                                 costs one residual evaluation, counted in newton_iters) */
} stm_solve_stats;

/* Device time of the last call's phases, measured with HIP events on the context stream. */
typedef struct {
  double kl_ms;               /* KL synthesis launches */
  double solve_ms;            /* team-solver launches */
  double stats_ms;            /* activation / MLMC statistics launches */
  double solve_bytes;         /* algorithmic bytes of the solver launches (sum over samples) */
  int solve_launches;
  int solve_teams;            /* teams (samples in flight) of the last solver launch */
  int solve_blocks;           /* workgroups of the last solver launch */
  int solve_block;            /* threads per workgroup of the last solver launch */
  double solve_bytes_model;   /* bytes of the solver launches by the per-step word model (model_bytes) */
} stm_timings;

/* Output of stm_mlmc_estimate. Device arrays are caller-owned, n_L = nodes of the finest level. */
typedef struct {
  /* P: the QoI's points, n_L (STM_QOI_ACTIVATION) or m_L n_L (STM_QOI_SPACETIME, row-major
     [k][i] for time levels k = 1 .. m_L) */
  double* mean;               /* device [P]: MLMC mean of the QoI */
  double* var;                /* device [P]: sum_l s^2(P Q_l) - s^2(P Q_{l-1}) */
  double* level_mean;         /* device [(L+1) P] or NULL: mean of Y_l = P Q_l - P Q_{l-1} */
  double* level_var;          /* device [(L+1) P] or NULL: unbiased variance of Y_l */
  /* host-side outputs */
  int N[STM_MAX_LEVELS];      /* samples used per level */
  double V[STM_MAX_LEVELS];   /* |D|^-1 int s^2(Y_l) (lumped quadrature on the finest grid); for the
                                 space-time QoI (|D| T)^-1 int int s^2(Y_l), trapezoid in time with
                                 the deterministic t = 0 level contributing nothing */
  double cost[STM_MAX_LEVELS];/* workgroup-seconds per sample pair of the level (measured) */
  double bias_estimate;       /* |D|^-1/2 || mean(Y_L) ||_2 / (2^alpha - 1), alpha fitted (0 if L < 2) */
  int64_t newton_iters;       /* over all samples */
  int64_t krylov_iters;
  int64_t censored;           /* nodes never activated, over all solved samples */
  int rounds;                 /* allocation rounds (1 for fixed counts) */
  int worst_status;
  double algorithmic_bytes;   /* over all solves, as in stm_solve_stats */
  int64_t dof_steps;          /* sum over solves of nodes x time steps (both pair members) */
  double model_bytes;         /* over all solves, by the per-step word model of stm_solve_stats */
} stm_mlmc_result;

typedef struct stm_ctx stm_ctx;

/*
 * Create a context for problem *p on the current HIP device.  hip_stream is a
 * hipStream_t (NULL = default stream).  Validates the problem, builds the
 * geometric-multigrid hierarchies of every level and the fibre tables.
 * On error *out is NULL and the status says why.
 */
stm_status stm_create(const stm_problem* p, void* hip_stream, stm_ctx** out);

/* Release the context and its device workspace (synchronises its stream). */
void stm_destroy(stm_ctx* ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next call. */
const char* stm_last_error(const stm_ctx* ctx);

/* Phase timings of the last kl/solve/activation/mlmc call on ctx (host output). */
stm_status stm_get_timings(const stm_ctx* ctx, stm_timings* out);

/* Nodes, elements and time steps of a level (host outputs, any may be NULL). */
stm_status stm_level_size(const stm_ctx* ctx, int level, int* n_nodes, int* n_elements, int* m);

/*
 * KL synthesis (Sec. 2.2, eq. KL-expansion), with g[s][e] = sum_k modes[e][k] * xi[s][k]:
 *   sigma[s][e] = sigma_f0 * exp(g[s][e])      (field_kind STM_FIELD_LOGNORMAL)
 *   sigma[s][e] = sigma_f0 * (1 + g[s][e])     (field_kind STM_FIELD_ADDITIVE),
 * modes[E][M] (the eigenfunctions at the element centroids of `level`, each
 * column pre-scaled by sqrt(lambda_k), and by the damping s for the additive
 * field), xi[S][M], sigma[S][E]; E is the element count of the level and
 * M = n_modes.  Computed as one matrix product on the matrix cores: float64
 * operands (STM_PREC_FP64) or split-fp16 operands with float32 accumulation
 * (STM_PREC_MIXED; relative error of g about 1e-7).  S >= 0 (S = 0 is a no-op).
 */
stm_status stm_kl_synthesize(stm_ctx* ctx, int level, const double* modes, const double* xi,
                             int S, double* sigma);

/*
 * Space-time solve of S samples on `level` (Sec. 3.3, eq. mono_disc, by
 * Newton's method, Sec. 3.5): for each s, u[s] solves
 *   M (u_k - u_{k-1}) / dt + K(sigma[s]) u_k - M f(u_k) = 0,  k = 1..m,
 * with u_0 the initial state.  sigma[S][E] element conductivities,
 * u[S][m][n] output.  u0_guess[S][m][n] (or NULL) is the initial Newton
 * iterate; with NULL each workgroup lane starts from the solution of the
 * previous sample it solved (the first from the initial state).
 * stats_host[S] (or NULL) receives per-sample statistics and makes the call
 * synchronous.  Returns the worst per-sample status.
 */
stm_status stm_st_solve(stm_ctx* ctx, int level, const double* sigma, const double* u0_guess,
                        int S, double* u, stm_solve_stats* stats_host);

/*
 * stm_st_solve without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors as
 * stm_st_solve.  Every device area the call needs beyond the caller's arrays
 * (team synchronisation, the launch's task table, per-sample statistics, the
 * team workspaces) lives in one fixed array of 64 MiB per device, held from
 * the first stm_create on that device until the process ends; the call takes
 * fewer concurrent lanes when the workspaces of all would not fit, and
 * returns STM_E_INVALID, before any work is enqueued, when the statistics of
 * S samples and one lane's workspace exceed it.  The array is shared by every
 * call on the device and keeps the last call's contents (the call clears what
 * must start at zero): calls that overlap on one device, from any context or
 * stream, race.
 */
stm_status stm_st_solve_noalloc(stm_ctx* ctx, int level, const double* sigma, const double* u0_guess,
                                int S, double* u, stm_solve_stats* stats_host);

/*
 * Activation map of S space-time solutions u[S][m][n] on `level`:
 * t_act[s][i] = 0 if u_0 >= threshold, else the first up-crossing of the
 * threshold, linear in t between the bracketing time levels, else T
 * (censored).  n_censored_host[S] (or NULL) receives the censored counts
 * and makes the call synchronous.
 */
stm_status stm_activation_map(stm_ctx* ctx, int level, const double* u, int S, double* t_act,
                              int* n_censored_host);

/*
 * Space-time prolongation P_t (x) P_h from level-1 to `level` (Sec. 3.4, the
 * tensor-product transfer P_l = P_{l,t} (x) P_{l,h} between space-time
 * levels), for a coarse solution to serve as the fine solve's first iterate
 * (stm_st_solve's u0_guess).  In space: Q1 interpolation of the nested coarse
 * grid at the fine nodes.  In time: fine level k at t = k dt_l lies at
 * j + w = k m_{l-1} / m_l coarse steps; the value is (1 - w) U_j + w U_{j+1}
 * of the space-interpolated coarse levels, with U_0 the fine grid's initial
 * state (the coarse initial state is not an unknown).
 *   u_coarse[S][m_{l-1}][n_{l-1}], u_fine[S][m_l][n_l], device, caller-owned;
 *   1 <= level < n_levels, S >= 0 (S = 0 is a no-op).  Asynchronous on the
 *   context stream.
 */
stm_status stm_prolong_st(stm_ctx* ctx, int level, const double* u_coarse, int S, double* u_fine);

/*
 * MLMC estimate of the mean and variance of the activation map on the
 * finest level (Sec. 3.1.2, eq. MLMC-estimator; single level = plain MC).
 *   modes_host[l] : device pointer to modes of level l, [E_l][M]
 *   xi_host[l]    : device pointer to [capacity_host[l]][M] KL coefficients
 *                   of level l's sample pairs; pair i uses row i for both
 *                   its fine (level l) and coarse (level l-1) member
 *   N_host        : samples per level, or NULL for adaptive counts: pilot
 *                   rounds of `pilot` samples, then N_l from the estimated
 *                   V_l and cost per sample until the variance part of the
 *                   mean-square error is below target_rmse^2 / 2, capped by
 *                   capacity_host[l].
 * With qoi = STM_QOI_ACTIVATION the solutions stay in workspace and only
 * activation maps are kept; with STM_QOI_SPACETIME every solution is kept
 * (capacity x m_l x n_l float64 per pair member) and its space-time
 * prolongation to the finest space-time grid (nested Q1 in space, linear in
 * time from the level's own initial state, Sec. 3.4) is the sample.  Either
 * way the samples are reduced by Welford per chunk of samples, merged in
 * sample order.  Synchronous.
 */
stm_status stm_mlmc_estimate(stm_ctx* ctx, const int* N_host, const double* const* modes_host,
                             const double* const* xi_host, const int* capacity_host,
                             double target_rmse, int pilot, stm_mlmc_result* out);

#ifdef __cplusplus
}
#endif

#endif /* STMLMC_H */
