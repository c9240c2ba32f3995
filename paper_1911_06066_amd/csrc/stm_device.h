// Device-side data structures and helpers shared by the kernels of the
// space-time MLMC library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stm {

constexpr int kMaxMG = 8;        // multigrid grids per MLMC level
constexpr int kMaxRestart = 30;  // Krylov dimension limit
constexpr int kWave = 64;
constexpr int kMaxTeam = 32;  // largest team of workgroups per sample

// One structured grid: nodes per axis, elements per axis, spacing.
struct GridDev {
  int nx, ny, nz;
  int n;              // nodes
  int ex, ey, ez;     // elements per axis
  int ne;             // elements
  double hx, hy, hz;
  unsigned mnx, mny, mex, mey;  // division magics (fdiv_magic) of nx, ny, ex, ey
};

// Exact unsigned division by a divisor d >= 2 that is fixed for many
// dividends: with m = ceil(2^32 / d), q / d = floor(q m / 2^32) whenever
// q d <= 2^32 (the rounding excess of m, below d, then moves q m / 2^32 by less
// than 1/d).  Index arithmetic keeps every dividend inside that range (the
// host rejects grids with n * max(nx, ny) >= 2^32).
__host__ __device__ inline unsigned fdiv_magic(unsigned d) {
  return (unsigned)((0x100000000ull + d - 1) / d);
}
__device__ __forceinline__ int fdiv(int q, unsigned m) { return (int)__umulhi((unsigned)q, m); }

// One MLMC level: its grid (index 0) and the coarser grids of its V-cycle.
// Byte offsets locate every array inside a team workspace.
struct LevelDev {
  int dim;
  int m;
  double dt, T;
  int nmg;                      // multigrid grids (>= 1)
  int sweeps;                   // Jacobi sweeps on the coarsest V-cycle grid
  double pc_words;              // words per grid-0 node that one preconditioner application moves
                                // (per-step model: 5 per sweep and per residual, on each grid
                                // weighted by its nodes)
  double cheb_ratio;            // Chebyshev interval ratio of the sweep weights
  GridDev g[kMaxMG];
  const double* fib[kMaxMG];    // fibre table of every grid: per element row (2D) / layer (3D): c^2, s^2, c s
                                // at that grid's own element centroids
  const double* u0;     // initial state at the nodes of grid 0 (filled by the host)
  // team workspace layout (bytes from the team base)
  int64_t off_u, off_uprev, off_wk1, off_tact;          // float64 [n0]
  int64_t off_V, off_Z;                                 // inner [restart+1][n0], [restart][n0]
  int64_t off_kd;                                       // float64 [n0] stiffness diagonal of grid 0
  int64_t off_dlt;                                      // float64 [n0] last Newton step (damping)
  int64_t off_dinv;                                     // inner [n0] inverse diagonal of the slab operator
  int64_t off_mgX[kMaxMG], off_mgT[kMaxMG], off_mgB[kMaxMG], off_mgW[kMaxMG];  // inner [n_l]
  int64_t off_mgI[kMaxMG];                              // inner [n_l] inverse slab diagonal (l >= 1)
  int64_t off_mgS[kMaxMG];                              // float64 [ne_l] conductivity: mean of children (l >= 1)
  int64_t off_mgK[kMaxMG];                              // float64 [n_l] stiffness diagonal (l >= 1)
  int64_t off_mgS32[kMaxMG];                            // float32 [ne_l] conductivity for the float32 3D passes
  int64_t off_U;                                        // float64 [m][n0] in-place warm-start buffer
  // global space-time mode only (0 otherwise): inner space-time vectors of
  // m slabs of stride vs = n0 rounded up to 64
  int64_t off_gV;                                       // [restart+1][m][vs] Krylov basis
  int64_t off_gW, off_gD;                               // [m][vs] reaction weights, inverse slab diagonals
  int64_t off_gZ;                                       // [m][vs] preconditioned vector / Newton step
  int64_t off_gT;                                       // [vs] forward-substitution right-hand side
  int64_t team_bytes;
  // LDS tiles of the stencil passes on every grid: node rows (y) and planes
  // (z) per tile, [grid][8-byte (0) or 4-byte (1) fields][2, 3 or 4 staged
  // nodal fields]
  int tile_y[kMaxMG][2][3], tile_z[kMaxMG][2][3];
  // node rows per tile of the fused two-sweep smoother pass (2D), for 8-byte
  // and 4-byte inner vectors
  int tile_p8, tile_p4;
};

// Physics and solver parameters (uniform across a launch).
struct SolverParams {
  double k_react, a_react;
  double tau;           // constant part of the transverse conductivity (0 when it is relative)
  double zr;            // D_zz = tau + zr sigma_e (3D)
  double threshold;
  double newton_tol;
  double gmres_rtol;
  double smooth_omega;
  int newton_max;
  int restart;
  int smooth_steps;
  int coarse_sweeps;
  int smoother;         // 0: fixed weight omega; 1: Chebyshev-root weights over [lmax/ratio, lmax]
  double cheb_ratio;
  int power_iters;      // power iterations estimating lmax(D^-1 A) per sample and grid
  double theta;         // weight of the new time level in the diffusion term (1: BE, 1/2: CN)
  int damping;          // 1: halve a Newton step while the residual grows; 0: full steps
  int global_st;        // 1: Newton on the whole space-time system with a global GMRES (st_global_kernel)
};

constexpr int kMaxSweeps = 32;

// Fibre table: per element row (2D) or layer (3D) the entries (c2, s2, cs) of
// D_e = (sigma_e c2 + tau s2, sigma_e s2 + tau c2, (sigma_e - tau) cs) in the
// x-y plane; D_zz = tau + zr sigma_e.  The fibre model takes
// (cos^2, sin^2, cos sin), tau = ratio sigma_f0 and zr = 0; a transverse
// conductivity ratio sigma_e takes (cos^2 + ratio sin^2, sin^2 + ratio cos^2,
// (1 - ratio) cos sin), tau = 0 and zr = ratio, which with ratio 1 is sigma_e I.
constexpr int kFibStride = 3;

// A team of G workgroups solves `count` samples s = first + i * stride in
// order.  One TeamTask per workgroup: the members of a team carry identical
// fields except `rank`.  With G > 1 each member owns a band of node rows of
// the level's grid and the members meet at team barriers.
struct TeamTask {
  int level;                 // index into the LevelDev table of the launch
  int first, stride, count;
  const int* order;          // null: sample first + i stride; else sample order[first + i stride]
  const double* sigma;       // [*][ne0]
  double* u_out;             // [*][m][n0] or null (use the team buffer)
  const double* u_guess;     // [*][m][n0] or null
  double* t_act;             // [*][n0] or null
  unsigned char* work;       // team workspace
  struct SampleStatsDev* stats;  // [*] or null
  int rank, G;               // member rank, team size
  unsigned* bar;             // team barrier counter, zero at launch (G > 1)
  double* part;              // team reduction partials [2][G][16] (G > 1)
  int* fault;                // set to 1 when a team barrier wait times out
};

struct SampleStatsDev {
  int status;
  int newton_max_per_slab;
  long long newton_iters;
  long long krylov_iters;
  double final_step;
  long long ticks;           // wall-clock ticks (100 MHz) spent on the sample
  int censored;
  int damped;                // Newton steps halved because the residual grew
  double alg_bytes;          // bytes the sample's passes must move (per-pass model)
  long long phase_ticks[8];  // per-phase wall-clock ticks when built with STM_PHASE_TIMERS, else 0
  double model_bytes;        // bytes by the per-step word model (see stm_solve_stats)
};

// ---------------------------------------------------------------------------
// wave64 / block reductions (deterministic: fixed shuffle tree, fixed wave order)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Sum NV values over the block; every thread receives the totals.
// scratch: shared double[NWAVES * NV].  Contains two barriers.
template <int BLOCK, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* scratch) {
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[wid * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += scratch[w * NV + i];
    v[i] = s;
  }
  __syncthreads();
}

template <int BLOCK>
__device__ __forceinline__ double block_max(double v, double* scratch) {
  constexpr int NW = BLOCK / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  v = wave_max(v);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = scratch[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) s = fmax(s, scratch[w]);
  __syncthreads();
  return s;
}

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

}  // namespace stm
