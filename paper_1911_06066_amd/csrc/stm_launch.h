// Host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "stm_device.h"

namespace stm {

// Fused team solver: one workgroup per task (see st_solver.hip).
// One workgroup per TeamTask; lds_bytes: dynamic LDS of each workgroup
// (staging tiles); cooperative: launch with guaranteed co-residency (needed
// when any team has G > 1).
// mg: some level of the launch has a multigrid hierarchy (nmg > 1).
// prm.global_st selects the global space-time kernel (256 or 512 threads).
hipError_t launch_team_solver(int dim, bool inner_fp32, bool mg, const LevelDev* levels, const TeamTask* tasks,
                              int n_blocks, SolverParams prm, int block, size_t lds_bytes, bool cooperative,
                              hipStream_t st);
// Co-resident solver workgroups per CU for a configuration (0 on error);
// global: the global space-time kernel (SolverParams::global_st).
int team_solver_occupancy(int dim, bool inner_fp32, bool mg, bool global, int block, size_t lds_bytes);

// sigma[s][e] = sigma_f0 * exp(sum_k modes[e][k] xi[s][k]) on the matrix cores.
// split_fp16: operands split into fp16 hi/lo pairs, fp32 accumulation; else float64 MFMA.
// sigma = sigma_f0 exp(g) (lognormal) or sigma_f0 (1 + g) (additive), g = xi modes^T.
hipError_t launch_kl_synthesize(const double* modes, const double* xi, double* sigma, int S, int E, int M,
                                double sigma_f0, bool split_fp16, bool additive, hipStream_t st);

// Space-time prolongation of S coarse solutions u_c[S][mc][gc.n] to u_f[S][mf][gf.n]:
// nested Q1 interpolation in space, linear in time, u0f[gf.n] the fine initial state.
hipError_t launch_prolong_st(const GridDev& gc, const GridDev& gf, int dim, int mc, int mf, const double* u0f,
                             const double* u_c, int S, double* u_f, hipStream_t st);

// Activation map of u[S][m][n] on grid g, with initial state u0[n] (device).
hipError_t launch_activation_map(const GridDev& g, int m, double dt, double T, double thr, const double* u0,
                                 const double* u, int S, double* t_act, int* censored_dev, hipStream_t st);

// MLMC statistics of one level on the finest grid.
struct StatsLevelArgs {
  GridDev gf;            // grid of level l
  GridDev gc;            // grid of level l-1 (unused when tc == null)
  GridDev gL;            // finest grid
  int dim;
  const double* tf;      // [N][gf.n]
  const double* tc;      // [N][gc.n] or null
  int N;
  int chunk;             // samples per Welford chunk
  double* part;          // [n_chunks][6][gL.n] partial states
  double* mean;          // [gL.n] accumulated MLMC mean
  double* var;           // [gL.n] accumulated MLMC variance
  double* level_mean;    // [gL.n] or null
  double* level_var;     // [gL.n] or null
  double* vpart;         // [ceil(P / 256)] partial sums of w_p s^2(Y_l)
  // space-time QoI (mL > 0): tf/tc hold [N][m][g.n] solutions, the points are
  // the finest grid's time levels 1 .. mL, P = mL gL.n; u0f/u0c: the levels'
  // initial states (time level 0)
  int mf, mc, mL;
  double dtL;
  const double* u0f;
  const double* u0c;
};
hipError_t launch_level_stats(const StatsLevelArgs& a, hipStream_t st);
hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t st);
hipError_t launch_fill_u32(unsigned* p, unsigned v, int64_t n, hipStream_t st);
// out[s] = min over the E entries of row s of a[S][E] (device)
hipError_t launch_row_min(const double* a, int S, int E, double* out, hipStream_t st);

}  // namespace stm
