// C interface of the library (include/stmlmc.h): validation, level setup,
// workspace management, schedules and the MLMC driver.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stmlmc.h"
#include "stm_launch.h"

using namespace stm;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct LevelHost {
  LevelDev dev;          // host copy (device pointers inside)
  int64_t team_bytes;    // workspace per team without the space-time buffer
  int64_t u_bytes;       // space-time buffer m * n0 float64
  double* fib[kMaxMG] = {}; // device fibre table of every grid
  double* u0 = nullptr;  // device initial state at the nodes of grid 0
};

}  // namespace

struct stm_ctx {
  stm_problem p{};
  hipStream_t stream = nullptr;
  int device = 0;
  int n_cu = 256;
  std::string err;
  std::vector<LevelHost> levels;
  LevelDev* d_levels = nullptr;  // device copy of all LevelDev
  SolverParams prm{};
  bool inner_fp32 = false;
  bool any_mg = false;           // some level has a multigrid hierarchy (selects the solver kernel)
  // growable device buffers
  void* work = nullptr;
  size_t work_bytes = 0;
  TeamTask* d_tasks = nullptr;
  size_t tasks_cap = 0;
  SampleStatsDev* d_stats = nullptr;
  size_t stats_cap = 0;
  int* d_int = nullptr;
  size_t int_cap = 0;
  double* d_scratch = nullptr;
  size_t scratch_cap = 0;
  unsigned char* d_sync = nullptr;
  size_t sync_cap = 0;
  int* d_order = nullptr;        // sample order of split groups (MLMC launch)
  size_t order_cap = 0;
  double* d_rowmin = nullptr;    // per-sample minimum conductivity (MLMC launch)
  size_t rowmin_cap = 0;
  // phase timing
  hipEvent_t ev[2] = {nullptr, nullptr};
  stm_timings tm{};
  // measured mean device seconds per sample of each level with a team of G
  // workgroups, tsec[level][G] (0 = not measured yet)
  double tsec[STM_MAX_LEVELS][kMaxTeam + 1] = {};
  // device seconds of the predicted-hard samples of a grid relative to the
  // others at the same team size (measured after every launch that splits)
  double hard_ratio[STM_MAX_LEVELS] = {1.3, 1.3, 1.3, 1.3, 1.3, 1.3, 1.3, 1.3};
  // slowest over mean device seconds of the rest of a split group, which also
  // runs one sample per team, so that its slowest sample decides its end too
  double tail_ratio[STM_MAX_LEVELS] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
  int stage_bytes = 48 * 1024;   // dynamic LDS per solver workgroup
  void* scratch_dev = nullptr;   // device address of this device's no-allocation scratch array
};

namespace {

stm_status fail(stm_ctx* c, stm_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

stm_status hip_fail(stm_ctx* c, hipError_t e, const char* where) {
  return fail(c, STM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define STM_HIP(ctx, call)                                       \
  do {                                                           \
    hipError_t _e = (call);                                      \
    if (_e != hipSuccess) return hip_fail((ctx), _e, #call);     \
  } while (0)

template <typename T>
stm_status grow(stm_ctx* c, T** ptr, size_t* cap, size_t need_bytes) {
  if (need_bytes <= *cap) return STM_OK;
  if (*ptr) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    (void)hipFree(*ptr);
    *ptr = nullptr;
    *cap = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, need_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, STM_E_NOMEM, "hipMalloc of " + std::to_string(need_bytes) + " bytes failed");
  }
  *ptr = static_cast<T*>(p);
  *cap = need_bytes;
  return STM_OK;
}

GridDev make_grid(int dim, int nx, int ny, int nz, double lx, double ly, double lz) {
  GridDev g{};
  g.nx = nx;
  g.ny = ny;
  g.nz = dim == 3 ? nz : 1;
  g.n = g.nx * g.ny * g.nz;
  g.ex = nx - 1;
  g.ey = ny - 1;
  g.ez = dim == 3 ? nz - 1 : 1;
  g.ne = g.ex * g.ey * g.ez;
  g.hx = lx / (nx - 1);
  g.hy = ly / (ny - 1);
  g.hz = dim == 3 ? lz / (nz - 1) : 1.0;
  g.mnx = fdiv_magic(g.nx);
  g.mny = fdiv_magic(g.ny);
  g.mex = fdiv_magic(g.ex);
  g.mey = fdiv_magic(g.ey);
  return g;
}

double fiber_angle(const stm_problem& p, double y, double z) {
  switch (p.fiber_law) {
    case STM_FIBER_DIAG2D: return M_PI / 4 + 0.5 * y;
    case STM_FIBER_ROT3D: return -M_PI / 3 + (2 * M_PI / 3) * z / p.lz;
    case STM_FIBER_X: return 0.0;
    default: return M_PI / 4;
  }
}

stm_status validate_problem(stm_ctx* c, const stm_problem& p) {
  if (p.dim != 2 && p.dim != 3) return fail(c, STM_E_INVALID, "dim must be 2 or 3");
  if (!(p.lx > 0 && p.ly > 0 && (p.dim == 2 || p.lz > 0) && p.T > 0))
    return fail(c, STM_E_INVALID, "box lengths and T must be positive");
  if (!(p.sigma_f0 > 0) || !(p.transverse_ratio >= 0) || !std::isfinite(p.k_react) || !std::isfinite(p.a_react))
    return fail(c, STM_E_INVALID, "invalid physical parameters");
  if (p.n_levels < 1 || p.n_levels > STM_MAX_LEVELS) return fail(c, STM_E_INVALID, "n_levels out of range");
  if (p.n_modes < 1 || p.n_modes > 256) return fail(c, STM_E_INVALID, "n_modes must be in 1..256");
  if (p.precision != STM_PREC_FP64 && p.precision != STM_PREC_MIXED) return fail(c, STM_E_INVALID, "bad precision");
  if (p.fiber_law < 0 || p.fiber_law > 3) return fail(c, STM_E_INVALID, "bad fiber_law");
  if (p.gmres_restart < 0 || p.gmres_restart > kMaxRestart) return fail(c, STM_E_INVALID, "gmres_restart > 30");
  if (p.coarse_sweeps < 0 || p.coarse_sweeps > kMaxSweeps || p.smooth_steps < 0 || p.smooth_steps > kMaxSweeps)
    return fail(c, STM_E_INVALID, "sweep counts must be in 0..32");
  if (p.smoother < 0 || p.smoother > 1) return fail(c, STM_E_INVALID, "smoother must be 0 or 1");
  if (p.mg_levels < -1 || p.mg_levels > kMaxMG)
    return fail(c, STM_E_INVALID, "mg_levels must be -1 (deepest), 0 (default 1) or 1 .. 8");
  if (p.field_kind != STM_FIELD_LOGNORMAL && p.field_kind != STM_FIELD_ADDITIVE)
    return fail(c, STM_E_INVALID, "field_kind must be 0 (lognormal) or 1 (additive)");
  if (p.tau_relative != 0 && p.tau_relative != 1) return fail(c, STM_E_INVALID, "tau_relative must be 0 or 1");
  if (p.ic_kind != STM_IC_BALL && p.ic_kind != STM_IC_GAUSS) return fail(c, STM_E_INVALID, "ic_kind must be 0 or 1");
  if (p.qoi != STM_QOI_ACTIVATION && p.qoi != STM_QOI_SPACETIME) return fail(c, STM_E_INVALID, "qoi must be 0 or 1");
  if (p.newton_damping < -1 || p.newton_damping > 1) return fail(c, STM_E_INVALID, "newton_damping must be -1, 0 or 1");
  if (p.st_mode < 0 || p.st_mode > 1) return fail(c, STM_E_INVALID, "st_mode must be 0 or 1");
  if (p.st_mode == 1 && p.block_threads == 1024)
    return fail(c, STM_E_INVALID, "st_mode 1 runs with 256 or 512 threads per workgroup");
  if (!(p.ic_radius >= 0)) return fail(c, STM_E_INVALID, "ic_radius must be >= 0");
  if (p.ic_kind == STM_IC_GAUSS && !(p.ic_radius > 0))
    return fail(c, STM_E_INVALID, "the Gaussian initial state needs ic_radius > 0");
  if (!(p.theta == 0 || (p.theta >= 0.5 && p.theta <= 1.0)))
    return fail(c, STM_E_INVALID, "theta must be 0 (default) or in [1/2, 1]");
  if (p.lds_kb < 0 || p.lds_kb > 160) return fail(c, STM_E_INVALID, "lds_kb must be in 0..160");
  if (p.block_threads != 0 && p.block_threads != 256 && p.block_threads != 512 && p.block_threads != 1024)
    return fail(c, STM_E_INVALID, "block_threads must be 0, 256, 512 or 1024");
  for (int l = 0; l < p.n_levels; ++l) {
    const stm_level& L = p.levels[l];
    const int nz = p.dim == 3 ? L.nz : 1;
    if (L.nx < 3 || L.ny < 2 || (p.dim == 3 && (L.ny < 3 || L.nz < 2)) || L.m < 1)
      return fail(c, STM_E_INVALID, "level " + std::to_string(l) + ": grid too small");
    if (L.smooth_sweeps < 0 || L.smooth_sweeps > kMaxSweeps || !(L.cheb_ratio == 0 || L.cheb_ratio > 1))
      return fail(c, STM_E_INVALID, "level " + std::to_string(l) + ": smooth_sweeps in 0..32, cheb_ratio 0 or > 1");
    for (int g = 0; g < 32; ++g)
      if (!(L.team_seconds[g] >= 0 && std::isfinite(L.team_seconds[g])))
        return fail(c, STM_E_INVALID, "level " + std::to_string(l) + ": team_seconds must be finite and >= 0");
    if ((int64_t)L.nx * L.ny * nz > (int64_t)1 << 28)
      return fail(c, STM_E_INVALID, "level " + std::to_string(l) + ": grid too large");
    // a 3D pass gives each thread at most four staged node columns of a tile
    // (one row plus two halo rows at 256 threads per workgroup)
    if (p.dim == 3 && L.nx > 340)
      return fail(c, STM_E_UNSUPPORTED, "level " + std::to_string(l) + ": 3D rows are limited to 340 nodes");
    if ((int64_t)L.nx * L.ny * nz * std::max(L.nx, L.ny) >= (int64_t)1 << 32)
      return fail(c, STM_E_UNSUPPORTED, "level " + std::to_string(l) + ": grid too large for 32-bit index arithmetic");
    if (l > 0) {
      const stm_level& P = p.levels[l - 1];
      // every axis refined 2:1 or kept (a strip keeps its single element row)
      auto nested = [](int f, int c0) { return f == 2 * c0 - 1 || f == c0; };
      if (!nested(L.nx, P.nx) || !nested(L.ny, P.ny) || (p.dim == 3 && !nested(L.nz, P.nz)))
        return fail(c, STM_E_INVALID, "levels must be nested: each axis refined 2:1 or kept");
    }
  }
  return STM_OK;
}

void fill_defaults(stm_problem& p) {
  const bool mixed = p.precision == STM_PREC_MIXED;
  if (p.newton_tol <= 0) p.newton_tol = 1e-10;
  if (p.newton_max <= 0) p.newton_max = 30;
  if (p.gmres_rtol <= 0) p.gmres_rtol = mixed ? 1e-5 : 1e-10;
  if (p.gmres_restart <= 0) p.gmres_restart = 16;
  if (p.smooth_steps <= 0) p.smooth_steps = 2;
  if (p.smooth_omega <= 0) p.smooth_omega = 0.7;
  if (p.coarse_sweeps <= 0) p.coarse_sweeps = 8;
  if (p.cheb_ratio <= 1) p.cheb_ratio = p.dim == 2 ? 10.0 : 30.0;
  if (p.theta == 0) p.theta = 1.0;
  if (p.lds_kb <= 0) p.lds_kb = 144;
  if (p.mg_levels == 0) p.mg_levels = 1;
  if (p.max_lanes <= 0) p.max_lanes = 1024;
}

// Threads per solver workgroup.  Launches of the multi-grid variant take
// 256: with four waves per workgroup the 3D variant may use up to 512
// registers per lane and needs no scratch memory.
int auto_block(const stm_problem& p, int n0, bool mg) {
  if (p.block_threads) return p.block_threads;
  if (mg || n0 <= 2500) return 256;
  return 512;
}

stm_status build_level(stm_ctx* c, int l, LevelHost& out) {
  const stm_problem& p = c->p;
  const stm_level& lv = p.levels[l];
  LevelDev& d = out.dev;
  std::memset(&d, 0, sizeof(d));
  d.dim = p.dim;
  d.m = lv.m;
  d.T = p.T;
  d.dt = p.T / lv.m;
  // multigrid hierarchy: halve while every axis stays odd and >= 3 nodes
  int nx = lv.nx, ny = lv.ny, nz = p.dim == 3 ? lv.nz : 1;
  int nmg = 0;
  const int max_mg = p.mg_levels > 0 ? std::min(p.mg_levels, kMaxMG) : kMaxMG;  // -1: deepest
  while (true) {
    d.g[nmg++] = make_grid(p.dim, nx, ny, nz, p.lx, p.ly, p.lz);
    if (nmg >= max_mg) break;
    const bool odd = (nx % 2 == 1) && (ny % 2 == 1) && (p.dim == 2 || nz % 2 == 1);
    const int cx = (nx + 1) / 2, cy = (ny + 1) / 2, cz = (nz + 1) / 2;
    if (!odd || cx < 5 || cy < 5 || (p.dim == 3 && cz < 3)) break;
    nx = cx;
    ny = cy;
    nz = cz;
  }
  d.nmg = nmg;
  d.sweeps = lv.smooth_sweeps > 0 ? lv.smooth_sweeps : p.coarse_sweeps;
  d.cheb_ratio = lv.cheb_ratio > 0 ? lv.cheb_ratio : p.cheb_ratio;

  // fibre table of every grid, per element row (2D) / layer (3D) at that grid's centroids
  const GridDev& g0 = d.g[0];
  const double ratio = p.transverse_ratio;
  for (int k = 0; k < nmg; ++k) {
    const GridDev& g = d.g[k];
    const int rows = p.dim == 2 ? g.ey : g.ez;
    std::vector<double> fib(kFibStride * rows);
    for (int r = 0; r < rows; ++r) {
      const double yc = (r + 0.5) * g.hy, zc = (r + 0.5) * g.hz;
      const double th = p.dim == 2 ? fiber_angle(p, yc, 0.0) : fiber_angle(p, 0.0, zc);
      const double cth = std::cos(th), sth = std::sin(th);
      double* f = fib.data() + kFibStride * r;
      if (p.tau_relative) {  // tau_e = ratio sigma_e
        f[0] = cth * cth + ratio * sth * sth;
        f[1] = sth * sth + ratio * cth * cth;
        f[2] = (1.0 - ratio) * cth * sth;
      } else {  // tau = ratio sigma_f0
        f[0] = cth * cth;
        f[1] = sth * sth;
        f[2] = cth * sth;
      }
    }
    STM_HIP(c, hipMalloc(&out.fib[k], fib.size() * sizeof(double)));
    STM_HIP(c, hipMemcpy(out.fib[k], fib.data(), fib.size() * sizeof(double), hipMemcpyHostToDevice));
    d.fib[k] = out.fib[k];
  }
  {
    // initial state at the nodes of grid 0: the ball or the Gaussian bump
    const GridDev& g = d.g[0];
    const double cx = p.ic_center[0], cy = p.ic_center[1], cz = p.dim == 3 ? p.ic_center[2] : 0.0;
    const double r2 = p.ic_radius * p.ic_radius;
    std::vector<double> u0((size_t)g.n);
    for (int k = 0; k < g.nz; ++k)
      for (int j = 0; j < g.ny; ++j)
        for (int i = 0; i < g.nx; ++i) {
          const double x = i * g.hx - cx, y = j * g.hy - cy, z = p.dim == 3 ? k * g.hz - cz : 0.0;
          const double d2 = x * x + y * y + z * z;
          u0[((size_t)k * g.ny + j) * g.nx + i] =
              p.ic_kind == STM_IC_GAUSS ? std::exp(-d2 / r2) : (d2 <= r2 ? 1.0 : 0.0);
        }
    STM_HIP(c, hipMalloc(&out.u0, u0.size() * sizeof(double)));
    STM_HIP(c, hipMemcpy(out.u0, u0.data(), u0.size() * sizeof(double), hipMemcpyHostToDevice));
    d.u0 = out.u0;
  }
  // team workspace layout
  const size_t ti = c->inner_fp32 ? 4 : 8;
  const int n0 = g0.n;
  const size_t vs = (size_t)((n0 + 63) & ~63);
  const int R = p.gmres_restart;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return (int64_t)o; };
  d.off_u = take(8 * (size_t)n0);
  d.off_uprev = take(8 * (size_t)n0);
  d.off_wk1 = take(8 * (size_t)n0);
  d.off_tact = take(8 * (size_t)n0);
  d.off_V = take(ti * vs * (R + 1));
  d.off_Z = take(ti * vs * R);
  d.off_kd = take(8 * (size_t)n0);
  d.off_dlt = take(8 * (size_t)n0);
  d.off_dinv = take(ti * n0);
  for (int k = 0; k < nmg; ++k) {
    const GridDev& g = d.g[k];
    d.off_mgT[k] = take(ti * g.n);
    d.off_mgW[k] = take(ti * g.n);
    if (k > 0) {
      d.off_mgX[k] = take(ti * g.n);
      d.off_mgB[k] = take(ti * g.n);
      d.off_mgI[k] = take(ti * g.n);
      d.off_mgS[k] = take(8 * (size_t)g.ne);
      d.off_mgK[k] = take(8 * (size_t)g.n);
    }
    // float32 copy of the conductivities, read by the float32 3D passes
    // (the value each of them rounds to anyway)
    if (c->inner_fp32 && p.dim == 3) d.off_mgS32[k] = take(4 * (size_t)g.ne);
  }
  // words per grid-0 node of one preconditioner application: smoothing sweeps
  // (5 words each) and, above the coarsest grid, the residual (5 words as a
  // sweep), each on grid k weighted by its nodes
  {
    const int nu = p.smooth_steps;
    double w = 0.0;
    for (int k = 0; k < nmg; ++k) {
      const double frac = (double)d.g[k].n / g0.n;
      w += frac * 5.0 * (k + 1 < nmg ? 2 * nu + 1 : d.sweeps);
    }
    d.pc_words = w;
  }
  if (p.st_mode == 1) {
    // global space-time mode: Krylov basis, per-slab weights and inverse
    // diagonals, preconditioned vector over all m slabs, one slab temporary
    const size_t gsz = ti * vs * (size_t)lv.m;
    d.off_gV = take(gsz * (R + 1));
    d.off_gW = take(gsz);
    d.off_gD = take(gsz);
    d.off_gZ = take(gsz);
    d.off_gT = take(ti * vs);
  }
  out.team_bytes = (int64_t)off;
  d.off_U = off;
  // LDS tiles: maximise interior / staged nodes within the staging budget,
  // per field size and number of staged nodal fields (2 to 4)
  const size_t budget = (size_t)c->stage_bytes;
  for (int k = 0; k < nmg && p.dim == 3; ++k) {
    // 3D passes march through the planes: four top-face contributions per
    // element of one layer, a ring of three planes of two nodal fields over
    // the tile's rows plus a one-row halo, four partial sums per element of
    // one layer with a one-element border, two slots of two nodal fields over
    // the tile's rows and of the layer's conductivities (float64).  The
    // tallest tile within the budget (the kernel lowers it further to its
    // per-thread counts).
    const GridDev& gk = d.g[k];
    for (int es = 0; es < 2; ++es) {
      const size_t fb = es == 0 ? 8 : 4;
      int by = 0;
      for (int ry = 1; ry <= gk.ny; ++ry) {
        const size_t sy = std::min(ry + 2, gk.ny), sey = std::min(ry + 1, gk.ey);
        const size_t bytes = fb * (4 * sey * gk.ex + 6 * sy * gk.nx + 4 * (sey + 2) * (gk.ex + 2) +
                                   4 * (size_t)ry * gk.nx) +
                             16 * sey * gk.ex + 8;
        if (bytes > budget) break;
        by = ry;
      }
      if (by == 0) return fail(c, STM_E_UNSUPPORTED, "grid row too wide for the LDS staging budget");
      for (int nfl = 2; nfl <= 4; ++nfl) {
        d.tile_y[k][es][nfl - 2] = by;
        d.tile_z[k][es][nfl - 2] = 1;
      }
    }
  }
  for (int k = 0; k < nmg && p.dim == 2; ++k) {
    const GridDev& gk = d.g[k];
    for (int es = 0; es < 2; ++es) {
      const size_t fb = es == 0 ? 8 : 4;
      for (int nfl = 2; nfl <= 4; ++nfl) {
        int by = 1, bz = 1;
        double best = -1.0;
        const int zmax = p.dim == 3 ? gk.nz : 1;
        for (int rz = 1; rz <= zmax; ++rz) {
          for (int ry = 1; ry <= gk.ny; ++ry) {
            const int sy = std::min(ry + 2, gk.ny), sz = p.dim == 3 ? std::min(rz + 2, gk.nz) : 1;
            const int ey = std::min(ry + 1, gk.ey), ez = p.dim == 3 ? std::min(rz + 1, gk.ez) : 1;
            const size_t nv = p.dim == 3 ? 8 : 4;  // per-element vertex contributions
            // staged nodal fields, element conductivities, element
            // contributions, fibre rows of the tile
            const size_t bytes = nfl * fb * (size_t)sy * sz * gk.nx + 16 +
                                 (8 + fb * nv) * (size_t)ey * ez * gk.ex + 16 +
                                 8 * kFibStride * (size_t)(p.dim == 2 ? ey : ez);
            if (bytes > budget) break;
            const double eff = (double)std::min(ry, gk.ny) * std::min(rz, zmax) / ((double)sy * sz) + 1e-6 * ry * rz;
            if (eff > best) {
              best = eff;
              by = ry;
              bz = rz;
            }
          }
        }
        if (best < 0) return fail(c, STM_E_UNSUPPORTED, "grid row too wide for the LDS staging budget");
        d.tile_y[k][es][nfl - 2] = by;
        d.tile_z[k][es][nfl - 2] = bz;
      }
    }
  }
  // fused two-sweep smoother pass (2D): five nodal fields over the tile's rows
  // plus two halo rows each side, element conductivities and contributions and
  // fibre rows of the tile's rows plus three
  for (int es = 0; es < 2 && p.dim == 2; ++es) {
    const size_t fb = es == 0 ? 8 : 4;
    int by = 0;
    for (int ry = 1; ry <= g0.ny; ++ry) {
      const size_t sy = std::min(ry + 4, g0.ny), sey = std::min(ry + 3, g0.ey);
      const size_t bytes = 5 * fb * sy * g0.nx + 16 + (8 + 4 * fb) * sey * g0.ex + 16 + 8 * kFibStride * sey;
      if (bytes > budget) break;
      by = ry;
    }
    if (by == 0) return fail(c, STM_E_UNSUPPORTED, "grid row too wide for the LDS staging budget");
    if (es == 0) d.tile_p8 = by; else d.tile_p4 = by;
  }
  out.u_bytes = (int64_t)align_up(8 * (size_t)n0 * lv.m);
  d.team_bytes = out.team_bytes;
  return STM_OK;
}

stm_status check_ptr(stm_ctx* c, const void* ptr, const char* name) {
  if (!ptr) return fail(c, STM_E_INVALID, std::string(name) + " is NULL");
  return STM_OK;
}

// Elapsed device time between two events recorded on the context stream.
stm_status timed_begin(stm_ctx* c) {
  STM_HIP(c, hipEventRecord(c->ev[0], c->stream));
  return STM_OK;
}
stm_status timed_end(stm_ctx* c, double* acc_ms) {
  STM_HIP(c, hipEventRecord(c->ev[1], c->stream));
  STM_HIP(c, hipEventSynchronize(c->ev[1]));
  float ms = 0.f;
  STM_HIP(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
  *acc_ms += ms;
  return STM_OK;
}

// Expand teams into one TeamTask per workgroup and launch the solver
// (synchronous).  Members of a team with G > 1 are placed on workgroup
// indices of one residue class mod 8, so that with round-robin dispatch over
// the 8 XCDs a team shares one L2; correctness does not depend on it.
// Device bytes of a launch's team synchronisation area: barrier counters (one
// 128-byte line per team), reduction partials and the fault flag.
size_t sync_bytes_for(size_t n_teams, int max_g) {
  return n_teams * 32 * 4 + n_teams * 2 * (size_t)max_g * 16 * 8 + 256;
}

// Caller-provided device areas for run_tasks (the allocation-free entry point);
// null members mean the context's growable buffers.
struct FixedAreas {
  unsigned char* sync = nullptr;
  size_t sync_cap = 0;
  TeamTask* tasks = nullptr;
  size_t tasks_cap = 0;
};

stm_status run_tasks(stm_ctx* c, std::vector<TeamTask>& teams, int block, const FixedAreas* fixed = nullptr) {
  if (teams.empty()) return STM_OK;
  int n_blocks = 0, n_multi = 0, max_g = 1;
  for (auto& t : teams) {
    n_blocks += t.G;
    if (t.G > 1) ++n_multi;
    max_g = std::max(max_g, t.G);
  }
  const bool coop = max_g > 1;
  const size_t ctr_words = (size_t)teams.size() * 32;
  const size_t part_doubles = (size_t)teams.size() * 2 * max_g * 16;
  const size_t sync_bytes = sync_bytes_for(teams.size(), max_g);
  stm_status st = STM_OK;
  unsigned char* sync = nullptr;
  if (fixed) {
    if (sync_bytes > fixed->sync_cap || (size_t)n_blocks * sizeof(TeamTask) > fixed->tasks_cap)
      return fail(c, STM_E_INVALID, "launch tables exceed the fixed scratch areas");
    sync = fixed->sync;
  } else {
    if ((st = grow(c, &c->d_sync, &c->sync_cap, sync_bytes))) return st;
    sync = c->d_sync;
  }
  unsigned* ctr = reinterpret_cast<unsigned*>(sync);
  double* part = reinterpret_cast<double*>(sync + ctr_words * 4);
  int* fault = reinterpret_cast<int*>(sync + ctr_words * 4 + part_doubles * 8);
  // placement: free slots per residue class
  std::vector<std::vector<int>> cls(8);
  for (int b = n_blocks - 1; b >= 0; --b) cls[b % 8].push_back(b);
  std::vector<TeamTask> blocks(n_blocks);
  std::vector<char> used(n_blocks, 0);
  auto take_any = [&]() {
    for (int r = 0; r < 8; ++r)
      while (!cls[r].empty()) {
        const int b = cls[r].back();
        cls[r].pop_back();
        if (!used[b]) return b;
      }
    return -1;
  };
  int next_cls = 0;
  for (size_t t = 0; t < teams.size(); ++t) {
    TeamTask base = teams[t];
    base.bar = ctr + t * 32;
    base.part = part + t * 2 * max_g * 16;
    base.fault = fault;
    if (base.G == 1) continue;
    int r = next_cls;
    next_cls = (next_cls + 1) % 8;
    for (int g = 0; g < base.G; ++g) {
      int b = -1;
      while (!cls[r].empty() && b < 0) {
        const int cand = cls[r].back();
        cls[r].pop_back();
        if (!used[cand]) b = cand;
      }
      if (b < 0) b = take_any();
      used[b] = 1;
      blocks[b] = base;
      blocks[b].rank = g;
    }
  }
  for (size_t t = 0; t < teams.size(); ++t) {
    if (teams[t].G != 1) continue;
    const int b = take_any();
    used[b] = 1;
    blocks[b] = teams[t];
    blocks[b].rank = 0;
    blocks[b].bar = ctr + t * 32;
    blocks[b].part = part + t * 2 * 16;
    blocks[b].fault = fault;
  }
  (void)n_multi;
  TeamTask* d_tasks = nullptr;
  if (fixed) {
    d_tasks = fixed->tasks;
  } else {
    if ((st = grow(c, &c->d_tasks, &c->tasks_cap, blocks.size() * sizeof(TeamTask)))) return st;
    d_tasks = c->d_tasks;
  }
  STM_HIP(c, hipMemcpyAsync(d_tasks, blocks.data(), blocks.size() * sizeof(TeamTask), hipMemcpyHostToDevice,
                            c->stream));
  hipError_t e = launch_fill_u32(ctr, 0u, (int64_t)(sync_bytes / 4), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "fill");
  if ((st = timed_begin(c))) return st;
  e = launch_team_solver(c->p.dim, c->inner_fp32, c->any_mg, c->d_levels, d_tasks, n_blocks, c->prm, block,
                         (size_t)c->stage_bytes, coop, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, coop ? "cooperative team solver launch" : "team solver launch");
  // the task table stays alive until the kernel has finished
  if ((st = timed_end(c, &c->tm.solve_ms))) return st;
  int hf = 0;
  STM_HIP(c, hipMemcpy(&hf, fault, sizeof(int), hipMemcpyDeviceToHost));
  if (hf) return fail(c, STM_E_DEVICE, "a team barrier wait timed out");
  c->tm.solve_launches += 1;
  c->tm.solve_teams = (int)teams.size();
  c->tm.solve_block = block;
  c->tm.solve_blocks = n_blocks;
  return STM_OK;
}

// Largest team size a level allows: single-grid V-cycle and >= 3 node rows per member
// (a member's staged tiles carry one halo row on each side).
int max_team(const stm_ctx* c, int level) {
  const LevelDev& d = c->levels[level].dev;
  if (d.nmg > 1) return 1;
  return std::max(1, std::min(kMaxTeam, d.g[0].ny / 3));
}

// Workgroups that can be resident at once for the solver configuration.
int block_capacity(stm_ctx* c, int block) {
  const int occ = team_solver_occupancy(c->p.dim, c->inner_fp32, c->any_mg, c->p.st_mode == 1, block,
                                        (size_t)c->stage_bytes);
  return std::max(1, occ) * c->n_cu;
}

void reset_timings(stm_ctx* c) { c->tm = stm_timings{}; }

void* device_scratch(int device);

}  // namespace

extern "C" {

stm_status stm_create(const stm_problem* p, void* hip_stream, stm_ctx** out) {
  if (!out) return STM_E_INVALID;
  *out = nullptr;
  if (!p) return STM_E_INVALID;
  stm_ctx* c = new stm_ctx();
  c->p = *p;
  stm_status st = validate_problem(c, c->p);
  if (st != STM_OK) {
    std::fprintf(stderr, "stm_create: %s\n", c->err.c_str());
    delete c;
    return st;
  }
  fill_defaults(c->p);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->inner_fp32 = c->p.precision == STM_PREC_MIXED;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  }
  if (e != hipSuccess) {
    delete c;
    return STM_E_DEVICE;
  }
  {
    // staging budget: requested KiB, within the per-workgroup LDS limit minus static use
    int max_lds = 65536;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
      max_lds = 65536;
    const int static_lds = 13 * 1024;
    c->stage_bytes = std::min(c->p.lds_kb * 1024, max_lds - static_lds);
  }
  c->levels.resize(c->p.n_levels);
  for (int l = 0; l < c->p.n_levels; ++l) {
    st = build_level(c, l, c->levels[l]);
    if (st != STM_OK) {
      std::fprintf(stderr, "stm_create: %s\n", c->err.c_str());
      stm_destroy(c);
      return st;
    }
    c->any_mg = c->any_mg || c->levels[l].dev.nmg > 1;
    for (int g = 1; g <= kMaxTeam; ++g) c->tsec[l][g] = std::max(0.0, c->p.levels[l].team_seconds[g - 1]);
  }
  // this device's no-allocation scratch array (stm_st_solve_noalloc); resolved
  // here, with the device current, once per device
  c->scratch_dev = device_scratch(c->device);
  if (hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess) {
    stm_destroy(c);
    return STM_E_DEVICE;
  }
  std::vector<LevelDev> lv(c->p.n_levels);
  for (int l = 0; l < c->p.n_levels; ++l) lv[l] = c->levels[l].dev;
  if (hipMalloc(&c->d_levels, lv.size() * sizeof(LevelDev)) != hipSuccess ||
      hipMemcpy(c->d_levels, lv.data(), lv.size() * sizeof(LevelDev), hipMemcpyHostToDevice) != hipSuccess) {
    stm_destroy(c);
    return STM_E_DEVICE;
  }
  SolverParams& s = c->prm;
  s.k_react = c->p.k_react;
  s.a_react = c->p.a_react;
  s.tau = c->p.tau_relative ? 0.0 : c->p.transverse_ratio * c->p.sigma_f0;
  s.zr = c->p.tau_relative ? c->p.transverse_ratio : 0.0;
  s.threshold = c->p.threshold;
  s.newton_tol = c->p.newton_tol;
  s.gmres_rtol = c->p.gmres_rtol;
  s.smooth_omega = c->p.smooth_omega;
  s.newton_max = c->p.newton_max;
  s.restart = c->p.gmres_restart;
  s.smooth_steps = c->p.smooth_steps;
  s.coarse_sweeps = c->p.coarse_sweeps;
  s.smoother = (c->p.smoother == 1) ? 0 : 1;  // kernel: 1 = Chebyshev weights, 0 = fixed
  s.cheb_ratio = c->p.cheb_ratio;
  s.power_iters = 40;
  s.theta = c->p.theta;
  s.damping = c->p.newton_damping >= 0 ? 1 : 0;
  s.global_st = c->p.st_mode;
  *out = c;
  return STM_OK;
}

void stm_destroy(stm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& l : c->levels) {
    for (double* f : l.fib)
      if (f) (void)hipFree(f);
    if (l.u0) (void)hipFree(l.u0);
  }
  if (c->d_levels) (void)hipFree(c->d_levels);
  if (c->work) (void)hipFree(c->work);
  if (c->d_tasks) (void)hipFree(c->d_tasks);
  if (c->d_stats) (void)hipFree(c->d_stats);
  if (c->d_int) (void)hipFree(c->d_int);
  if (c->d_order) (void)hipFree(c->d_order);
  if (c->d_rowmin) (void)hipFree(c->d_rowmin);
  if (c->d_scratch) (void)hipFree(c->d_scratch);
  if (c->d_sync) (void)hipFree(c->d_sync);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

const char* stm_last_error(const stm_ctx* c) { return c ? c->err.c_str() : "null context"; }

stm_status stm_get_timings(const stm_ctx* c, stm_timings* out) {
  if (!c || !out) return STM_E_INVALID;
  *out = c->tm;
  return STM_OK;
}

stm_status stm_level_size(const stm_ctx* c, int level, int* n_nodes, int* n_elements, int* m) {
  if (!c || level < 0 || level >= c->p.n_levels) return STM_E_INVALID;
  const LevelDev& d = c->levels[level].dev;
  if (n_nodes) *n_nodes = d.g[0].n;
  if (n_elements) *n_elements = d.g[0].ne;
  if (m) *m = d.m;
  return STM_OK;
}

stm_status stm_kl_synthesize(stm_ctx* c, int level, const double* modes, const double* xi, int S, double* sigma) {
  if (!c) return STM_E_INVALID;
  c->err.clear();
  if (level < 0 || level >= c->p.n_levels) return fail(c, STM_E_INVALID, "level out of range");
  if (S < 0) return fail(c, STM_E_INVALID, "S < 0");
  if (S == 0) return STM_OK;
  stm_status st;
  if ((st = check_ptr(c, modes, "modes")) || (st = check_ptr(c, xi, "xi")) || (st = check_ptr(c, sigma, "sigma")))
    return st;
  const int E = c->levels[level].dev.g[0].ne;
  reset_timings(c);
  if ((st = timed_begin(c))) return st;
  hipError_t e = launch_kl_synthesize(modes, xi, sigma, S, E, c->p.n_modes, c->p.sigma_f0,
                                      c->p.precision == STM_PREC_MIXED, c->p.field_kind == STM_FIELD_ADDITIVE,
                                      c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kl launch");
  return timed_end(c, &c->tm.kl_ms);
}

}  // extern "C"

// The no-allocation area (see stm_st_solve_noalloc): one per device, resolved
// once per device with the device current.  In host code the array's name is
// only a stand-in for the symbol; its device address comes from
// hipGetSymbolAddress and is the only one used.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (null on error).
void* device_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

// stm_st_solve and stm_st_solve_noalloc.  With noalloc every device area the
// launch needs beyond the caller's arrays -- team synchronisation, the task
// table, per-sample statistics and the team workspaces -- is carved from the
// device's scratch array (fewer lanes if the workspaces do not all fit), and
// no device memory is allocated.
stm_status st_solve_impl(stm_ctx* c, int level, const double* sigma, const double* u0_guess, int S, double* u,
                         stm_solve_stats* stats_host, bool noalloc) {
  if (!c) return STM_E_INVALID;
  c->err.clear();
  if (level < 0 || level >= c->p.n_levels) return fail(c, STM_E_INVALID, "level out of range");
  if (S < 0) return fail(c, STM_E_INVALID, "S < 0");
  if (S == 0) return STM_OK;
  stm_status st;
  if ((st = check_ptr(c, sigma, "sigma")) || (st = check_ptr(c, u, "u"))) return st;
  LevelHost& L = c->levels[level];
  const int block = auto_block(c->p, L.dev.g[0].n, c->any_mg);
  const int cap = std::min(c->p.max_lanes, block_capacity(c, block));
  // few samples: several workgroups per sample (up to the level's limit)
  int G = 1;
  if (c->p.team_size > 0) G = std::min(c->p.team_size, max_team(c, level));
  else if (S * 2 <= cap) G = std::min(max_team(c, level), std::max(1, cap / S));
  int lanes = std::max(1, std::min(S, cap / G));
  unsigned char* work = nullptr;
  SampleStatsDev* d_stats = nullptr;
  FixedAreas areas;
  if (noalloc) {
    unsigned char* base = static_cast<unsigned char*>(c->scratch_dev);
    if (!base) return fail(c, STM_E_DEVICE, "the no-allocation scratch array of this device is not available");
    const size_t stats_bytes = align_up((size_t)S * sizeof(SampleStatsDev));
    auto need = [&](int ln) {
      return align_up(sync_bytes_for((size_t)ln, G)) + align_up((size_t)ln * G * sizeof(TeamTask)) + stats_bytes +
             (size_t)ln * (size_t)L.team_bytes;
    };
    while (lanes > 1 && need(lanes) > kNoAllocBytes) --lanes;
    if (need(lanes) > kNoAllocBytes)
      return fail(c, STM_E_INVALID,
                  "stm_st_solve_noalloc needs " + std::to_string(need(lanes)) + " bytes of scratch for " +
                      std::to_string(S) + " samples on level " + std::to_string(level) + "; the array holds " +
                      std::to_string(kNoAllocBytes));
    size_t off = 0;
    areas.sync = base + off;
    areas.sync_cap = align_up(sync_bytes_for((size_t)lanes, G));
    off += areas.sync_cap;
    areas.tasks = reinterpret_cast<TeamTask*>(base + off);
    areas.tasks_cap = align_up((size_t)lanes * G * sizeof(TeamTask));
    off += areas.tasks_cap;
    d_stats = reinterpret_cast<SampleStatsDev*>(base + off);
    off += stats_bytes;
    work = base + off;
  } else {
    if ((st = grow(c, &c->work, &c->work_bytes, (size_t)lanes * L.team_bytes))) return st;
    if ((st = grow(c, &c->d_stats, &c->stats_cap, (size_t)S * sizeof(SampleStatsDev)))) return st;
    work = static_cast<unsigned char*>(c->work);
    d_stats = c->d_stats;
  }
  std::vector<TeamTask> tasks(lanes);
  for (int i = 0; i < lanes; ++i) {
    TeamTask& t = tasks[i];
    t = TeamTask{};
    t.level = level;
    t.first = i;
    t.stride = lanes;
    t.count = (S - i + lanes - 1) / lanes;
    t.sigma = sigma;
    t.u_out = u;
    t.u_guess = u0_guess;
    t.t_act = nullptr;
    t.work = work + (size_t)i * L.team_bytes;
    t.stats = d_stats;
    t.G = G;
  }
  reset_timings(c);
  if ((st = run_tasks(c, tasks, block, noalloc ? &areas : nullptr))) return st;
  int worst = 0;
  SampleStatsDev sd[64];
  for (int s0 = 0; s0 < S; s0 += 64) {
    const int ns = std::min(64, S - s0);
    STM_HIP(c, hipMemcpy(sd, d_stats + s0, ns * sizeof(SampleStatsDev), hipMemcpyDeviceToHost));
    for (int q = 0; q < ns; ++q) {
      const int s = s0 + q;
      if (sd[q].status < worst) worst = sd[q].status;
      c->tm.solve_bytes += sd[q].alg_bytes;
      c->tm.solve_bytes_model += sd[q].model_bytes;
      if (stats_host) {
        stm_solve_stats& o = stats_host[s];
        o.status = sd[q].status;
        o.newton_max_per_slab = sd[q].newton_max_per_slab;
        o.newton_iters = sd[q].newton_iters;
        o.krylov_iters = sd[q].krylov_iters;
        o.final_step = sd[q].final_step;
        o.device_seconds = sd[q].ticks * 1e-8;
        o.algorithmic_bytes = sd[q].alg_bytes;
        o.model_bytes = sd[q].model_bytes;
        o.damped_steps = sd[q].damped;
        for (int k = 0; k < 8; ++k) o.phase_seconds[k] = sd[q].phase_ticks[k] * 1e-8;
      }
    }
  }
  if (worst == STM_E_NONFINITE) return fail(c, STM_E_NONFINITE, "non-finite residual in a sample");
  if (worst == STM_E_NOT_CONVERGED) return fail(c, STM_E_NOT_CONVERGED, "Newton iteration limit reached in a sample");
  return STM_OK;
}

}  // namespace

extern "C" {

stm_status stm_st_solve(stm_ctx* c, int level, const double* sigma, const double* u0_guess, int S, double* u,
                        stm_solve_stats* stats_host) {
  return st_solve_impl(c, level, sigma, u0_guess, S, u, stats_host, false);
}

stm_status stm_st_solve_noalloc(stm_ctx* c, int level, const double* sigma, const double* u0_guess, int S,
                                double* u, stm_solve_stats* stats_host) {
  return st_solve_impl(c, level, sigma, u0_guess, S, u, stats_host, true);
}

stm_status stm_activation_map(stm_ctx* c, int level, const double* u, int S, double* t_act, int* n_censored_host) {
  if (!c) return STM_E_INVALID;
  c->err.clear();
  if (level < 0 || level >= c->p.n_levels) return fail(c, STM_E_INVALID, "level out of range");
  if (S < 0) return fail(c, STM_E_INVALID, "S < 0");
  if (S == 0) return STM_OK;
  stm_status st;
  if ((st = check_ptr(c, u, "u")) || (st = check_ptr(c, t_act, "t_act"))) return st;
  const LevelDev& d = c->levels[level].dev;
  int* cen = nullptr;
  if (n_censored_host) {
    if ((st = grow(c, &c->d_int, &c->int_cap, (size_t)S * sizeof(int)))) return st;
    // a fill kernel rather than a memset node, so that the call stays correct under graph capture
    const hipError_t fe = launch_fill_u32(reinterpret_cast<unsigned*>(c->d_int), 0u, (int64_t)S, c->stream);
    if (fe != hipSuccess) return hip_fail(c, fe, "fill");
    cen = c->d_int;
  }
  reset_timings(c);
  if ((st = timed_begin(c))) return st;
  hipError_t e = launch_activation_map(d.g[0], d.m, d.dt, d.T, c->p.threshold, d.u0, u, S, t_act, cen, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "activation launch");
  if ((st = timed_end(c, &c->tm.stats_ms))) return st;
  if (n_censored_host) {
    STM_HIP(c, hipMemcpyAsync(n_censored_host, c->d_int, S * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    STM_HIP(c, hipStreamSynchronize(c->stream));
  }
  return STM_OK;
}

stm_status stm_prolong_st(stm_ctx* c, int level, const double* u_coarse, int S, double* u_fine) {
  if (!c) return STM_E_INVALID;
  c->err.clear();
  if (level < 1 || level >= c->p.n_levels) return fail(c, STM_E_INVALID, "level must be in 1 .. n_levels - 1");
  if (S < 0) return fail(c, STM_E_INVALID, "S < 0");
  if (S > 65535) return fail(c, STM_E_INVALID, "S > 65535 samples per call");
  if (S == 0) return STM_OK;
  stm_status st;
  if ((st = check_ptr(c, u_coarse, "u_coarse")) || (st = check_ptr(c, u_fine, "u_fine"))) return st;
  const LevelDev& dc = c->levels[level - 1].dev;
  const LevelDev& df = c->levels[level].dev;
  if (df.m > 65535) return fail(c, STM_E_UNSUPPORTED, "more than 65535 time steps");
  reset_timings(c);
  if ((st = timed_begin(c))) return st;
  hipError_t e = launch_prolong_st(dc.g[0], df.g[0], c->p.dim, dc.m, df.m, df.u0, u_coarse, S, u_fine, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "prolongation launch");
  return timed_end(c, &c->tm.stats_ms);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// MLMC driver
// ---------------------------------------------------------------------------
namespace {

struct Group {          // all fine or all coarse members of one MLMC level
  int grid;             // level index of the grid solved
  int mlmc_level;
  bool coarse;
  int n0, n1;           // samples [n0, n1) solved in this round
  bool ordered = false; // the group's samples are order[o0 .. o1) of the round's order list
  bool hard = false;    // the predicted-hard part of a split group
  int o0 = 0, o1 = 0;
  double t[kMaxTeam + 1];  // device seconds per sample with a team of G workgroups (G = 1 .. gmax)
  int lanes;            // teams
  int G;                // workgroups per team
  int gmax;             // largest team the grid allows
};

// Per-sample seconds of grid l for team sizes 1 .. gmax.  Measured values
// (the problem's table, then every launch's own timings) are used where
// known; the rest come from t(G) = t1 (a + (1 - a) / G), the part a of a
// sample's time that does not shrink with the team (synchronisation, per-pass
// overheads) fitted to the two measured sizes furthest apart, a = 0.15
// without two, and t1 from the static model without any.
void team_times(const stm_ctx* c, int l, int gmax, double* t) {
  const LevelDev& d = c->levels[l].dev;
  int g0 = 0, g1 = 0;
  for (int g = 1; g <= gmax; ++g)
    if (c->tsec[l][g] > 0) {
      if (!g0) g0 = g;
      g1 = g;
    }
  double a = 0.15, t1 = 2e-8 * (double)(d.g[0].n + 3000) * d.m;
  auto shape = [&](double aa, int g) { return aa + (1.0 - aa) / g; };
  if (g0 && g1 > g0) {
    // ratio r = t(g1) / t(g0) = shape(a, g1) / shape(a, g0), solved for a
    const double r = c->tsec[l][g1] / c->tsec[l][g0];
    const double p0 = 1.0 / g0, p1 = 1.0 / g1;
    const double den = (1.0 - p1) - r * (1.0 - p0);
    if (den != 0.0) a = std::min(1.0, std::max(0.0, (r * p0 - p1) / den));
  }
  if (g0) t1 = c->tsec[l][g0] / shape(a, g0);
  for (int g = 1; g <= gmax; ++g) t[g] = c->tsec[l][g] > 0 ? c->tsec[l][g] : t1 * shape(a, g);
}

// Team allocation for one persistent launch: the smallest makespan target T
// (bisection) for which every group fits, each group taking the team size
// that needs the fewest workgroups -- a team of G runs floor(T / t(G))
// samples in sequence (each warm-started from the previous) -- and the
// workgroups of all groups fit the co-resident budget.
int group_count(const Group& g) { return g.ordered ? g.o1 - g.o0 : g.n1 - g.n0; }

bool fit_lanes(std::vector<Group>& gs, double T, int budget) {
  long used = 0;
  for (auto& g : gs) {
    const int N = group_count(g);
    g.lanes = 0;
    g.G = 1;
    if (N <= 0) continue;
    long best = -1;
    for (int G = 1; G <= g.gmax; ++G) {
      if (g.t[G] > T) continue;
      const long per = std::max(1L, (long)std::floor(T / g.t[G] + 1e-9));
      const long lanes = (N + per - 1) / per;
      if (best < 0 || lanes * G < best) {
        best = lanes * G;
        g.G = G;
        g.lanes = (int)lanes;
      }
    }
    if (best < 0) return false;
    used += best;
  }
  return used <= budget;
}

void allocate_lanes(std::vector<Group>& gs, int budget) {
  double lo = 0.0, hi = 0.0;
  for (auto& g : gs) {
    if (group_count(g) <= 0) continue;
    double tmin = g.t[1];
    for (int G = 2; G <= g.gmax; ++G) tmin = std::min(tmin, g.t[G]);
    lo = std::max(lo, tmin);
    hi += group_count(g) * g.t[1];
  }
  if (hi <= 0.0) {
    for (auto& g : gs) {
      g.G = 1;
      g.lanes = 0;
    }
    return;
  }
  hi = std::max(hi, lo);
  if (!fit_lanes(gs, hi, budget)) {  // budget too small for any balance: one workgroup per group
    for (auto& g : gs) {
      g.G = 1;
      g.lanes = (group_count(g) > 0) ? 1 : 0;
    }
    return;
  }
  for (int it = 0; it < 60 && hi - lo > 1e-4 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (fit_lanes(gs, mid, budget)) hi = mid;
    else lo = mid;
  }
  fit_lanes(gs, hi, budget);
}

}  // namespace

extern "C" stm_status stm_mlmc_estimate(stm_ctx* c, const int* N_host, const double* const* modes_host,
                                        const double* const* xi_host, const int* capacity_host, double target_rmse,
                                        int pilot, stm_mlmc_result* out) {
  if (!c) return STM_E_INVALID;
  c->err.clear();
  stm_status st;
  if (!modes_host || !xi_host || !out) return fail(c, STM_E_INVALID, "modes, xi and out are required");
  if (!out->mean || !out->var) return fail(c, STM_E_INVALID, "out->mean and out->var are required");
  const int L1 = c->p.n_levels;
  const int M = c->p.n_modes;
  std::vector<int> cap(L1), N(L1, 0);
  for (int l = 0; l < L1; ++l) {
    if (!modes_host[l] || !xi_host[l]) return fail(c, STM_E_INVALID, "modes/xi pointer of a level is NULL");
    cap[l] = capacity_host ? capacity_host[l] : (N_host ? N_host[l] : 0);
    if (N_host) {
      if (N_host[l] < 2) return fail(c, STM_E_INVALID, "each level needs at least 2 samples");
      if (N_host[l] > cap[l]) return fail(c, STM_E_INVALID, "N exceeds capacity");
    }
  }
  const bool adaptive = (N_host == nullptr);
  if (adaptive) {
    if (!(target_rmse > 0) || pilot < 2) return fail(c, STM_E_INVALID, "adaptive mode needs target_rmse > 0, pilot >= 2");
    for (int l = 0; l < L1; ++l)
      if (cap[l] < pilot) return fail(c, STM_E_INVALID, "capacity below pilot");
  }
  const LevelDev& dL = c->levels[L1 - 1].dev;
  const int nL = dL.g[0].n;
  const bool st_qoi = c->p.qoi == STM_QOI_SPACETIME;
  const size_t P = st_qoi ? (size_t)dL.m * nL : (size_t)nL;  // QoI points on the finest (space-time) grid
  if (P >= ((size_t)1 << 31) - 256) return fail(c, STM_E_UNSUPPORTED, "too many QoI points for one launch");
  // device buffers: sigma and activation maps of every sample (fine and coarse
  // members), and for the space-time QoI their solutions
  std::vector<size_t> off_sf(L1), off_sc(L1), off_tf(L1), off_tc(L1), off_uf(L1, 0), off_uc(L1, 0);
  size_t tot = 0;
  for (int l = 0; l < L1; ++l) {
    const LevelDev& df = c->levels[l].dev;
    const int nf = df.g[0].n, ef = df.g[0].ne;
    off_sf[l] = tot; tot += (size_t)cap[l] * ef;
    off_tf[l] = tot; tot += (size_t)cap[l] * nf;
    if (st_qoi) { off_uf[l] = tot; tot += (size_t)cap[l] * df.m * nf; }
    if (l > 0) {
      const LevelDev& dc = c->levels[l - 1].dev;
      const int nc = dc.g[0].n, ec = dc.g[0].ne;
      off_sc[l] = tot; tot += (size_t)cap[l] * ec;
      off_tc[l] = tot; tot += (size_t)cap[l] * nc;
      if (st_qoi) { off_uc[l] = tot; tot += (size_t)cap[l] * dc.m * nc; }
    }
  }
  int max_cap = 0;
  for (int l = 0; l < L1; ++l) max_cap = std::max(max_cap, cap[l]);
  const int chunk = 64;
  const size_t part_sz = (size_t)((max_cap + chunk - 1) / chunk) * 6 * P;
  const size_t vpart_sz = (P + 255) / 256;
  const size_t off_part = tot; tot += part_sz;
  const size_t off_vpart = tot; tot += vpart_sz;
  if ((st = grow(c, &c->d_scratch, &c->scratch_cap, tot * sizeof(double)))) return st;
  double* S0 = c->d_scratch;
  // per-sample stats for every (level, member, sample)
  std::vector<size_t> off_stf(L1), off_stc(L1);
  size_t nst = 0;
  for (int l = 0; l < L1; ++l) {
    off_stf[l] = nst; nst += cap[l];
    off_stc[l] = nst; nst += cap[l];
  }
  if ((st = grow(c, &c->d_stats, &c->stats_cap, nst * sizeof(SampleStatsDev)))) return st;

  std::vector<int> Ndone(L1, 0);
  std::vector<int> Ntarget(L1);
  for (int l = 0; l < L1; ++l) Ntarget[l] = adaptive ? pilot : N_host[l];
  std::vector<double> V(L1, 0.0), cost(L1, 0.0);
  std::vector<double> level_norm(L1, 0.0);
  std::vector<SampleStatsDev> sh(nst);
  int rounds = 0;
  int worst = 0;
  const bool mixed = c->p.precision == STM_PREC_MIXED;
  const bool additive = c->p.field_kind == STM_FIELD_ADDITIVE;
  const int lane_budget = c->p.max_lanes;

  reset_timings(c);
  while (true) {
    ++rounds;
    if ((st = timed_begin(c))) return st;
    // 1) KL synthesis for the new samples of every level (fine and coarse member share xi)
    for (int l = 0; l < L1; ++l) {
      const int n0 = Ndone[l], n1 = Ntarget[l];
      if (n1 <= n0) continue;
      const int ef = c->levels[l].dev.g[0].ne;
      hipError_t e = launch_kl_synthesize(modes_host[l], xi_host[l] + (size_t)n0 * M, S0 + off_sf[l] + (size_t)n0 * ef,
                                          n1 - n0, ef, M, c->p.sigma_f0, mixed, additive, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "kl launch");
      if (l > 0) {
        const int ec = c->levels[l - 1].dev.g[0].ne;
        e = launch_kl_synthesize(modes_host[l - 1], xi_host[l] + (size_t)n0 * M, S0 + off_sc[l] + (size_t)n0 * ec,
                                 n1 - n0, ec, M, c->p.sigma_f0, mixed, additive, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "kl launch");
      }
    }
    if ((st = timed_end(c, &c->tm.kl_ms))) return st;
    // 2) one persistent launch over all groups
    std::vector<Group> gs;
    for (int l = 0; l < L1; ++l) {
      if (Ntarget[l] <= Ndone[l]) continue;
      for (int cm = 0; cm < (l > 0 ? 2 : 1); ++cm) {
        Group g;
        g.grid = cm ? l - 1 : l;
        g.mlmc_level = l;
        g.coarse = cm == 1;
        g.n0 = Ndone[l];
        g.n1 = Ntarget[l];
        g.lanes = 0;
        g.G = 1;
        g.gmax = max_team(c, g.grid);
        team_times(c, g.grid, g.gmax, g.t);
        gs.push_back(g);
      }
    }
    // Solve times within the finest level's fine member vary with the field:
    // samples whose conductivity has the smallest minimum need the most
    // Krylov iterations, and with one sample per team the slowest decides the
    // launch.  The eighth with the smallest minimum becomes a group of its
    // own, priced at hard_ratio times the others (the ratio of its slowest
    // sample, measured), so that the allocation can give it larger teams; the
    // others are priced at their own measured slowest-to-mean tail_ratio.
    std::vector<int> order;
    for (size_t gi = 0; gi < gs.size(); ++gi) {
      const int N = gs[gi].n1 - gs[gi].n0;
      if (gs[gi].coarse || gs[gi].mlmc_level != L1 - 1 || N < 8 || gs[gi].gmax < 2) continue;
      const int ef = c->levels[gs[gi].grid].dev.g[0].ne;
      if ((st = grow(c, &c->d_rowmin, &c->rowmin_cap, (size_t)N * sizeof(double)))) return st;
      hipError_t e = launch_row_min(S0 + off_sf[gs[gi].mlmc_level] + (size_t)gs[gi].n0 * ef, N, ef, c->d_rowmin,
                                    c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "row min launch");
      std::vector<double> mins(N);
      STM_HIP(c, hipMemcpyAsync(mins.data(), c->d_rowmin, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      STM_HIP(c, hipStreamSynchronize(c->stream));
      std::vector<int> idx(N);
      for (int i = 0; i < N; ++i) idx[i] = i;
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return mins[a] < mins[b]; });
      const int k = std::max(1, N / 8);
      const int base = (int)order.size();
      for (int i = 0; i < N; ++i) order.push_back(gs[gi].n0 + idx[i]);
      Group h = gs[gi];
      h.ordered = true;
      h.hard = true;
      h.o0 = base;
      h.o1 = base + k;
      for (int G = 1; G <= h.gmax; ++G) h.t[G] = gs[gi].t[G] * c->hard_ratio[gs[gi].grid];
      for (int G = 1; G <= gs[gi].gmax; ++G) gs[gi].t[G] *= c->tail_ratio[gs[gi].grid];
      gs[gi].ordered = true;
      gs[gi].o0 = base + k;
      gs[gi].o1 = base + N;
      gs.push_back(h);
      break;
    }
    if (!order.empty()) {
      if ((st = grow(c, &c->d_order, &c->order_cap, order.size() * sizeof(int)))) return st;
      STM_HIP(c, hipMemcpyAsync(c->d_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice,
                                c->stream));
    }
    int block = 256;
    for (auto& g : gs) block = std::max(block, auto_block(c->p, c->levels[g.grid].dev.g[0].n, c->any_mg));
    allocate_lanes(gs, std::min(lane_budget, block_capacity(c, block)));
    size_t ws = 0;
    for (auto& g : gs) ws += (size_t)g.lanes * (c->levels[g.grid].team_bytes + c->levels[g.grid].u_bytes);
    if ((st = grow(c, &c->work, &c->work_bytes, ws))) return st;
    std::vector<TeamTask> tasks;
    size_t woff = 0;
    for (auto& g : gs) {
      const LevelHost& LH = c->levels[g.grid];
      const int l = g.mlmc_level;
      const int N = group_count(g);
      for (int i = 0; i < g.lanes; ++i) {
        TeamTask t{};
        t.G = g.G;
        t.level = g.grid;
        t.order = g.ordered ? c->d_order : nullptr;
        t.first = (g.ordered ? g.o0 : g.n0) + i;
        t.stride = g.lanes;
        t.count = (N - i + g.lanes - 1) / g.lanes;
        t.sigma = S0 + (g.coarse ? off_sc[l] : off_sf[l]);
        t.u_out = st_qoi ? S0 + (g.coarse ? off_uc[l] : off_uf[l]) : nullptr;
        t.u_guess = nullptr;
        t.t_act = S0 + (g.coarse ? off_tc[l] : off_tf[l]);
        t.work = static_cast<unsigned char*>(c->work) + woff;
        t.stats = c->d_stats + (g.coarse ? off_stc[l] : off_stf[l]);
        woff += LH.team_bytes + LH.u_bytes;
        tasks.push_back(t);
      }
    }
    if ((st = run_tasks(c, tasks, block))) return st;
    // measured seconds per sample of each grid at the team sizes used (the
    // cost model of later calls)
    {
      std::vector<SampleStatsDev> tmp(nst);
      STM_HIP(c, hipMemcpy(tmp.data(), c->d_stats, nst * sizeof(SampleStatsDev), hipMemcpyDeviceToHost));
      std::vector<double> acc(L1 * (kMaxTeam + 1), 0.0), cnt(L1 * (kMaxTeam + 1), 0.0);
      auto sample_of = [&](const Group& g, int j) { return g.ordered ? order[g.o0 + j] : g.n0 + j; };
      auto mean_seconds = [&](const Group& g) {
        const size_t base = g.coarse ? off_stc[g.mlmc_level] : off_stf[g.mlmc_level];
        double s = 0.0;
        for (int j = 0; j < group_count(g); ++j) s += tmp[base + sample_of(g, j)].ticks * 1e-8;
        return s / std::max(1, group_count(g));
      };
      for (auto& g : gs) {
        if (g.hard) continue;  // the hard part informs hard_ratio, not the grid's table
        const size_t base = g.coarse ? off_stc[g.mlmc_level] : off_stf[g.mlmc_level];
        for (int j = 0; j < group_count(g); ++j) {
          acc[g.grid * (kMaxTeam + 1) + g.G] += tmp[base + sample_of(g, j)].ticks * 1e-8;
          cnt[g.grid * (kMaxTeam + 1) + g.G] += 1.0;
        }
      }
      // hard_ratio: the slowest hard sample (it decides when its team ends)
      // and the normal part's mean, each relative to the model of the normal
      // samples at the team size it ran with
      auto max_seconds = [&](const Group& g) {
        const size_t base = g.coarse ? off_stc[g.mlmc_level] : off_stf[g.mlmc_level];
        double s = 0.0;
        for (int j = 0; j < group_count(g); ++j) s = std::max(s, tmp[base + sample_of(g, j)].ticks * 1e-8);
        return s;
      };
      for (auto& h : gs) {
        if (!h.hard || h.lanes == 0 || group_count(h) == 0) continue;
        for (auto& g : gs) {
          if (g.hard || !g.ordered || g.grid != h.grid || g.mlmc_level != h.mlmc_level || g.coarse != h.coarse) continue;
          if (g.lanes == 0 || group_count(g) == 0) break;
          // g.t carries this launch's tail factor: divide it out to compare with the mean model
          const double tail = c->tail_ratio[g.grid];
          const double rh = max_seconds(h) / (g.t[h.G] / tail), rn = mean_seconds(g) / (g.t[g.G] / tail);
          if (rh > 0 && rn > 0) c->hard_ratio[h.grid] = std::min(3.0, std::max(1.0, rh / rn));
          const double mn = mean_seconds(g);
          if (mn > 0) c->tail_ratio[g.grid] = std::min(2.0, std::max(1.0, max_seconds(g) / mn));
          break;
        }
      }
      for (int l = 0; l < L1; ++l)
        for (int G = 1; G <= kMaxTeam; ++G)
          if (cnt[l * (kMaxTeam + 1) + G] > 0)
            c->tsec[l][G] = acc[l * (kMaxTeam + 1) + G] / cnt[l * (kMaxTeam + 1) + G];
    }
    for (int l = 0; l < L1; ++l) Ndone[l] = std::max(Ndone[l], Ntarget[l]);
    // 3) statistics over all samples so far
    if (out->level_mean == nullptr || out->level_var == nullptr) {
      // level fields are still needed internally only as scalars
    }
    if ((st = timed_begin(c))) return st;
    hipError_t e = launch_fill(out->mean, 0.0, (int64_t)P, c->stream);
    if (e == hipSuccess) e = launch_fill(out->var, 0.0, (int64_t)P, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "fill");
    std::vector<double> vpart(vpart_sz);
    double vol = c->p.lx * c->p.ly * (c->p.dim == 3 ? c->p.lz : 1.0) * (st_qoi ? c->p.T : 1.0);
    for (int l = 0; l < L1; ++l) {
      StatsLevelArgs a{};
      a.gf = c->levels[l].dev.g[0];
      a.gc = l > 0 ? c->levels[l - 1].dev.g[0] : a.gf;
      a.gL = dL.g[0];
      a.dim = c->p.dim;
      a.tf = S0 + off_tf[l];
      a.tc = l > 0 ? S0 + off_tc[l] : nullptr;
      a.N = Ndone[l];
      a.chunk = chunk;
      a.part = S0 + off_part;
      a.mean = out->mean;
      a.var = out->var;
      a.level_mean = out->level_mean ? out->level_mean + (size_t)l * P : nullptr;
      a.level_var = out->level_var ? out->level_var + (size_t)l * P : nullptr;
      a.vpart = S0 + off_vpart;
      if (st_qoi) {
        a.tf = S0 + off_uf[l];
        a.tc = l > 0 ? S0 + off_uc[l] : nullptr;
        a.mf = c->levels[l].dev.m;
        a.mc = l > 0 ? c->levels[l - 1].dev.m : 0;
        a.mL = dL.m;
        a.dtL = dL.dt;
        a.u0f = c->levels[l].dev.u0;
        a.u0c = l > 0 ? c->levels[l - 1].dev.u0 : nullptr;
      }
      e = launch_level_stats(a, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "stats launch");
      if (l == L1 - 1) {
        if ((st = timed_end(c, &c->tm.stats_ms))) return st;
      }
      STM_HIP(c, hipMemcpyAsync(vpart.data(), S0 + off_vpart, vpart_sz * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
      STM_HIP(c, hipStreamSynchronize(c->stream));
      double sum = 0.0;
      for (double v : vpart) sum += v;
      V[l] = sum / vol;
    }
    // per-level mean norms for the bias estimate
    if (out->level_mean) {
      std::vector<double> lm(P);
      for (int l = 0; l < L1; ++l) {
        STM_HIP(c, hipMemcpy(lm.data(), out->level_mean + (size_t)l * P, P * sizeof(double), hipMemcpyDeviceToHost));
        double s2 = 0.0;
        for (double v : lm) s2 += v * v;
        level_norm[l] = std::sqrt(s2 / (double)P);
      }
    }
    STM_HIP(c, hipMemcpy(sh.data(), c->d_stats, nst * sizeof(SampleStatsDev), hipMemcpyDeviceToHost));
    for (int l = 0; l < L1; ++l) {  // workgroup-seconds per sample pair of the level
      double tf[kMaxTeam + 1], tc[kMaxTeam + 1];
      team_times(c, l, 1, tf);
      if (l > 0) team_times(c, l - 1, 1, tc);
      cost[l] = tf[1] + (l > 0 ? tc[1] : 0.0);
    }
    if (!adaptive) break;
    // 4) Giles allocation: N_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k))
    double ssum = 0.0;
    for (int l = 0; l < L1; ++l) ssum += std::sqrt(std::max(V[l], 0.0) * cost[l]);
    bool grow_any = false;
    for (int l = 0; l < L1; ++l) {
      const double Vl = std::max(V[l], 0.0);
      int want = (int)std::ceil(2.0 / (target_rmse * target_rmse) * std::sqrt(Vl / std::max(cost[l], 1e-12)) * ssum);
      want = std::max(want, Ndone[l]);
      want = std::min(want, cap[l]);
      Ntarget[l] = want;
      if (want > Ndone[l]) grow_any = true;
    }
    if (!grow_any || rounds >= 20) break;
  }
  // summarise
  out->rounds = rounds;
  out->newton_iters = 0;
  out->krylov_iters = 0;
  out->censored = 0;
  out->algorithmic_bytes = 0.0;
  out->model_bytes = 0.0;
  out->dof_steps = 0;
  for (int l = 0; l < L1; ++l) {
    out->N[l] = Ndone[l];
    out->V[l] = V[l];
    out->cost[l] = cost[l];
    for (int cm = 0; cm < (l > 0 ? 2 : 1); ++cm) {
      const size_t base = cm ? off_stc[l] : off_stf[l];
      for (int i = 0; i < Ndone[l]; ++i) {
        const SampleStatsDev& s = sh[base + i];
        out->newton_iters += s.newton_iters;
        out->krylov_iters += s.krylov_iters;
        out->censored += s.censored;
        out->algorithmic_bytes += s.alg_bytes;
        out->model_bytes += s.model_bytes;
        worst = std::min(worst, s.status);
      }
      const LevelDev& dg = c->levels[cm ? l - 1 : l].dev;
      out->dof_steps += (int64_t)Ndone[l] * dg.g[0].n * dg.m;
    }
  }
  // bias estimate from the decay of the level corrections
  out->bias_estimate = 0.0;
  if (L1 >= 3 && level_norm[L1 - 1] > 0 && level_norm[L1 - 2] > 0) {
    double alpha = std::log2(level_norm[L1 - 2] / level_norm[L1 - 1]);
    if (alpha > 0.1) out->bias_estimate = level_norm[L1 - 1] / (std::pow(2.0, alpha) - 1.0);
  }
  out->worst_status = worst;
  c->tm.solve_bytes = out->algorithmic_bytes;
  c->tm.solve_bytes_model = out->model_bytes;
  if (worst == STM_E_NONFINITE) return fail(c, STM_E_NONFINITE, "non-finite residual in a sample");
  if (worst == STM_E_NOT_CONVERGED) return fail(c, STM_E_NOT_CONVERGED, "Newton iteration limit reached in a sample");
  return STM_OK;
}
