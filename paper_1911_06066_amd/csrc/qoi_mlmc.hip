// Activation map and MLMC statistics kernels (float64).
//
// Activation time of a node: 0 if the initial state is at or above the
// threshold, else the first up-crossing in time located by linear
// interpolation between the bracketing time levels, else T (censored).
//
// MLMC statistics (Sec. 3.1.2, eq. MLMC-estimator): each level's activation
// maps are interpolated (nested Q1) to the finest grid; per finest node, the
// samples of P Q_l, P Q_{l-1} and Y_l = P Q_l - P Q_{l-1} are reduced by
// Welford updates over fixed chunks of samples and the chunk states merged in
// chunk order (Chan et al.), so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "stm_launch.h"

namespace stm {

__global__ void activation_kernel(GridDev g, int m, double dt, double T, double thr,
                                  const double* __restrict__ u0, const double* __restrict__ u, int S,
                                  double* __restrict__ t_act, int* __restrict__ censored) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  int cen = 0;
  if (i < g.n) {
    double prev = u0[i];
    double t = -1.0;
    if (prev >= thr) {
      t = 0.0;
    } else {
      const double* us = u + (int64_t)s * m * g.n + i;
      for (int k = 0; k < m; ++k) {
        const double cur = us[(int64_t)k * g.n];
        if (cur >= thr) {
          t = k * dt + dt * (thr - prev) / (cur - prev);
          break;
        }
        prev = cur;
      }
    }
    if (t < 0.0) {
      t = T;
      cen = 1;
    }
    t_act[(int64_t)s * g.n + i] = t;
  }
  // per-block count, then one integer atomic per block (exact)
  __shared__ int sc[256];
  sc[threadIdx.x] = cen;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sc[threadIdx.x] += sc[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && censored && sc[0]) atomicAdd(censored + s, sc[0]);
}

hipError_t launch_activation_map(const GridDev& g, int m, double dt, double T, double thr, const double* u0,
                                 const double* u, int S, double* t_act, int* censored_dev, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  dim3 grid((g.n + 255) / 256, S);
  hipLaunchKernelGGL(activation_kernel, grid, dim3(256), 0, st, g, m, dt, T, thr, u0, u, S, t_act,
                     censored_dev);
  return hipGetLastError();
}

__global__ void fill_kernel(double* p, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_u32_kernel(unsigned* p, unsigned v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// out[s] = min_e a[s][e]: one block per row
__global__ void row_min_kernel(const double* __restrict__ a, int E, double* __restrict__ out) {
  __shared__ double sh[256];
  const double* r = a + (int64_t)blockIdx.x * E;
  double v = 1.0e300;
  for (int e = threadIdx.x; e < E; e += 256) v = fmin(v, r[e]);
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

hipError_t launch_row_min(const double* a, int S, int E, double* out, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_min_kernel, dim3(S), dim3(256), 0, st, a, E, out);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, unsigned v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

// Q1 interpolation of a field on grid gc (nested in gL, ratio 2^r per axis) at finest node p.
__device__ __forceinline__ double interp_nested(const GridDev& gc, const GridDev& gL, int dim, const double* f,
                                                int p) {
  const int rx = (gL.nx - 1) / (gc.nx - 1);
  const int ry = (gL.ny - 1) / (gc.ny - 1);
  const int rz = (dim == 3) ? (gL.nz - 1) / (gc.nz - 1) : 1;
  const int ix = p % gL.nx;
  const int r = p / gL.nx;
  const int iy = (dim == 2) ? r : r % gL.ny;
  const int iz = (dim == 2) ? 0 : r / gL.ny;
  const int I = ix / rx, J = iy / ry, K = iz / rz;
  const double fx = double(ix - I * rx) / rx, fy = double(iy - J * ry) / ry, fz = double(iz - K * rz) / rz;
  double acc = 0.0;
  for (int c = 0; c < (dim == 3 ? 2 : 1); ++c) {
    const double wz = (dim == 3) ? (c ? fz : 1.0 - fz) : 1.0;
    if (wz == 0.0) continue;
    for (int b = 0; b < 2; ++b) {
      const double wy = b ? fy : 1.0 - fy;
      if (wy == 0.0) continue;
      for (int a = 0; a < 2; ++a) {
        const double wx = a ? fx : 1.0 - fx;
        if (wx == 0.0) continue;
        const int q = (dim == 3) ? (((K + c) * gc.ny + (J + b)) * gc.nx + (I + a)) : ((J + b) * gc.nx + (I + a));
        acc += wx * wy * wz * f[q];
      }
    }
  }
  return acc;
}

// Space-time prolongation (Sec. 3.4): fine time level k + 1 (t = (k + 1) dt_f)
// sits at j + w = (k + 1) mc / mf coarse steps; blend the space-interpolated
// coarse levels j and j + 1, coarse level 0 being the fine initial state.
__global__ void prolong_st_kernel(GridDev gc, GridDev gf, int dim, int mc, int mf, const double* __restrict__ u0f,
                                  const double* __restrict__ u_c, double* __restrict__ u_f) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;  // fine time level k + 1
  const int s = blockIdx.z;
  if (p >= gf.n) return;
  const int64_t num = (int64_t)(k + 1) * mc;
  const int j = (int)(num / mf);
  const double w = double(num % mf) / mf;
  const double* uc = u_c + (int64_t)s * mc * gc.n;
  const double a = (j == 0) ? u0f[p] : interp_nested(gc, gf, dim, uc + (int64_t)(j - 1) * gc.n, p);
  const double b = (w > 0.0) ? interp_nested(gc, gf, dim, uc + (int64_t)j * gc.n, p) : 0.0;
  u_f[((int64_t)s * mf + k) * gf.n + p] = (1.0 - w) * a + w * b;
}

hipError_t launch_prolong_st(const GridDev& gc, const GridDev& gf, int dim, int mc, int mf, const double* u0f,
                             const double* u_c, int S, double* u_f, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(prolong_st_kernel, dim3((gf.n + 255) / 256, mf, S), dim3(256), 0, st, gc, gf, dim, mc, mf, u0f,
                     u_c, u_f);
  return hipGetLastError();
}

// Number of QoI points: the finest nodes, or the finest space-time points.
__device__ __host__ __forceinline__ int64_t qoi_points(const StatsLevelArgs& a) {
  return a.mL ? (int64_t)a.mL * a.gL.n : (int64_t)a.gL.n;
}

// Sample s of a level's QoI at QoI point q: the nested Q1 interpolant of its
// activation map, or of its space-time solution at finest time level k + 1
// (q = k n_L + p), linear in time between the level's bracketing time levels,
// time level 0 being the level's initial state.
__device__ __forceinline__ double qoi_value(const StatsLevelArgs& a, const GridDev& g, int m, const double* f,
                                            const double* u0, int s, int q) {
  if (a.mL == 0) return interp_nested(g, a.gL, a.dim, f + (int64_t)s * g.n, q);
  const int p = q % a.gL.n, k = q / a.gL.n;
  const int64_t num = (int64_t)(k + 1) * m;
  const int j = (int)(num / a.mL);
  const double w = double(num % a.mL) / a.mL;
  const double* us = f + (int64_t)s * m * g.n;
  const double lo = interp_nested(g, a.gL, a.dim, j == 0 ? u0 : us + (int64_t)(j - 1) * g.n, p);
  const double hi = (w > 0.0) ? interp_nested(g, a.gL, a.dim, us + (int64_t)j * g.n, p) : 0.0;
  return (1.0 - w) * lo + w * hi;
}

// Pass 1: Welford over each chunk of samples. part[c][0..5][p]: mean_f, M2_f, mean_c, M2_c, mean_y, M2_y.
__global__ void level_chunk_kernel(StatsLevelArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (p >= qoi_points(a)) return;
  const int s0 = c * a.chunk, s1 = min(a.N, s0 + a.chunk);
  double mf = 0, qf2 = 0, mc = 0, qc2 = 0, my = 0, qy2 = 0;
  int cnt = 0;
  for (int s = s0; s < s1; ++s) {
    const double vf = qoi_value(a, a.gf, a.mf, a.tf, a.u0f, s, p);
    const double vc = a.tc ? qoi_value(a, a.gc, a.mc, a.tc, a.u0c, s, p) : 0.0;
    const double vy = vf - vc;
    ++cnt;
    double d = vf - mf; mf += d / cnt; qf2 += d * (vf - mf);
    d = vc - mc; mc += d / cnt; qc2 += d * (vc - mc);
    d = vy - my; my += d / cnt; qy2 += d * (vy - my);
  }
  const int64_t n = qoi_points(a);
  double* q = a.part + (int64_t)c * 6 * n + p;
  q[0] = mf; q[n] = qf2; q[2 * n] = mc; q[3 * n] = qc2; q[4 * n] = my; q[5 * n] = qy2;
}

// Pass 2: merge the chunk states in order, accumulate the MLMC mean/variance,
// write the level fields, and per-block partial sums of w_p s^2(Y_l)(p).
__global__ void level_merge_kernel(StatsLevelArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = qoi_points(a);
  double contrib = 0.0;
  if (p < n) {
    const int nch = (a.N + a.chunk - 1) / a.chunk;
    double cnt = 0, mf = 0, qf2 = 0, mc = 0, qc2 = 0, my = 0, qy2 = 0;
    for (int c = 0; c < nch; ++c) {
      const double nb = (double)(min(a.N, (c + 1) * a.chunk) - c * a.chunk);
      const double* q = a.part + (int64_t)c * 6 * n + p;
      const double tot = cnt + nb;
      double d = q[0] - mf; mf += d * nb / tot; qf2 += q[n] + d * d * cnt * nb / tot;
      d = q[2 * n] - mc; mc += d * nb / tot; qc2 += q[3 * n] + d * d * cnt * nb / tot;
      d = q[4 * n] - my; my += d * nb / tot; qy2 += q[5 * n] + d * d * cnt * nb / tot;
      cnt = tot;
    }
    const double den = a.N > 1 ? 1.0 / (a.N - 1) : 0.0;
    const double vf = qf2 * den, vc = qc2 * den, vy = qy2 * den;
    a.mean[p] += my;
    a.var[p] += vf - (a.tc ? vc : 0.0);
    if (a.level_mean) a.level_mean[p] = my;
    if (a.level_var) a.level_var[p] = vy;
    // lumped (trapezoid) weight of the finest node, times the trapezoid
    // weight in time of the space-time point (the t = 0 level has no variance)
    const int pn = a.mL ? p % a.gL.n : p;
    const int ix = pn % a.gL.nx;
    const int r = pn / a.gL.nx;
    const int iy = (a.dim == 2) ? r : r % a.gL.ny;
    const int iz = (a.dim == 2) ? 0 : r / a.gL.ny;
    double w = a.gL.hx * a.gL.hy * ((ix == 0 || ix == a.gL.nx - 1) ? 0.5 : 1.0) *
               ((iy == 0 || iy == a.gL.ny - 1) ? 0.5 : 1.0);
    if (a.dim == 3) w *= a.gL.hz * ((iz == 0 || iz == a.gL.nz - 1) ? 0.5 : 1.0);
    if (a.mL) w *= (p / a.gL.n == a.mL - 1) ? 0.5 * a.dtL : a.dtL;
    contrib = w * vy;
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = contrib;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.vpart[blockIdx.x] = sh[0];
}

hipError_t launch_level_stats(const StatsLevelArgs& a, hipStream_t st) {
  if (a.N <= 0) return hipErrorInvalidValue;
  const int nch = (a.N + a.chunk - 1) / a.chunk;
  const int64_t P = qoi_points(a);
  if (P >= ((int64_t)1 << 31) - 256) return hipErrorInvalidValue;
  dim3 g1((unsigned)((P + 255) / 256), nch);
  hipLaunchKernelGGL(level_chunk_kernel, g1, dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(level_merge_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace stm
