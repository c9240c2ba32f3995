// KL synthesis on the matrix cores: the only dense contraction of the method.
//
//   g[s][e] = sum_k xi[s][k] * modes[e][k],   sigma[s][e] = sigma_f0 * exp(g[s][e])
//
// (Sec. 2.2, eq. KL-expansion; lognormal form.)  A = xi (S x M), B = modes^T
// (M x E), C = g (S x E).  Each wave owns a 16 x 64 output tile (four 16 x 16
// MFMA accumulators) and walks K = M.  The exponential is fused into the
// epilogue; the float64 result is written once.
//
// Two operand paths:
//  * float64: v_mfma_f64_16x16x4f64, exact float64 arithmetic.
//  * split fp16: every operand x is split into hi = fp16(x) and
//    lo = fp16((x - hi) * 2^11); with fp32 accumulation
//    g = hi_a.hi_b + 2^-11 (hi_a.lo_b + lo_a.hi_b), dropping the 2^-22 lo.lo
//    term (three v_mfma_f32_16x16x16f16 per K-step of 16).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "stm_launch.h"

namespace stm {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

constexpr int KL_TILE_E = 64;  // output columns per wave
constexpr int KL_WAVES = 4;    // waves per block, stacked along s

// Lane layout of the 16x16 MFMA tiles used here (CDNA3/CDNA4):
//  f64 16x16x4 : A[i][k] at lane i + 16 k; B[k][j] at lane j + 16 k;
//                D[(l/16) + 4 r][l % 16] in accumulator register r (rows interleaved).
//  f16 16x16x16: A[i][4 (l/16) + v] in element v of lane l with i = l % 16;
//                B[4 (l/16) + v][j] likewise with j = l % 16;
//                D[4 (l/16) + r][l % 16] in accumulator register r.
__global__ __launch_bounds__(64 * KL_WAVES) void kl_f64_kernel(const double* __restrict__ modes,
                                                               const double* __restrict__ xi,
                                                               double* __restrict__ sigma, int S, int E, int M,
                                                               double sigma_f0) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int s0 = (blockIdx.y * KL_WAVES + wave) * 16;
  const int e0 = blockIdx.x * KL_TILE_E;
  if (s0 >= S) return;
  const int li = lane & 15, lk = lane >> 4;
  double4_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = double4_t{0.0, 0.0, 0.0, 0.0};
  const int srow = s0 + li;
  for (int k0 = 0; k0 < M; k0 += 4) {
    const int k = k0 + lk;
    const double a = (srow < S && k < M) ? xi[(int64_t)srow * M + k] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = e0 + 16 * t + li;
      const double b = (e < E && k < M) ? modes[(int64_t)e * M + k] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = e0 + 16 * t + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int s = s0 + lk + 4 * r;
      if (s < S && e < E) sigma[(int64_t)s * E + e] = sigma_f0 * exp(acc[t][r]);
    }
  }
}

__device__ __forceinline__ void split_h(double x, _Float16& hi, _Float16& lo) {
  hi = (_Float16)x;
  lo = (_Float16)((x - (double)hi) * 2048.0);
}

__global__ __launch_bounds__(64 * KL_WAVES) void kl_f16x3_kernel(const double* __restrict__ modes,
                                                                 const double* __restrict__ xi,
                                                                 double* __restrict__ sigma, int S, int E, int M,
                                                                 double sigma_f0) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int s0 = (blockIdx.y * KL_WAVES + wave) * 16;
  const int e0 = blockIdx.x * KL_TILE_E;
  if (s0 >= S) return;
  const int li = lane & 15, lk = lane >> 4;
  float4_t acc_hh[4], acc_x[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    acc_hh[t] = float4_t{0.f, 0.f, 0.f, 0.f};
    acc_x[t] = float4_t{0.f, 0.f, 0.f, 0.f};
  }
  const int srow = s0 + li;
  for (int k0 = 0; k0 < M; k0 += 16) {
    half4_t ahi, alo;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + 4 * lk + v;
      const double a = (srow < S && k < M) ? xi[(int64_t)srow * M + k] : 0.0;
      _Float16 h, l;
      split_h(a, h, l);
      ahi[v] = h;
      alo[v] = l;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = e0 + 16 * t + li;
      half4_t bhi, blo;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = k0 + 4 * lk + v;
        const double b = (e < E && k < M) ? modes[(int64_t)e * M + k] : 0.0;
        _Float16 h, l;
        split_h(b, h, l);
        bhi[v] = h;
        blo[v] = l;
      }
      acc_hh[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ahi, bhi, acc_hh[t], 0, 0, 0);
      acc_x[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ahi, blo, acc_x[t], 0, 0, 0);
      acc_x[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(alo, bhi, acc_x[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = e0 + 16 * t + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int s = s0 + 4 * lk + r;
      const float g = acc_hh[t][r] + acc_x[t][r] * (1.0f / 2048.0f);
      if (s < S && e < E) sigma[(int64_t)s * E + e] = sigma_f0 * (double)expf(g);
    }
  }
}

hipError_t launch_kl_synthesize(const double* modes, const double* xi, double* sigma, int S, int E, int M,
                                double sigma_f0, bool split_fp16, hipStream_t st) {
  if (S <= 0 || E <= 0) return hipSuccess;
  dim3 grid((E + KL_TILE_E - 1) / KL_TILE_E, (S + 16 * KL_WAVES - 1) / (16 * KL_WAVES));
  dim3 block(64 * KL_WAVES);
  if (split_fp16)
    hipLaunchKernelGGL(kl_f16x3_kernel, grid, block, 0, st, modes, xi, sigma, S, E, M, sigma_f0);
  else
    hipLaunchKernelGGL(kl_f64_kernel, grid, block, 0, st, modes, xi, sigma, S, E, M, sigma_f0);
  return hipGetLastError();
}

}  // namespace stm
