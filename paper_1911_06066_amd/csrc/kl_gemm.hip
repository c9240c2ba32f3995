// KL synthesis on the matrix cores: the only dense contraction of the method.
//
//   g[s][e] = sum_k xi[s][k] * modes[e][k],   sigma[s][e] = sigma_f0 * exp(g[s][e])
//
// (Sec. 2.2, eq. KL-expansion; lognormal form.)  A = xi (S x M), B = modes^T
// (M x E), C = g (S x E).  A block of 4 waves owns a 64 x 64 output tile
// (16 sample rows per wave, four 16 x 16 MFMA accumulators each) and walks
// K = M in chunks of 32: the chunk's 64 x 32 panels of xi and modes are loaded
// with coalesced row reads into LDS (split into fp16 halves once, on the way
// in, for the split path), then fed to the matrix cores.  The
// exponential is fused into the epilogue; the float64 result is written once.
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

constexpr int KL_TILE_E = 64;  // output columns per block
constexpr int KL_WAVES = 4;    // waves per block, stacked along s (16 rows each)
constexpr int KL_TILE_S = 16 * KL_WAVES;
constexpr int KL_KC = 32;      // K chunk staged in LDS
constexpr int KL_LD = KL_KC + 4;  // LDS row stride in doubles (padding spreads the banks)

// Lane layout of the 16x16 MFMA tiles used here (CDNA3/CDNA4):
//  f64 16x16x4 : A[i][k] at lane i + 16 k; B[k][j] at lane j + 16 k;
//                D[(l/16) + 4 r][l % 16] in accumulator register r (rows interleaved).
//  f16 16x16x16: A[i][4 (l/16) + v] in element v of lane l with i = l % 16;
//                B[4 (l/16) + v][j] likewise with j = l % 16;
//                D[4 (l/16) + r][l % 16] in accumulator register r.

// rows [r0, r0 + 64) x columns [k0, k0 + KL_KC) of a row-major (rows x M)
// matrix into LDS, zero outside; consecutive threads read consecutive columns
__device__ __forceinline__ void kl_stage(const double* __restrict__ g, int rows, int M, int r0, int k0,
                                         double (*lds)[KL_LD]) {
#pragma unroll
  for (int u = 0; u < (64 * KL_KC) / (64 * KL_WAVES); ++u) {
    const int q = threadIdx.x + u * 64 * KL_WAVES;
    const int r = q / KL_KC, c = q % KL_KC;
    const int gr = r0 + r, gc = k0 + c;
    lds[r][c] = (gr < rows && gc < M) ? g[(int64_t)gr * M + gc] : 0.0;
  }
}

__global__ __launch_bounds__(64 * KL_WAVES) void kl_f64_kernel(const double* __restrict__ modes,
                                                               const double* __restrict__ xi,
                                                               double* __restrict__ sigma, int S, int E, int M,
                                                               double sigma_f0) {
  __shared__ double As[KL_TILE_S][KL_LD], Bs[KL_TILE_E][KL_LD];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int e0 = blockIdx.x * KL_TILE_E;
  const int sb = blockIdx.y * KL_TILE_S;
  const int li = lane & 15, lk = lane >> 4;
  double4_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = double4_t{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < M; k0 += KL_KC) {
    kl_stage(xi, S, M, sb, k0, As);
    kl_stage(modes, E, M, e0, k0, Bs);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KL_KC; kk += 4) {
      const double a = As[wave * 16 + li][kk + lk];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[16 * t + li][kk + lk], acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
  const int s0 = sb + wave * 16;
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

constexpr int KL_LDH = KL_KC + 8;  // half-precision LDS row stride (keeps half4 rows 8-byte aligned)

// As kl_stage, each value split once into its hi and lo halves
__device__ __forceinline__ void kl_stage_split(const double* __restrict__ g, int rows, int M, int r0, int k0,
                                               _Float16 (*hi)[KL_LDH], _Float16 (*lo)[KL_LDH]) {
#pragma unroll
  for (int u = 0; u < (64 * KL_KC) / (64 * KL_WAVES); ++u) {
    const int q = threadIdx.x + u * 64 * KL_WAVES;
    const int r = q / KL_KC, c = q % KL_KC;
    const int gr = r0 + r, gc = k0 + c;
    _Float16 h, l;
    split_h((gr < rows && gc < M) ? g[(int64_t)gr * M + gc] : 0.0, h, l);
    hi[r][c] = h;
    lo[r][c] = l;
  }
}

__global__ __launch_bounds__(64 * KL_WAVES) void kl_f16x3_kernel(const double* __restrict__ modes,
                                                                 const double* __restrict__ xi,
                                                                 double* __restrict__ sigma, int S, int E, int M,
                                                                 double sigma_f0) {
  __shared__ __attribute__((aligned(16))) _Float16 Ah[KL_TILE_S][KL_LDH], Al[KL_TILE_S][KL_LDH];
  __shared__ __attribute__((aligned(16))) _Float16 Bh[KL_TILE_E][KL_LDH], Bl[KL_TILE_E][KL_LDH];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int e0 = blockIdx.x * KL_TILE_E;
  const int sb = blockIdx.y * KL_TILE_S;
  const int li = lane & 15, lk = lane >> 4;
  float4_t acc_hh[4], acc_x[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    acc_hh[t] = float4_t{0.f, 0.f, 0.f, 0.f};
    acc_x[t] = float4_t{0.f, 0.f, 0.f, 0.f};
  }
  for (int k0 = 0; k0 < M; k0 += KL_KC) {
    kl_stage_split(xi, S, M, sb, k0, Ah, Al);
    kl_stage_split(modes, E, M, e0, k0, Bh, Bl);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KL_KC; kk += 16) {
      const int kc = kk + 4 * lk;
      const half4_t ahi = *reinterpret_cast<const half4_t*>(&Ah[wave * 16 + li][kc]);
      const half4_t alo = *reinterpret_cast<const half4_t*>(&Al[wave * 16 + li][kc]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const half4_t bhi = *reinterpret_cast<const half4_t*>(&Bh[16 * t + li][kc]);
        const half4_t blo = *reinterpret_cast<const half4_t*>(&Bl[16 * t + li][kc]);
        acc_hh[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ahi, bhi, acc_hh[t], 0, 0, 0);
        acc_x[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ahi, blo, acc_x[t], 0, 0, 0);
        acc_x[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(alo, bhi, acc_x[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int s0 = sb + wave * 16;
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
  dim3 grid((E + KL_TILE_E - 1) / KL_TILE_E, (S + KL_TILE_S - 1) / KL_TILE_S);
  dim3 block(64 * KL_WAVES);
  if (split_fp16)
    hipLaunchKernelGGL(kl_f16x3_kernel, grid, block, 0, st, modes, xi, sigma, S, E, M, sigma_f0);
  else
    hipLaunchKernelGGL(kl_f64_kernel, grid, block, 0, st, modes, xi, sigma, S, E, M, sigma_f0);
  return hipGetLastError();
}

}  // namespace stm
