// KL synthesis on the matrix cores: the only dense contraction of the method.
//
//   g[s][e] = sum_k xi[s][k] * modes[e][k],   sigma[s][e] = sigma_f0 * exp(g[s][e])
//
// (Sec. 2.2, eq. KL-expansion; lognormal form.)  A = xi (S x M), B = modes^T
// (M x E), C = g (S x E).  The output is cut into 64 x 64 tiles (16 sample
// rows per wave, four 16 x 16 MFMA accumulators each), numbered sample-tile
// fastest; a block of 4 waves takes a contiguous run of tiles, so the modes
// panel of an element tile is reused from its XCD's L2 across sample tiles.
// A block walks (tile, K chunk) steps as a software pipeline: the next
// chunk's 64 x KC panels of xi and modes are read (coalesced rows) into
// registers while the matrix cores work on the current chunk from one of two
// LDS buffers, so one barrier per step suffices.  The split path splits each
// value into its fp16 halves once, when it is written to LDS.  The exponential
// (1 + g for the additive field) is fused into the epilogue; the float64
// result is written once.
//
// Two operand paths:
//  * float64: v_mfma_f64_16x16x4f64, exact float64 arithmetic.
//  * split fp16: every operand x is split into hi = fp16(x) and
//    lo = fp16((x - hi) * 2^11); with fp32 accumulation
//    g = hi_a.hi_b + 2^-11 (hi_a.lo_b + lo_a.hi_b), dropping the 2^-22 lo.lo
//    term (three v_mfma_f32_16x16x16f16 per K-step of 16).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <climits>

#include "stm_launch.h"

namespace stm {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

constexpr int KL_TILE_E = 64;  // output columns per block
constexpr int KL_WAVES = 4;    // waves per block, stacked along s (16 rows each)
constexpr int KL_TILE_S = 16 * KL_WAVES;
// Lane layout of the 16x16 MFMA tiles used here (CDNA3/CDNA4):
//  f64 16x16x4 : A[i][k] at lane i + 16 k; B[k][j] at lane j + 16 k;
//                D[(l/16) + 4 r][l % 16] in accumulator register r (rows interleaved).
//  f16 16x16x16: A[i][4 (l/16) + v] in element v of lane l with i = l % 16;
//                B[4 (l/16) + v][j] likewise with j = l % 16;
//                D[4 (l/16) + r][l % 16] in accumulator register r.

constexpr int KL_THREADS = 64 * KL_WAVES;
static_assert(KL_TILE_S == KL_TILE_E, "square tiles: both panels have the same shape");

// rows [r0, r0 + 64) x columns [k0, k0 + KC) of a row-major (rows x M) matrix
// into registers, zero outside; consecutive threads read consecutive columns
template <int KC>
__device__ __forceinline__ void kl_fetch(const double* __restrict__ g, int rows, int M, int r0, int k0,
                                         double (&v)[KL_TILE_S * KC / KL_THREADS]) {
  constexpr int PER = KL_TILE_S * KC / KL_THREADS;
  if (r0 + KL_TILE_S <= rows && k0 + KC <= M) {  // whole panel inside: no per-value checks
    const double* __restrict__ p = g + (int64_t)r0 * M + k0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = threadIdx.x + u * KL_THREADS;
      v[u] = p[(int64_t)(q / KC) * M + q % KC];
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = threadIdx.x + u * KL_THREADS;
    const int r = q / KC, c = q % KC;
    const int gr = r0 + r, gc = k0 + c;
    v[u] = (gr < rows && gc < M) ? g[(int64_t)gr * M + gc] : 0.0;
  }
}

// fp16(fp32(v)) by the two hardware conversions.  The empty asm keeps the
// compiler from merging them into one correctly rounded float64 -> fp16
// conversion, which it expands into a long integer sequence.
__device__ __forceinline__ _Float16 to_h(double v) {
  float f = (float)v;
  asm volatile("" : "+v"(f));
  return (_Float16)f;
}

// hi is within one fp16 ulp of x, which is all the split needs: x - hi is
// exact in float64 and is what lo keeps.
__device__ __forceinline__ void split_h(double x, _Float16& hi, _Float16& lo) {
  hi = to_h(x);
  lo = to_h((x - (double)hi) * 2048.0);
}

// The block's pipeline position: step j is K chunk j % nk of tile t_begin + j / nk.
struct KlStep {
  int sb, e0, k0;
};

__device__ __forceinline__ KlStep kl_step(int j, int t_begin, int nk, int nts, int kc) {
  const int t = t_begin + j / nk;
  return KlStep{(t % nts) * KL_TILE_S, (t / nts) * KL_TILE_E, (j % nk) * kc};
}

// float64 operands: K chunks of 32 (two LDS buffers, 72 KiB, two blocks per
// CU) measured faster than chunks of 16 with four blocks per CU
struct KlF64 {
  static constexpr int KC = 32;
  static constexpr int LD = KC + 4;  // row stride in doubles (padding spreads the banks)
  static constexpr int PER = KL_TILE_S * KC / KL_THREADS;
  struct Lds {
    double a[2][KL_TILE_S][LD], b[2][KL_TILE_E][LD];
  };
  double4_t acc[4];
  __device__ void zero() {
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = double4_t{0.0, 0.0, 0.0, 0.0};
  }
  static __device__ void put(Lds& L, int buf, const double (&ra)[PER], const double (&rb)[PER]) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = threadIdx.x + u * KL_THREADS;
      L.a[buf][q / KC][q % KC] = ra[u];
      L.b[buf][q / KC][q % KC] = rb[u];
    }
  }
  __device__ void mma(const Lds& L, int buf, int wave, int li, int lk) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const double a = L.a[buf][wave * 16 + li][kk + lk];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, L.b[buf][16 * t + li][kk + lk], acc[t], 0, 0, 0);
    }
  }
  __device__ void store(double* __restrict__ sigma, int S, int E, int s0, int e0, int li, int lk,
                        double sigma_f0, bool additive) const {
    const bool inside = s0 + 16 <= S && e0 + KL_TILE_E <= E;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = e0 + 16 * t + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = s0 + lk + 4 * r;
        const double g = acc[t][r];
        if (inside || (s < S && e < E)) sigma[(int64_t)s * E + e] = sigma_f0 * (additive ? 1.0 + g : exp(g));
      }
    }
  }
};

struct KlF16x3 {
  static constexpr int KC = 32;
  static constexpr int LDH = KC + 8;  // row stride in halves (keeps half4 reads 8-byte aligned)
  static constexpr int PER = KL_TILE_S * KC / KL_THREADS;
  struct Lds {
    __attribute__((aligned(16))) _Float16 ah[2][KL_TILE_S][LDH], al[2][KL_TILE_S][LDH];
    __attribute__((aligned(16))) _Float16 bh[2][KL_TILE_E][LDH], bl[2][KL_TILE_E][LDH];
  };
  float4_t acc_hh[4], acc_x[4];
  __device__ void zero() {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc_hh[t] = float4_t{0.f, 0.f, 0.f, 0.f};
      acc_x[t] = float4_t{0.f, 0.f, 0.f, 0.f};
    }
  }
  static __device__ void put(Lds& L, int buf, const double (&ra)[PER], const double (&rb)[PER]) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = threadIdx.x + u * KL_THREADS;
      const int r = q / KC, c = q % KC;
      split_h(ra[u], L.ah[buf][r][c], L.al[buf][r][c]);
      split_h(rb[u], L.bh[buf][r][c], L.bl[buf][r][c]);
    }
  }
  __device__ void mma(const Lds& L, int buf, int wave, int li, int lk) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 16) {
      const int kc = kk + 4 * lk;
      const half4_t ahi = *reinterpret_cast<const half4_t*>(&L.ah[buf][wave * 16 + li][kc]);
      const half4_t alo = *reinterpret_cast<const half4_t*>(&L.al[buf][wave * 16 + li][kc]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const half4_t bhi = *reinterpret_cast<const half4_t*>(&L.bh[buf][16 * t + li][kc]);
        const half4_t blo = *reinterpret_cast<const half4_t*>(&L.bl[buf][16 * t + li][kc]);
        acc_hh[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ahi, bhi, acc_hh[t], 0, 0, 0);
        acc_x[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(ahi, blo, acc_x[t], 0, 0, 0);
        acc_x[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(alo, bhi, acc_x[t], 0, 0, 0);
      }
    }
  }
  __device__ void store(double* __restrict__ sigma, int S, int E, int s0, int e0, int li, int lk,
                        double sigma_f0, bool additive) const {
    const bool inside = s0 + 16 <= S && e0 + KL_TILE_E <= E;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = e0 + 16 * t + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = s0 + 4 * lk + r;
        const float g = acc_hh[t][r] + acc_x[t][r] * (1.0f / 2048.0f);
        if (inside || (s < S && e < E))
          sigma[(int64_t)s * E + e] = sigma_f0 * (additive ? 1.0 + (double)g : (double)expf(g));
      }
    }
  }
};

// Tiles [blockIdx.x * tiles_per_block, +tiles_per_block) of the nts x nte tile
// grid (sample tile fastest), each as nk K chunks.
template <class P>
__global__ __launch_bounds__(KL_THREADS) void kl_kernel(const double* __restrict__ modes,
                                                        const double* __restrict__ xi,
                                                        double* __restrict__ sigma, int S, int E, int M,
                                                        double sigma_f0, int tiles_per_block, int additive) {
  constexpr int KC = P::KC;
  __shared__ typename P::Lds L;
  const int nts = (S + KL_TILE_S - 1) / KL_TILE_S;
  const int nte = (E + KL_TILE_E - 1) / KL_TILE_E;
  const int nk = (M + KC - 1) / KC;
  const int t_begin = blockIdx.x * tiles_per_block;
  const int t_end = min(nts * nte, t_begin + tiles_per_block);
  if (t_begin >= t_end) return;  // the whole block leaves together
  const int nsteps = (t_end - t_begin) * nk;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  P p;
  p.zero();
  double ra[P::PER], rb[P::PER];
  KlStep cur = kl_step(0, t_begin, nk, nts, KC);
  kl_fetch<KC>(xi, S, M, cur.sb, cur.k0, ra);
  kl_fetch<KC>(modes, E, M, cur.e0, cur.k0, rb);
  for (int j = 0; j < nsteps; ++j) {
    const int buf = j & 1;
    // buffer buf was last read in step j - 2; every wave finished that step
    // before it arrived at the barrier of step j - 1
    P::put(L, buf, ra, rb);
    __syncthreads();
    const KlStep now = cur;
    if (j + 1 < nsteps) {
      cur = kl_step(j + 1, t_begin, nk, nts, KC);
      kl_fetch<KC>(xi, S, M, cur.sb, cur.k0, ra);
      kl_fetch<KC>(modes, E, M, cur.e0, cur.k0, rb);
    }
    p.mma(L, buf, wave, li, lk);
    if (now.k0 + KC >= M) {
      p.store(sigma, S, E, now.sb + wave * 16, now.e0, li, lk, sigma_f0, additive != 0);
      p.zero();
    }
  }
}

hipError_t launch_kl_synthesize(const double* modes, const double* xi, double* sigma, int S, int E, int M,
                                double sigma_f0, bool split_fp16, bool additive, hipStream_t st) {
  if (S <= 0 || E <= 0) return hipSuccess;
  // resident blocks of each variant on the current device, looked up once
  static int resident[64][2];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  int& res = resident[dev][split_fp16 ? 1 : 0];
  if (res == 0) {
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = split_fp16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kl_kernel<KlF16x3>, KL_THREADS, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kl_kernel<KlF64>, KL_THREADS, 0);
    if (e != hipSuccess) return e;
    res = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
  }
  const long long ntiles = (long long)((S + KL_TILE_S - 1) / KL_TILE_S) * ((E + KL_TILE_E - 1) / KL_TILE_E);
  if (ntiles > INT_MAX) return hipErrorInvalidValue;
  const int per_block = (int)((ntiles + res - 1) / res);
  const int blocks = (int)((ntiles + per_block - 1) / per_block);
  if (split_fp16)
    hipLaunchKernelGGL(kl_kernel<KlF16x3>, dim3(blocks), dim3(KL_THREADS), 0, st, modes, xi, sigma, S, E, M,
                       sigma_f0, per_block, additive ? 1 : 0);
  else
    hipLaunchKernelGGL(kl_kernel<KlF64>, dim3(blocks), dim3(KL_THREADS), 0, st, modes, xi, sigma, S, E, M,
                       sigma_f0, per_block, additive ? 1 : 0);
  return hipGetLastError();
}

}  // namespace stm
