// Fused space-time solver: a team of G workgroups owns one sample at a time
// and runs its whole nonlinear space-time solve without leaving the kernel.
//
// Method (Sec. 3.3 eq. mono_disc, Sec. 3.5): the backward-Euler space-time
// system is block lower bidiagonal, so Newton's method on it can be carried
// out slab by slab in time order (block forward substitution, eq. system_C):
// slab k is iterated with Newton steps A_k delta = -R_k until its correction is
// below tolerance, given the converged slab k-1.  Each linear step is GMRES,
// right-preconditioned by one geometric-multigrid V-cycle with weighted-Jacobi
// smoothing on the slab operator A_k = M/dt + K - M diag f'(u_k) (with one
// grid the V-cycle reduces to its smoothing sweeps).  The Jacobi weights are
// either fixed or the reciprocal Chebyshev roots of an interval
// [lmax/ratio, lmax] of D^-1 A, lmax estimated by power iteration once per
// sample.  The initial iterate of slab k takes the time increment of a
// previous solution (u_{k-1} + W_k - W_{k-1}; the paper initialises Newton
// from already computed samples) or, without one, u_{k-1}.  The activation
// map is updated as each slab is accepted.
//
// Teams: with G = 1 a workgroup owns the sample.  With G > 1 (levels without
// coarse V-cycle grids) member r owns a box of the grid (Team::set_box): a band
// of node rows, in 3D of one group of planes;
// passes end with a team barrier (agent-scope release/acquire around an
// atomic counter, bounded wait) and reductions sum the members' partials in
// rank order, so every member takes identical control-flow decisions.  Such
// launches are cooperative: co-residency is guaranteed or the launch fails.
//
// Memory: stencil passes stage tiles of their nodal fields and element
// conductivities into LDS with batched loads, compute each element's vertex
// contributions once (sum factorisation) and gather them per node, on the
// level's grid and on every coarse V-cycle grid alike; restriction and
// prolongation between grids are plain loops over global memory.
//
// Precision: the residual R_k, the update u += delta, the activation
// interpolation and every stored solution are float64.  The Krylov and
// multigrid vectors use TI (double, or float for iterative refinement).
#include "stm_device.h"
#include "q1_stencil.h"
#include "stm_launch.h"

namespace stm {

// Optional per-phase timers (development builds with -DSTM_PHASE_TIMERS):
// thread 0 accumulates wall-clock ticks of each solver phase.
#ifdef STM_PHASE_TIMERS
#define STM_T0(v) long long v = wall_clock64()
#define STM_T1(v, slot) \
  if (threadIdx.x == 0) ph_acc[slot] += wall_clock64() - v
#define STM_T1P(v, slot) \
  if (threadIdx.x == 0) ph[slot] += wall_clock64() - v
#else
#define STM_T0(v)
#define STM_T1(v, slot)
#define STM_T1P(v, slot)
#endif

// A wave-uniform float64 value moved to scalar registers: uniform solver state
// (tolerances, norms, step sizes) then stays out of the vector register file,
// which the stencil passes need.
__device__ __forceinline__ double uni(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Global-memory views of generic pointers.  An access through a generic
// pointer that the compiler cannot place compiles to a flat instruction, and
// flat instructions count against the LDS wait counter as well: every LDS wait
// of a pass would then also wait for the pass's global loads and stores in
// flight.  Device arrays are global; these views make their accesses global
// (cmem: read-only tables, loaded through the scalar cache when uniform).
#define STM_GLOBAL __attribute__((address_space(1)))
#define STM_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ STM_GLOBAL T* gmem(T* p) {
  return (STM_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const STM_GLOBAL T* gmem(const T* p) {
  return (const STM_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const STM_CONST T* cmem(const T* p) {
  return (const STM_CONST T*)p;
}

// The stiffness argument c * v of a pass (kval(v, .) = c v).  The 3D pass
// folds c into the element's conductivity factors instead of scaling the
// eight vertex values; for c a power of two (the theta of backward Euler and
// Crank-Nicolson, 1 - theta) both give the same floating-point result.
template <typename T>
struct KScale {
  T c;
  __device__ __forceinline__ T operator()(T a, T) const { return c * a; }
};
template <typename F>
struct IsKScale {
  static constexpr bool value = false;
};
template <typename T>
struct IsKScale<KScale<T>> {
  static constexpr bool value = true;
};

// Storage type of the element conductivities a 3D pass in T reads.
template <typename T>
struct SigmaOf {
  using type = double;
};
template <>
struct SigmaOf<float> {
  using type = float;
};

constexpr int kPartStride = 16;       // doubles per member in the partials buffer
constexpr double kMinStep = 1.0 / 64;  // smallest damped fraction of a Newton step
constexpr unsigned kSpinLimit = 1u << 25;

template <int DIM>
__device__ __forceinline__ void decode(const GridDev& g, int idx, int& i, int& j, int& k) {
  const int r = fdiv(idx, g.mnx);
  i = idx - r * g.nx;
  if constexpr (DIM == 2) {
    j = r;
    k = 0;
  } else {
    k = fdiv(r, g.mny);
    j = r - k * g.ny;
  }
}

template <typename T, int DIM>
struct TensorOf;
template <typename T>
struct TensorOf<T, 2> { using type = Tensor2<T>; };
template <typename T>
struct TensorOf<T, 3> { using type = Tensor3<T>; };

// Element tensor from the fibre conductivity s and the fibre-table row f
// (kFibStride entries; the layout is described with kFibStride); zr is uniform.
template <typename T, int DIM>
__device__ __forceinline__ typename TensorOf<T, DIM>::type tensor_from(double s, const double* __restrict__ f,
                                                                       double tau, double zr) {
  const double c2 = f[0], s2 = f[1], cs = f[2];
  if constexpr (DIM == 2) {
    return Tensor2<T>{T(s * c2 + tau * s2), T(s * s2 + tau * c2), T((s - tau) * cs)};
  } else {
    return Tensor3<T>{T(s * c2 + tau * s2), T(s * s2 + tau * c2), T(fma(s, zr, tau)), T((s - tau) * cs)};
  }
}

template <typename T, int DIM>
__device__ __forceinline__ typename TensorOf<T, DIM>::type tensor_stored(const T* __restrict__ D,
                                                                         const GridDev& g, int ex, int ey,
                                                                         int ez) {
  const int e = (DIM == 2) ? (ey * g.ex + ex) : ((ez * g.ey + ey) * g.ex + ex);
  if constexpr (DIM == 2) {
    return Tensor2<T>{D[4 * e], D[4 * e + 1], D[4 * e + 3]};
  } else {
    return Tensor3<T>{D[4 * e], D[4 * e + 1], D[4 * e + 2], D[4 * e + 3]};
  }
}

// y = M fm + K fk at node (i, j, k); accessors take coordinates.
template <typename T, int DIM, typename FM, typename FK, typename FD>
__device__ __forceinline__ T apply_at(const GridDev& g, int i, int j, int k, FM fm, FK fk, FD fd, T wself,
                                      T* diag) {
  if constexpr (DIM == 2) {
    return q1_apply_2d<T>(g, i, j, [&](int a, int b) { return fm(a, b, 0); },
                          [&](int a, int b) { return fk(a, b, 0); }, [&](int ex, int ey) { return fd(ex, ey, 0); },
                          wself, diag);
  } else {
    return q1_apply_3d<T>(g, i, j, k, fm, fk, fd, wself, diag);
  }
}

__device__ __forceinline__ double react(double u, double kr, double ar) { return kr * u * (u - ar) * (1.0 - u); }
__device__ __forceinline__ double react_d(double u, double kr, double ar) {
  return kr * (-3.0 * u * u + 2.0 * (1.0 + ar) * u - ar);
}

// MG: the launch contains a level with a multigrid hierarchy.  Without one the
// V-cycle is the Chebyshev-weighted sweeps on the level's grid and no
// coarse-grid code is compiled into the kernel (it would cost registers).
template <typename TI, int DIM, int BLOCK, bool MG>
struct Team {
  const LevelDev* L;
  SolverParams prm;
  const double* sigma;
  TI *V, *Z;
  int64_t vstride;
  unsigned char* work;
  unsigned char* smem;   // dynamic LDS staging area
  double* kdiag0;        // diagonal of the stiffness matrix on grid 0 (per sample)
  TI* dinv;              // inverse diagonal of the slab operator on grid 0 (per Newton step)
  TI* w0;                // reaction weights 1/dt - f'(u) of the slab operator on grid 0
  double* omega;         // shared: per grid, the sweep weights [kMaxMG][kMaxSweeps]
  double* red;           // shared: block reduction scratch
  // team membership
  int rank, G;
  int jb0, jb1;          // owned node rows of grid 0
  int kb0, kb1;          // owned node planes of grid 0 (3D; 0, 1 in 2D)
  unsigned* bar;
  double* part;
  int* fault;
  mutable unsigned gen;  // barriers passed
  mutable unsigned rslot;  // reductions done (partials double buffer)
  mutable bool broken;   // a barrier wait timed out: stop waiting
  // Algorithmic bytes of the passes run so far: every array a pass reads or
  // writes counted once per pass (neighbour and halo re-reads are cache/LDS
  // traffic, not counted).  Uniform across the team; rank 0 reports it.
  mutable double bytes;
#ifdef STM_PHASE_TIMERS
  long long* ph;         // shared per-phase tick accumulators
#endif

  __device__ __forceinline__ double dbytes(int l) const { return 8.0 * L->g[l].ne; }
  __device__ __forceinline__ TI* mgX(int l) const {
    return l == 0 ? nullptr : reinterpret_cast<TI*>(work + L->off_mgX[l]);
  }
  __device__ __forceinline__ TI* mgT(int l) const { return reinterpret_cast<TI*>(work + L->off_mgT[l]); }
  __device__ __forceinline__ TI* mgB(int l) const { return reinterpret_cast<TI*>(work + L->off_mgB[l]); }
  __device__ __forceinline__ TI* mgW(int l) const {
    return l == 0 ? w0 : reinterpret_cast<TI*>(work + L->off_mgW[l]);
  }
  // inverse slab diagonal, conductivities and stiffness diagonal of grid l
  __device__ __forceinline__ TI* mgI(int l) const {
    return l == 0 ? dinv : reinterpret_cast<TI*>(work + L->off_mgI[l]);
  }
  __device__ __forceinline__ const double* mgS(int l) const {
    return l == 0 ? sigma : reinterpret_cast<const double*>(work + L->off_mgS[l]);
  }
  // conductivities of grid l in the precision of a 3D pass in T (float32:
  // the copy made once per sample)
  template <typename T>
  __device__ __forceinline__ const typename SigmaOf<T>::type* mgST(int l) const {
    if constexpr (sizeof(T) == 4)
      return reinterpret_cast<const float*>(work + L->off_mgS32[l]);
    else
      return mgS(l);
  }
  __device__ __forceinline__ double* mgK(int l) const {
    return l == 0 ? kdiag0 : reinterpret_cast<double*>(work + L->off_mgK[l]);
  }

  // ---- team synchronisation and reductions --------------------------------
  // Every wave first waits until its own global stores have completed (a
  // workgroup barrier alone does not wait for them); thread 0 then releases
  // the block's writes at agent scope (write-back of the L2), arrives, waits
  // for the other members and acquires, which invalidates the CU's caches for
  // every wave of the block.
  __device__ __forceinline__ void team_barrier() const {
    if (G > 1) __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (G > 1) {
      if (threadIdx.x == 0) {
        gen += 1;
        if (!broken) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const unsigned target = gen * (unsigned)G;
          unsigned spins = 0;
          while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
              broken = true;
              __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              break;
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
      }
      __syncthreads();
    }
  }
  // End of a pass whose results other members read.
  __device__ __forceinline__ void sync() const { team_barrier(); }

  template <int NV>
  __device__ __forceinline__ void tsum(double (&v)[NV]) const {
    block_sum<BLOCK, NV>(v, red);
    if (G == 1) return;
    double* slot = part + (size_t)(rslot & 1) * G * kPartStride;
    rslot += 1;
    if (threadIdx.x == 0)
      for (int i = 0; i < NV; ++i)
        __hip_atomic_store(slot + rank * kPartStride + i, v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    team_barrier();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int r = 0; r < G; ++r)
        s += __hip_atomic_load(slot + r * kPartStride + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      v[i] = s;
    }
  }
  __device__ __forceinline__ double tmax(double v) const {
    v = block_max<BLOCK>(v, red);
    if (G == 1) return v;
    double* slot = part + (size_t)(rslot & 1) * G * kPartStride;
    rslot += 1;
    if (threadIdx.x == 0)
      __hip_atomic_store(slot + rank * kPartStride, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    team_barrier();
    double s = 0.0;
    for (int r = 0; r < G; ++r)
      s = fmax(s, __hip_atomic_load(slot + r * kPartStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    return s;
  }

  // ---- owned nodes of grid 0 ----------------------------------------------
  // Rows per tile of a z-marching pass on grid l with fields of fbytes bytes:
  // the LDS budget (set on the host) and the per-thread element, staged-node
  // and output-node counts.
  static constexpr int kCE = 3, kCN = 4, kCB = 3;
  __device__ __forceinline__ int zrows_max(int l, int fbytes) const {
    const GridDev& g = L->g[l];
    return max(1, min((int)L->tile_y[l][fbytes == 8 ? 0 : 1][0],
                      min(kCE * BLOCK / g.ex - 1, min(kCN * BLOCK / g.nx - 2, kCB * BLOCK / g.nx))));
  }
  // A member owns node rows [jb0, jb1) of planes [kb0, kb1) (3D), q-th in
  // plane-major order.
  __device__ __forceinline__ int nband() const {
    const GridDev& g = L->g[0];
    return (jb1 - jb0) * g.nx * ((DIM == 3) ? (kb1 - kb0) : 1);
  }
  __device__ __forceinline__ int bidx(int q) const {
    const GridDev& g = L->g[0];
    if constexpr (DIM == 2) {
      return jb0 * g.nx + q;
    } else {
      if (G == 1) return q;
      const int w = (jb1 - jb0) * g.nx;
      const int kk = q / w;
      return ((kb0 + kk) * g.ny + jb0) * g.nx + (q - kk * w);
    }
  }
  // The member's box of grid 0: in 3D the G members are split into Gz
  // groups of planes and each group into G / Gz bands of rows (a z-step of a
  // pass then carries more nodes than with bands of rows alone).
  __device__ __forceinline__ void set_box() {
    const GridDev& g = L->g[0];
    int Gz = 1;
    if constexpr (DIM == 3) {
      // Gz minimises the z-steps of a member's pass: tiles x (planes + the
      // step on the layer below + about two steps of prologue), every member
      // keeping at least 4 planes
      const int Rmax = zrows_max(0, sizeof(TI));
      int best = -1;
      for (int d = 1; d <= G; ++d) {
        if (G % d != 0 || g.nz < 4 * d) continue;
        const int Gy = G / d;
        const int rows = (g.ny + Gy - 1) / Gy, planes = (g.nz + d - 1) / d;
        const int cost = ((rows + Rmax - 1) / Rmax) * (planes + (d > 1 ? 1 : 0) + 2);
        if (best < 0 || cost < best) {
          best = cost;
          Gz = d;
        }
      }
    }
    const int Gy = G / Gz, ry = rank / Gz, rz = rank - ry * Gz;
    jb0 = (int)((long long)ry * g.ny / Gy);
    jb1 = (int)((long long)(ry + 1) * g.ny / Gy);
    kb0 = (DIM == 3) ? (int)((long long)rz * g.nz / Gz) : 0;
    kb1 = (DIM == 3) ? (int)((long long)(rz + 1) * g.nz / Gz) : 1;
  }

  // ---- staged pass on grid 0 ----------------------------------------------
  // For each tile of the owned rows: stage nodal fields f0, f1 (with a
  // one-node halo), f2, f3 (optional, may be null), the tile's element
  // conductivities and fibre rows into LDS, every thread issuing all of its
  // loads before using any; compute every element's vertex contributions of
  // M mval + K kval once (phase A, kval/mval from the raw f0, f1 values); sum
  // the adjacent elements' contributions per node (phase B) and call
  // body(idx, i, j, k, y, o0, o1, o2, o3) with o* the staged values at the
  // node.  Phases A and B read LDS only; every LDS array is laid out so that
  // consecutive lanes touch consecutive words.  Index decoding uses exact
  // multiply-high division.  Ends with a team barrier.
  // Grid l >= 1 (a coarse V-cycle grid, one-workgroup teams) is staged the
  // same way, with its own conductivities, fibre rows and tiles, every row
  // owned.
  template <typename T, typename KV, typename MV, typename Body>
  __device__ __forceinline__ void staged(int l, const T* __restrict__ f0, const T* __restrict__ f1, const T* __restrict__ f2,
                         const T* __restrict__ f3, KV kval, MV mval, Body body) const {
    if constexpr (DIM == 3) {
      zmarch<T>(l, f0, f1, f2, f3, kval, mval, body);
    } else {
      staged_tiles<T>(l, f0, f1, f2, f3, kval, mval, body);
    }
  }

  // ---- z-marching pass (3D) -------------------------------------------------
  // The owned rows of grid l are cut into y-tiles of Ry rows over the whole x
  // extent, and each tile marches through the owned planes [kb0, kb1), with
  // one step on the layer below kb0 first (its top-face contributions) when
  // kb0 > 0.  LDS holds per thread the top-face contributions of its elements
  // of the previous layer (element q always belongs to thread q % BLOCK; four
  // values per element, read and written as one vector), a ring of three
  // planes of f0, f1 over the tile's rows plus a one-row halo, four partial
  // sums per element of one element layer with a border of zeros (one element
  // each side in x and y), and two slots of f2, f3 on the output rows and of
  // the layer conductivities.  Step k:
  //   * direct-to-LDS loads (no registers) of plane k+2 of f0, f1 into the
  //     free ring slot, of the conductivities of layer k+1 and of f2, f3 on
  //     plane k+1 into the other slots;
  //   * phase A: the vertex contributions of the thread's elements of layer k
  //     (between planes k and k+1) by sum factorisation; bottom-face ones plus
  //     the stored top-face ones of layer k-1 are the four sums the element
  //     gives plane k (to LDS); the new top-face ones replace the stored ones;
  //   * an LDS-only barrier (the loads stay in flight);
  //   * phase B: every output node of plane k adds the sums of the four
  //     elements around it in its plane (the zero border stands for elements
  //     outside the grid) and calls body;
  //   * a workgroup barrier, which also waits for the step's loads.
  // f0 and f1 are read from memory once per tile (plus the halo rows), f2, f3
  // and the conductivities once.  A stiffness argument kval = KScale{c} is
  // folded into the element factors.  Ends with a team barrier.
  template <typename T, typename KV, typename MV, typename Body>
  __device__ __forceinline__ void zmarch(int l, const T* __restrict__ f0, const T* __restrict__ f1,
                                         const T* __restrict__ f2, const T* __restrict__ f3, KV kval, MV mval,
                                         Body body) const {
    using T4 = T __attribute__((ext_vector_type(4)));
    const GridDev& g = L->g[l];
    const int nx = g.nx, ny = g.ny, nz = g.nz, EX = g.ex, EY = g.ey, EZ = g.ez;
    const unsigned mnx = g.mnx, mex = g.mex;
    const int plane = ny * nx, eplane = EY * EX;
    const int EXP = EX + 2;  // padded element row
    // tile rows: the LDS budget (set on the host) and the per-thread counts
    const int jb0 = l == 0 ? this->jb0 : 0, jb1 = l == 0 ? this->jb1 : ny;
    const int kb0 = l == 0 ? this->kb0 : 0, kb1 = l == 0 ? this->kb1 : nz;
    const int ks = max(kb0 - 1, 0);  // first step: the layer below the first owned plane
    const int Rmax = zrows_max(l, sizeof(T));
    // as few tiles as Rmax allows, of equal height
    const int ntl = (jb1 - jb0 + Rmax - 1) / Rmax;
    const int Ry = (jb1 - jb0 + ntl - 1) / max(ntl, 1);
    using TS = typename SigmaOf<T>::type;
    constexpr int WS = sizeof(TS) / 4;  // dwords per conductivity
    const STM_GLOBAL TS* __restrict__ sg = gmem(mgST<T>(l));
    const STM_CONST double* __restrict__ fib = cmem(L->fib[l]);
    const STM_GLOBAL T* __restrict__ g0 = gmem(f0);
    const STM_GLOBAL T* __restrict__ g1 = gmem(f1);
    const STM_GLOBAL T* __restrict__ g2 = gmem(f2);
    const STM_GLOBAL T* __restrict__ g3 = gmem(f3);
    const double tau = prm.tau, zr = prm.zr;
    const T hx = T(g.hx), hy = T(g.hy), hz = T(g.hz);
    // the stiffness scale of a KScale argument goes into the element factors
    T ksc = T(1);
    if constexpr (IsKScale<KV>::value) ksc = kval.c;
    const T cxx = ksc * (hy * hz / (T(36) * hx)), cyy = ksc * (hx * hz / (T(36) * hy));
    const T czz = ksc * (hx * hy / (T(36) * hz)), cxy = ksc * (hz / T(24));
    const T cm = hx * hy * hz / T(216);
    const int tid = threadIdx.x;
    constexpr int WT = sizeof(T) / 4;  // dwords per value
    for (int j0 = jb0; j0 < jb1; j0 += Ry) {
      const int je = min(j0 + Ry, jb1);          // output rows [j0, je)
      const int jr0 = max(j0 - 1, 0);            // staged node rows [jr0, jr1]; element rows start there too
      const int jr1 = min(je, ny - 1);
      const int ey1 = min(je - 1, EY - 1);       // element rows [jr0, ey1]
      const int lay = (jr1 - jr0 + 1) * nx;      // staged nodes per plane
      const int elay = (ey1 - jr0 + 1) * EX;     // elements per layer
      const int slay = (ey1 - jr0 + 3) * EXP;    // padded sums per vertex slot
      const int nc = (je - j0) * nx;             // output nodes per plane
      const int gn0 = jr0 * nx, ge0 = jr0 * EX, go0 = j0 * nx;
      T4* __restrict__ TP = reinterpret_cast<T4*>(smem);  // [elay] top-face contributions (per thread)
      T* __restrict__ P = reinterpret_cast<T*>(TP + elay);  // [3 slots][2][lay] f0, f1
      T* __restrict__ S = P + 6 * lay;                      // [4][slay] sums for plane k
      T* __restrict__ Q = S + 4 * slay;                     // [2 slots][2][nc] f2, f3 on plane k
      // [2 slots][elay] conductivities, 8-byte aligned after Q
      TS* __restrict__ SG = reinterpret_cast<TS*>(
          smem + (((size_t)elay * sizeof(T4) + (size_t)(6 * lay + 4 * slay + 4 * nc) * sizeof(T) + 7) & ~(size_t)7));
      // loads of plane kp of f0, f1 into ring slot sl, of layer kl's
      // conductivities and of f2, f3 on plane kq into slot parity
      auto load_plane = [&](int kp, int sl) {
        const size_t base = (size_t)kp * plane + gn0;
        dma_dwords(reinterpret_cast<const STM_GLOBAL unsigned*>(g0 + base), P + (2 * sl) * lay, WT * lay);
        dma_dwords(reinterpret_cast<const STM_GLOBAL unsigned*>(g1 + base), P + (2 * sl + 1) * lay, WT * lay);
      };
      auto load_sigma = [&](int kl) {
        dma_dwords(reinterpret_cast<const STM_GLOBAL unsigned*>(sg + (size_t)kl * eplane + ge0), SG + (kl & 1) * elay,
                   WS * elay);
      };
      auto load_q = [&](int kq) {
        T* qs = Q + (kq & 1) * 2 * nc;
        if (f2) dma_dwords(reinterpret_cast<const STM_GLOBAL unsigned*>(g2 + (size_t)kq * plane + go0), qs, WT * nc);
        if (f3) dma_dwords(reinterpret_cast<const STM_GLOBAL unsigned*>(g3 + (size_t)kq * plane + go0), qs + nc, WT * nc);
      };
      // prologue: zero top-face contributions and sums (the border stays
      // zero), planes ks and ks + 1, conductivities of layer ks, and f2, f3
      // on plane kb0 when the march starts there
      for (int q = tid; q < elay; q += BLOCK) TP[q] = T4{T(0), T(0), T(0), T(0)};
      for (int q = tid; q < 4 * slay; q += BLOCK) S[q] = T(0);
      if (!f2 || !f3)
        for (int q = tid; q < 4 * nc; q += BLOCK) Q[q] = T(0);
      __syncthreads();
      load_plane(ks, 0);
      load_plane(ks + 1, 1);
      load_sigma(ks);
      if (ks == kb0) load_q(kb0);
      __syncthreads();
      int s0 = 0;  // ring slot of plane k
      for (int k = ks; k < kb1; ++k) {
        const int s1 = s0 == 2 ? 0 : s0 + 1;
        const int s2 = s1 == 2 ? 0 : s1 + 1;
        STM_T0(t_za);
        // ---- loads for the next step: plane k+2 and layer k+1 when layer
        // k+1 is computed (it adds to plane k+1 < kb1); f2, f3 of the next
        // owned plane ----
        if (k + 2 <= min(kb1, nz - 1)) load_plane(k + 2, s2);
        if (k + 1 < min(kb1, EZ)) load_sigma(k + 1);
        if (k + 1 < kb1) load_q(k + 1);
        const T* __restrict__ a0 = P + (2 * s0) * lay;
        const T* __restrict__ a1 = P + (2 * s0 + 1) * lay;
        const TS* __restrict__ sgk = SG + (k & 1) * elay;
        // ---- phase A: element layer k ----
        if (k < EZ) {
          const T* __restrict__ b0 = P + (2 * s1) * lay;
          const T* __restrict__ b1 = P + (2 * s1 + 1) * lay;
          // the layer's fibre row (uniform: scalar loads) folded with the
          // element constants: ax = cxx (s c2 + tau s2), ay = cyy (s s2 + tau c2),
          // az = czz (s zr + tau), axy = cxy (s - tau) cs for conductivity s
          const double c2 = fib[kFibStride * k], s2 = fib[kFibStride * k + 1], cs = fib[kFibStride * k + 2];
          const T kx1 = T(c2) * cxx, kx0 = T(tau * s2) * cxx;
          const T ky1 = T(s2) * cyy, ky0 = T(tau * c2) * cyy;
          const T kz1 = T(zr) * czz, kz0 = T(tau) * czz;
          const T kxy = T(cs) * cxy, tauT = T(tau);
          // every LDS read of an element is issued before its arithmetic (a
          // scheduling barrier keeps the compiler from interleaving them with
          // waits), so one LDS round trip per element
#pragma unroll 1
          for (int q = tid; q < elay; q += BLOCK) {
            const int r = (int)fdiv(q, mex);
            const int o = q + r;                // staged node of the element's vertex (0, 0)
            const int qp = o + r + EXP + 1;     // its padded sum slot
            T x0[8], x1[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
              const int off = o + (v & 1) + ((v >> 1) & 1) * nx;
              x0[v] = (v & 4) ? b0[off] : a0[off];
              x1[v] = (v & 4) ? b1[off] : a1[off];
            }
            const TS se = sgk[q];
            const T4 tp = TP[q];
            __builtin_amdgcn_sched_barrier(0);
            T kv[8], mv[8], out[8];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
              if constexpr (IsKScale<KV>::value)
                kv[v] = x0[v];
              else
                kv[v] = kval(x0[v], x1[v]);
              mv[v] = mval(x0[v], x1[v]);
            }
            const T sT = T(se);
            elem_apply_3d<T>(kv, mv, sT * kx1 + kx0, sT * ky1 + ky0, sT * kz1 + kz0, (sT - tauT) * kxy, cm, out);
            S[qp] = tp.x + out[0];
            S[slay + qp] = tp.y + out[1];
            S[2 * slay + qp] = tp.z + out[2];
            S[3 * slay + qp] = tp.w + out[3];
            TP[q] = T4{out[4], out[5], out[6], out[7]};
          }
        } else {
#pragma unroll 1
          for (int q = tid; q < elay; q += BLOCK) {
            const int r = (int)fdiv(q, mex);
            const int qp = q + 2 * r + EXP + 1;
            const T4 tp = TP[q];
            S[qp] = tp.x;
            S[slay + qp] = tp.y;
            S[2 * slay + qp] = tp.z;
            S[3 * slay + qp] = tp.w;
          }
        }
        STM_T1P(t_za, 6);
        STM_T0(t_zb);
        lds_barrier();
        // ---- phase B: output nodes of plane k (an owned plane) ----
        const T* __restrict__ qk = Q + (k & 1) * 2 * nc;
#pragma unroll 1
        for (int q = tid; q < (k >= kb0 ? nc : 0); q += BLOCK) {
          const int r = fdiv(q, mnx);
          const int i = q - r * nx;
          const int j = j0 + r;
          // element (i - 1 + a, j - 1 + b) gives vertex (1 - a) + 2 (1 - b)
          const int e = (j - jr0) * EXP + i;
          const T c0 = S[3 * slay + e], c1 = S[2 * slay + e + 1];
          const T c2 = S[slay + e + EXP], c3 = S[e + EXP + 1];
          const int o = (j - jr0) * nx + i;
          const T o0 = a0[o], o1 = a1[o], o2 = qk[q], o3 = qk[nc + q];
          __builtin_amdgcn_sched_barrier(0);
          T y = T(0);
          y += c0;
          y += c1;
          y += c2;
          y += c3;
          body(k * plane + go0 + q, i, j, k, y, o0, o1, o2, o3);
        }
        __syncthreads();  // also waits for the step's direct-to-LDS loads
        STM_T1P(t_zb, 7);
        s0 = s1;
      }
    }
    if (G > 1) team_barrier();
  }

  // n dwords from global memory to LDS by direct-to-LDS loads: lane i of the
  // wave whose first thread is w writes dword w + i + c BLOCK of the range
  // (the LDS address of a wave's load is uniform; lanes past n do not load).
  // Complete after the next workgroup barrier that follows a fence.
  __device__ __forceinline__ void dma_dwords(const STM_GLOBAL unsigned* __restrict__ src, void* dst, int n) const {
    const int tid = threadIdx.x;
    unsigned* d = reinterpret_cast<unsigned*>(dst);
    const int wbase = tid & ~(kWave - 1);
    for (int c0 = 0; c0 < n; c0 += BLOCK) {
      if (c0 + tid < n)
        __builtin_amdgcn_global_load_lds(src + c0 + tid, (__attribute__((address_space(3))) void*)(d + c0 + wbase), 4,
                                         0, 0);
    }
  }
  // Workgroup barrier ordering LDS accesses only: direct-to-LDS loads in
  // flight stay in flight (a fence would wait for them).
  __device__ __forceinline__ void lds_barrier() const { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

  // ---- tiled pass (2D) --------------------------------------------------------
  template <typename T, typename KV, typename MV, typename Body>
  __device__ __forceinline__ void staged_tiles(int l, const T* __restrict__ f0, const T* __restrict__ f1,
                                               const T* __restrict__ f2, const T* __restrict__ f3, KV kval, MV mval,
                                               Body body) const {
    constexpr int NV = (DIM == 3) ? 8 : 4;
    constexpr int U = 4;                      // batched loads per thread in the staging loop
    constexpr int UA = (DIM == 3) ? 1 : 2;    // independent elements per thread in phase A
    const GridDev& g = L->g[l];
    const int nx = g.nx, EX = g.ex;
    const unsigned mnx = g.mnx, mex = g.mex;
    const int nf = 2 + (f2 ? 1 : 0) + (f3 ? 1 : 0);
    const int Ry = L->tile_y[l][sizeof(T) == 8 ? 0 : 1][nf - 2];
    const int Rz = (DIM == 3) ? L->tile_z[l][sizeof(T) == 8 ? 0 : 1][nf - 2] : 1;
    const int nzz = (DIM == 3) ? g.nz : 1;
    const int jb0 = l == 0 ? this->jb0 : 0, jb1 = l == 0 ? this->jb1 : g.ny;
    const double* __restrict__ sg = mgS(l);
    const double* __restrict__ fib = L->fib[l];
    const double tau = prm.tau, zr = prm.zr;
    const T hx = T(g.hx), hy = T(g.hy), hz = T(g.hz);
    const T cxx = (DIM == 3) ? hy * hz / (T(36) * hx) : hy / (T(6) * hx);
    const T cyy = (DIM == 3) ? hx * hz / (T(36) * hy) : hx / (T(6) * hy);
    const T czz = hx * hy / (T(36) * hz), cxy = hz / T(24);
    const T cm = (DIM == 3) ? hx * hy * hz / T(216) : hx * hy / T(36);
    for (int k0 = 0; k0 < nzz; k0 += Rz) {
      for (int j0 = jb0; j0 < jb1; j0 += Ry) {
        const int je = min(j0 + Ry, jb1);  // computed rows [j0, je)
        const int ke = min(k0 + Rz, nzz);  // computed planes [k0, ke)
        const int jr0 = max(j0 - 1, 0), jr1 = min(je, g.ny - 1);
        const int kr0 = (DIM == 3) ? max(k0 - 1, 0) : 0, kr1 = (DIM == 3) ? min(ke, g.nz - 1) : 0;
        const int sy = jr1 - jr0 + 1;
        const int lay = sy * nx;  // staged nodes per plane
        const int nst = lay * (kr1 - kr0 + 1);
        const int ey0 = max(j0 - 1, 0), ey1 = min(je - 1, g.ey - 1);
        const int ez0 = (DIM == 3) ? max(k0 - 1, 0) : 0, ez1 = (DIM == 3) ? min(ke - 1, g.ez - 1) : 0;
        const int sey = ey1 - ey0 + 1;
        const int elay = sey * EX;  // staged elements per plane
        const int nse = elay * (ez1 - ez0 + 1);
        const int nfr = (DIM == 3) ? (ez1 - ez0 + 1) : sey;  // fibre rows
        const int fr0 = (DIM == 3) ? ez0 : ey0;
        const unsigned mlay = (DIM == 3) ? fdiv_magic((unsigned)lay) : 0u;
        const unsigned melay = (DIM == 3) ? fdiv_magic((unsigned)elay) : 0u;
        T* l0 = reinterpret_cast<T*>(smem);
        T* l1 = l0 + nst;
        T* l2 = l1 + nst;
        T* l3 = l2 + (f2 ? nst : 0);
        double* ls = reinterpret_cast<double*>(smem + ((nf * (size_t)nst * sizeof(T) + 15) & ~(size_t)15));
        T* lc = reinterpret_cast<T*>(ls + nse);  // [NV][nse]
        double* lf = reinterpret_cast<double*>(
            reinterpret_cast<unsigned char*>(lc) + ((NV * (size_t)nse * sizeof(T) + 15) & ~(size_t)15));
        // ---- stage: batched loads, then LDS stores ----
        STM_T0(t_st);
        const int gq0 = (DIM == 3) ? (kr0 * g.ny + jr0) * nx : jr0 * nx;
        const int plane = g.ny * nx;
        for (int qb = threadIdx.x; qb < nst; qb += BLOCK * U) {
          T r0[U], r1[U], r2[U], r3[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int q = qb + u * BLOCK;
            if (q < nst) {
              int gq;
              if constexpr (DIM == 3) {
                const int lz = fdiv(q, mlay);
                gq = gq0 + lz * plane + (q - lz * lay);
              } else {
                gq = gq0 + q;
              }
              r0[u] = f0[gq];
              r1[u] = f1[gq];
              if (f2) r2[u] = f2[gq];
              if (f3) r3[u] = f3[gq];
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int q = qb + u * BLOCK;
            if (q < nst) {
              l0[q] = r0[u];
              l1[q] = r1[u];
              if (f2) l2[q] = r2[u];
              if (f3) l3[q] = r3[u];
            }
          }
        }
        {
          const int ge0 = (DIM == 3) ? (ez0 * g.ey + ey0) * EX : ey0 * EX;
          const int eplane = g.ey * EX;
          for (int qb = threadIdx.x; qb < nse; qb += BLOCK * U) {
            double rs[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int q = qb + u * BLOCK;
              if (q < nse) {
                int ge;
                if constexpr (DIM == 3) {
                  const int lz = fdiv(q, melay);
                  ge = ge0 + lz * eplane + (q - lz * elay);
                } else {
                  ge = ge0 + q;
                }
                rs[u] = sg[ge];
              }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int q = qb + u * BLOCK;
              if (q < nse) ls[q] = rs[u];
            }
          }
          for (int q = threadIdx.x; q < kFibStride * nfr; q += BLOCK) lf[q] = fib[kFibStride * fr0 + q];
        }
        __syncthreads();
        STM_T1P(t_st, 6);
        STM_T0(t_pa);
        // ---- phase A: element contributions (UA elements per iteration) ----
        for (int qb = threadIdx.x; qb < nse; qb += UA * BLOCK) {
          T kv[UA][NV], mv[UA][NV], out[UA][NV];
          typename TensorOf<T, DIM>::type D[UA];
#pragma unroll
          for (int h = 0; h < UA; ++h) {
            const int q = qb + h * BLOCK;
            const int qq = q < nse ? q : 0;
            int lz = 0, rem = qq;
            if constexpr (DIM == 3) {
              lz = fdiv(qq, melay);
              rem = qq - lz * elay;
            }
            const int r = fdiv(rem, mex);
            const int ex = rem - r * EX;
            const int ey = ey0 + r, ez = ez0 + lz;
            D[h] = tensor_from<T, DIM>(ls[qq], lf + kFibStride * ((DIM == 3) ? lz : r), tau, zr);
            const int base = ((ez - kr0) * sy + (ey - jr0)) * nx + ex;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const int o = base + ((v >> 2) & 1) * lay + ((v >> 1) & 1) * nx + (v & 1);
              const T a = l0[o], b = l1[o];
              kv[h][v] = kval(a, b);
              mv[h][v] = mval(a, b);
            }
          }
#pragma unroll
          for (int h = 0; h < UA; ++h) {
            if constexpr (DIM == 3) elem_apply_3d<T>(kv[h], mv[h], D[h], cxx, cyy, czz, cxy, cm, out[h]);
            else elem_apply_2d<T>(kv[h], mv[h], D[h], cxx, cyy, cm, out[h]);
          }
#pragma unroll
          for (int h = 0; h < UA; ++h) {
            const int q = qb + h * BLOCK;
            if (q < nse) {
#pragma unroll
              for (int v = 0; v < NV; ++v) lc[v * nse + q] = out[h][v];
            }
          }
        }
        __syncthreads();
        STM_T1P(t_pa, 7);
        // ---- phase B: nodes of the tile ----
        const int cy = je - j0;
        const int clay = cy * nx;
        const int nc = clay * (ke - k0);
        const unsigned mclay = (DIM == 3) ? fdiv_magic((unsigned)clay) : 0u;
        for (int q = threadIdx.x; q < nc; q += BLOCK) {
          int lz = 0, rem = q;
          if constexpr (DIM == 3) {
            lz = fdiv(q, mclay);
            rem = q - lz * clay;
          }
          const int r = fdiv(rem, mnx);
          const int i = rem - r * nx;
          const int j = j0 + r, k = k0 + lz;
          const int idx = (DIM == 3) ? ((k * g.ny + j) * nx + i) : (j * nx + i);
          T y = T(0);
#pragma unroll
          for (int c = 0; c < ((DIM == 3) ? 2 : 1); ++c) {
            const int ez = k - 1 + c;
            const bool okz = (DIM == 2) || (ez >= 0 && ez < g.ez);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              const int ey = j - 1 + b;
              const bool oky = okz && ey >= 0 && ey < g.ey;
#pragma unroll
              for (int a = 0; a < 2; ++a) {
                const int ex = i - 1 + a;
                const bool ok = oky && ex >= 0 && ex < EX;
                const int el = (((DIM == 3) ? (ez - ez0) : 0) * sey + (ey - ey0)) * EX + ex;
                const int v = (1 - a) + 2 * (1 - b) + ((DIM == 3) ? 4 * (1 - c) : 0);
                const T cv = lc[v * nse + (ok ? el : 0)];
                y += ok ? cv : T(0);
              }
            }
          }
          const int o = (((DIM == 3) ? (k - kr0) : 0) * sy + (j - jr0)) * nx + i;
          body(idx, i, j, k, y, l0[o], l1[o], f2 ? l2[o] : T(0), f3 ? l3[o] : T(0));
        }
        __syncthreads();
      }
    }
    if (G > 1) team_barrier();
  }

  // ---- per-sample operator data ----------------------------------------------
  // On every coarse V-cycle grid (one-workgroup teams): the conductivity of an
  // element = mean of its 2^d children, and the stiffness diagonal from it and
  // the grid's own fibre rows (rediscretisation).  On grid 0: the stiffness
  // diagonal at the owned nodes.  Ends with a team barrier.
  __device__ __forceinline__ void setup_operator() const {
    const int tid = threadIdx.x;
    const double tau = prm.tau, zr = prm.zr;
    for (int l = 1; l < (MG ? L->nmg : 1); ++l) {
      const GridDev& gc = L->g[l];
      const GridDev& gf = L->g[l - 1];
      double* Sc = const_cast<double*>(mgS(l));
      const double* Sf = mgS(l - 1);
      for (int e = tid; e < gc.ne; e += BLOCK) {
        const int E = e % gc.ex;
        const int F = (DIM == 2) ? e / gc.ex : (e / gc.ex) % gc.ey;
        const int Gz = (DIM == 2) ? 0 : e / (gc.ex * gc.ey);
        double acc = 0.0;
        const int cz = (DIM == 3) ? 2 : 1;
        for (int c = 0; c < cz; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
              const int fx = 2 * E + a, fy = 2 * F + b, fz = 2 * Gz + c;
              acc += Sf[(DIM == 2) ? (fy * gf.ex + fx) : ((fz * gf.ey + fy) * gf.ex + fx)];
            }
        Sc[e] = acc / (4 * cz);
        if constexpr (DIM == 3 && sizeof(TI) == 4)
          const_cast<float*>(mgST<TI>(l))[e] = float(Sc[e]);
      }
      __syncthreads();
      double* Kc = mgK(l);
      const double* fibc = L->fib[l];
      for (int idx = tid; idx < gc.n; idx += BLOCK) {
        int i, j, k;
        decode<DIM>(gc, idx, i, j, k);
        auto z = [&](int, int, int) { return 0.0; };
        double dd;
        apply_at<double, DIM>(
            gc, i, j, k, z, z,
            [&](int ex, int ey, int ez) {
              const int e = (DIM == 3) ? ((ez * gc.ey + ey) * gc.ex + ex) : (ey * gc.ex + ex);
              return tensor_from<double, DIM>(Sc[e], fibc + kFibStride * ((DIM == 3) ? ez : ey), tau, zr);
            },
            0.0, &dd);
        Kc[idx] = dd;
      }
      __syncthreads();
    }
    const GridDev& g0 = L->g[0];
    const int nb = nband();
    for (int q = tid; q < nb; q += BLOCK) {
      const int idx = bidx(q);
      int i, j, k;
      decode<DIM>(g0, idx, i, j, k);
      auto z = [&](int, int, int) { return 0.0; };
      double dd;
      apply_at<double, DIM>(
          g0, i, j, k, z, z,
          [&](int ex, int ey, int ez) {
            const int e = (DIM == 3) ? ((ez * g0.ey + ey) * g0.ex + ex) : (ey * g0.ex + ex);
            return tensor_from<double, DIM>(sigma[e], L->fib[0] + kFibStride * ((DIM == 3) ? ez : ey), tau, zr);
          },
          0.0, &dd);
      kdiag0[idx] = dd;
    }
    if constexpr (DIM == 3 && sizeof(TI) == 4) {
      // the members share the float32 conductivity copy of grid 0 out by
      // element; the closing team barrier publishes it
      float* s32 = const_cast<float*>(mgST<TI>(0));
      for (int e = rank * BLOCK + tid; e < g0.ne; e += G * BLOCK) s32[e] = float(sigma[e]);
    }
    sync();
  }

  // Reaction weights injected from grid-0 values u and the slab diagonal on
  // every coarse V-cycle grid (one-workgroup teams; no barrier).
  __device__ __forceinline__ void coarse_weights(const double* __restrict__ u, double inv_dt) const {
    const GridDev& g0 = L->g[0];
    const double kr = prm.k_react, ar = prm.a_react, th = prm.theta;
    for (int l = 1; l < (MG ? L->nmg : 1); ++l) {
      const GridDev& gc = L->g[l];
      TI* wl = mgW(l);
      TI* dl = mgI(l);
      const double* Kc = mgK(l);
      const double cmc = (DIM == 3) ? 8.0 * gc.hx * gc.hy * gc.hz / 216.0 : 4.0 * gc.hx * gc.hy / 36.0;
      const int st = 1 << l;
      for (int idx = threadIdx.x; idx < gc.n; idx += BLOCK) {
        int I, J, K;
        decode<DIM>(gc, idx, I, J, K);
        const int q = (DIM == 3) ? (((K * st) * g0.ny + J * st) * g0.nx + I * st) : ((J * st) * g0.nx + I * st);
        const double w = inv_dt - react_d(u[q], kr, ar);
        wl[idx] = TI(w);
        dl[idx] = TI(1.0 / (th * Kc[idx] + nel(l, I, J, K) * cmc * w));
      }
    }
  }

  // number of elements adjacent to node (i, j, k) of grid l
  __device__ __forceinline__ int nel(int l, int i, int j, int k) const {
    const GridDev& g = L->g[l];
    int c = ((i > 0) + (i < g.nx - 1)) * ((j > 0) + (j < g.ny - 1));
    if constexpr (DIM == 3) c *= (k > 0) + (k < g.nz - 1);
    return c;
  }
  // mass diagonal per adjacent element (times the nodal weight)
  __device__ __forceinline__ TI cmd0() const {
    const GridDev& g = L->g[0];
    return (DIM == 3) ? TI(8.0 * g.hx * g.hy * g.hz / 216.0) : TI(4.0 * g.hx * g.hy / 36.0);
  }

  // ---- smoothing -----------------------------------------------------------
  // out = x + om (b - A x) / diag on grid l;  x == null means x = 0 (out = om b / diag)
  __device__ __forceinline__ void jacobi(int l, const TI* __restrict__ b, const TI* __restrict__ x, TI* __restrict__ out,
                         TI om) const {
    const int n = L->g[l].n;
    bytes = uni(bytes + ((x ? 5.0 : 4.0) * sizeof(TI) * n + (x ? dbytes(l) : 0.0)));
    const TI* __restrict__ w = mgW(l);
    const TI* __restrict__ di = mgI(l);
    if (!x) {
      const int nb = l == 0 ? nband() : n;
      for (int qb = threadIdx.x; qb < nb; qb += BLOCK * 4) {
        TI rb[4], rd[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int q = qb + v * BLOCK;
          if (q < nb) {
            const int idx = l == 0 ? bidx(q) : q;
            rb[v] = b[idx];
            rd[v] = di[idx];
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int q = qb + v * BLOCK;
          if (q < nb) out[l == 0 ? bidx(q) : q] = om * rb[v] * rd[v];
        }
      }
      sync();
      return;
    }
    staged<TI>(
        l, x, w, b, di, KScale<TI>{TI(prm.theta)}, [](TI a, TI ww) { return ww * a; },
        [&](int idx, int, int, int, TI y, TI xo, TI, TI bo, TI dio) { gmem(out)[idx] = xo + om * (bo - y) * dio; });
  }

  // Two Jacobi sweeps on grid 0 in one pass over the tiles (2D):
  // out = J2(J1(x)), Jq(v) = v + omq (b - A v) dinv.  A tile stages x, the
  // mass weights, b and dinv over its rows plus two halo rows each side,
  // computes the first sweep on its rows plus one row each side into LDS, and
  // the second sweep on its rows from there.  Halo rows of the first sweep take
  // the same operations in the same order as in the pass that owns them, so the
  // result equals two single sweeps.  x == null stands for the sweep from zero,
  // x = om0 b dinv, formed while staging (three sweeps in the pass).  out must
  // not alias x.  Ends with a team barrier.
  __device__ __forceinline__ void jacobi_pair(const TI* __restrict__ x, const TI* __restrict__ b, TI* __restrict__ out, TI om0,
                              TI om1, TI om2) const {
    static_assert(DIM == 2, "the fused sweep pair is 2D");
    using T = TI;
    constexpr int NV = 4;
    constexpr int U = 4;
    constexpr int UA = 2;
    const GridDev& g = L->g[0];
    bytes = uni(bytes + ((x ? 5.0 : 4.0) * sizeof(TI) * g.n + dbytes(0)));
    const T* __restrict__ w = mgW(0);
    const T* __restrict__ di = dinv;
    const int nx = g.nx, EX = g.ex;
    const unsigned mnx = g.mnx, mex = g.mex;
    const int Ry = sizeof(T) == 8 ? L->tile_p8 : L->tile_p4;
    const double* __restrict__ sg = sigma;
    const double* __restrict__ fib = L->fib[0];
    const double tau = prm.tau, zr = prm.zr;
    const T hx = T(g.hx), hy = T(g.hy);
    const T cxx = hy / (T(6) * hx), cyy = hx / (T(6) * hy), cm = hx * hy / T(36);
    const T th = T(prm.theta);
    for (int j0 = jb0; j0 < jb1; j0 += Ry) {
      const int je = min(j0 + Ry, jb1);                          // second sweep: rows [j0, je)
      const int a0 = max(j0 - 1, 0), a1 = min(je + 1, g.ny);     // first sweep: rows [a0, a1)
      const int jr0 = max(j0 - 2, 0), jr1 = min(je + 1, g.ny - 1);  // staged node rows [jr0, jr1]
      const int ey0 = jr0, ey1 = min(je, g.ey - 1);              // staged element rows [ey0, ey1]
      const int nst = (jr1 - jr0 + 1) * nx;
      const int nse = (ey1 - ey0 + 1) * EX;
      T* lx0 = reinterpret_cast<T*>(smem);
      T* lw = lx0 + nst;
      T* lb = lw + nst;
      T* ld = lb + nst;
      T* lx1 = ld + nst;
      double* ls = reinterpret_cast<double*>(smem + ((5 * (size_t)nst * sizeof(T) + 15) & ~(size_t)15));
      T* lc = reinterpret_cast<T*>(ls + nse);  // [NV][nse]
      double* lf = reinterpret_cast<double*>(
          reinterpret_cast<unsigned char*>(lc) + ((NV * (size_t)nse * sizeof(T) + 15) & ~(size_t)15));
      // ---- stage ----
      const int gq0 = jr0 * nx;
      for (int qb = threadIdx.x; qb < nst; qb += BLOCK * U) {
        T r0[U], r1[U], r2[U], r3[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = qb + u * BLOCK;
          if (q < nst) {
            if (x) r0[u] = x[gq0 + q];
            r1[u] = w[gq0 + q];
            r2[u] = b[gq0 + q];
            r3[u] = di[gq0 + q];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int q = qb + u * BLOCK;
          if (q < nst) {
            lx0[q] = x ? r0[u] : om0 * r2[u] * r3[u];
            lw[q] = r1[u];
            lb[q] = r2[u];
            ld[q] = r3[u];
          }
        }
      }
      {
        const int ge0 = ey0 * EX;
        for (int qb = threadIdx.x; qb < nse; qb += BLOCK * U) {
          double rs[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int q = qb + u * BLOCK;
            if (q < nse) rs[u] = sg[ge0 + q];
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int q = qb + u * BLOCK;
            if (q < nse) ls[q] = rs[u];
          }
        }
        for (int q = threadIdx.x; q < kFibStride * (ey1 - ey0 + 1); q += BLOCK) lf[q] = fib[kFibStride * ey0 + q];
      }
      __syncthreads();
#pragma unroll 1
      for (int sweep = 0; sweep < 2; ++sweep) {
        // element rows [e0, e1] whose contributions this sweep gathers
        const int e0 = sweep == 0 ? ey0 : max(j0 - 1, 0);
        const int e1 = sweep == 0 ? ey1 : min(je - 1, g.ey - 1);
        const T* __restrict__ lxs = sweep == 0 ? lx0 : lx1;
        const int ne = (e1 - e0 + 1) * EX;
        // ---- phase A: element contributions of M (w v) + K (theta v) ----
        for (int qb = threadIdx.x; qb < ne; qb += UA * BLOCK) {
          T kv[UA][NV], mv[UA][NV], o4[UA][NV];
          Tensor2<T> D[UA];
          int qs[UA];
#pragma unroll
          for (int h = 0; h < UA; ++h) {
            const int q = qb + h * BLOCK;
            const int qq = q < ne ? q : 0;
            const int r = fdiv(qq, mex);
            const int ex = qq - r * EX;
            const int rr = e0 - ey0 + r;  // staged element row
            qs[h] = rr * EX + ex;
            D[h] = tensor_from<T, 2>(ls[qs[h]], lf + kFibStride * rr, tau, zr);
            const int base = rr * nx + ex;  // staged node rows start at ey0
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const int o = base + ((v >> 1) & 1) * nx + (v & 1);
              const T a = lxs[o], ww = lw[o];
              kv[h][v] = th * a;
              mv[h][v] = ww * a;
            }
          }
#pragma unroll
          for (int h = 0; h < UA; ++h) elem_apply_2d<T>(kv[h], mv[h], D[h], cxx, cyy, cm, o4[h]);
#pragma unroll
          for (int h = 0; h < UA; ++h) {
            if (qb + h * BLOCK < ne) {
#pragma unroll
              for (int v = 0; v < NV; ++v) lc[v * nse + qs[h]] = o4[h][v];
            }
          }
        }
        __syncthreads();
        // ---- phase B: nodes of rows [n0r, n1r) ----
        const int n0r = sweep == 0 ? a0 : j0, n1r = sweep == 0 ? a1 : je;
        const int nc = (n1r - n0r) * nx;
        const T om = sweep == 0 ? om1 : om2;
        for (int q = threadIdx.x; q < nc; q += BLOCK) {
          const int r = fdiv(q, mnx);
          const int i = q - r * nx;
          const int j = n0r + r;
          T y = T(0);
#pragma unroll
          for (int bb = 0; bb < 2; ++bb) {
            const int ey = j - 1 + bb;
            const bool oky = ey >= 0 && ey < g.ey;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const int ex = i - 1 + a;
              const bool ok = oky && ex >= 0 && ex < EX;
              const int el = (ey - ey0) * EX + ex;
              const int v = (1 - a) + 2 * (1 - bb);
              const T cv = lc[v * nse + (ok ? el : 0)];
              y += ok ? cv : T(0);
            }
          }
          const int o = (j - jr0) * nx + i;
          const T xn = lxs[o] + om * (lb[o] - y) * ld[o];
          if (sweep == 0) lx1[o] = xn;
          else out[j * nx + i] = xn;
        }
        __syncthreads();
      }
    }
    if (G > 1) team_barrier();
  }

  // Every sweep of the smoother in one pass, for a one-workgroup team whose
  // grid fits one tile (2D): the mass weights, b, dinv, sigma and the fibre
  // rows are staged once; the first sweep (from x = 0) is om b dinv, the later
  // ones alternate between two LDS vectors, and the last is written to out.
  // Each sweep takes the operations of a single sweep in the same order.  Ends
  // with a workgroup barrier.
  __device__ __forceinline__ void jacobi_resident(const TI* __restrict__ b, TI* __restrict__ out, int nc) const {
    static_assert(DIM == 2, "the resident smoother is 2D");
    using T = TI;
    constexpr int NV = 4;
    constexpr int U = 4;
    constexpr int UA = 2;
    const GridDev& g = L->g[0];
    bytes = uni(bytes + (4.0 * sizeof(TI) * g.n + dbytes(0)));
    const T* __restrict__ w = mgW(0);
    const T* __restrict__ di = dinv;
    const int nx = g.nx, EX = g.ex;
    const unsigned mnx = g.mnx, mex = g.mex;
    const double tau = prm.tau, zr = prm.zr;
    const T hx = T(g.hx), hy = T(g.hy);
    const T cxx = hy / (T(6) * hx), cyy = hx / (T(6) * hy), cm = hx * hy / T(36);
    const T th = T(prm.theta);
    const int nst = g.n, nse = g.ne;
    T* lx0 = reinterpret_cast<T*>(smem);
    T* lw = lx0 + nst;
    T* lb = lw + nst;
    T* ld = lb + nst;
    T* lx1 = ld + nst;
    double* ls = reinterpret_cast<double*>(smem + ((5 * (size_t)nst * sizeof(T) + 15) & ~(size_t)15));
    T* lc = reinterpret_cast<T*>(ls + nse);  // [NV][nse]
    double* lf = reinterpret_cast<double*>(
        reinterpret_cast<unsigned char*>(lc) + ((NV * (size_t)nse * sizeof(T) + 15) & ~(size_t)15));
    // ---- stage ----
    for (int qb = threadIdx.x; qb < nst; qb += BLOCK * U) {
      T r1[U], r2[U], r3[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = qb + u * BLOCK;
        if (q < nst) {
          r1[u] = w[q];
          r2[u] = b[q];
          r3[u] = di[q];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = qb + u * BLOCK;
        if (q < nst) {
          lw[q] = r1[u];
          lb[q] = r2[u];
          ld[q] = r3[u];
        }
      }
    }
    for (int qb = threadIdx.x; qb < nse; qb += BLOCK * U) {
      double rs[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = qb + u * BLOCK;
        if (q < nse) rs[u] = sigma[q];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = qb + u * BLOCK;
        if (q < nse) ls[q] = rs[u];
      }
    }
    for (int q = threadIdx.x; q < kFibStride * g.ey; q += BLOCK) lf[q] = L->fib[0][q];
    __syncthreads();
    // ---- sweep 1 from x = 0 ----
    {
      const T om = wgt(0, 0);
      T* dst = nc == 1 ? out : lx0;
      for (int q = threadIdx.x; q < nst; q += BLOCK) dst[q] = om * lb[q] * ld[q];
      __syncthreads();
    }
#pragma unroll 1
    for (int s = 2; s <= nc; ++s) {
      const T* __restrict__ cur = (s % 2 == 0) ? lx0 : lx1;
      T* nxt = (s % 2 == 0) ? lx1 : lx0;
      // ---- phase A: element contributions of M (w v) + K (theta v) ----
      for (int qb = threadIdx.x; qb < nse; qb += UA * BLOCK) {
        T kv[UA][NV], mv[UA][NV], o4[UA][NV];
        Tensor2<T> D[UA];
#pragma unroll
        for (int h = 0; h < UA; ++h) {
          const int q = qb + h * BLOCK;
          const int qq = q < nse ? q : 0;
          const int r = fdiv(qq, mex);
          const int ex = qq - r * EX;
          D[h] = tensor_from<T, 2>(ls[qq], lf + kFibStride * r, tau, zr);
          const int base = r * nx + ex;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const int o = base + ((v >> 1) & 1) * nx + (v & 1);
            const T a = cur[o], ww = lw[o];
            kv[h][v] = th * a;
            mv[h][v] = ww * a;
          }
        }
#pragma unroll
        for (int h = 0; h < UA; ++h) elem_apply_2d<T>(kv[h], mv[h], D[h], cxx, cyy, cm, o4[h]);
#pragma unroll
        for (int h = 0; h < UA; ++h) {
          const int q = qb + h * BLOCK;
          if (q < nse) {
#pragma unroll
            for (int v = 0; v < NV; ++v) lc[v * nse + q] = o4[h][v];
          }
        }
      }
      __syncthreads();
      // ---- phase B: every node ----
      const T om = wgt(0, s - 1);
      for (int q = threadIdx.x; q < nst; q += BLOCK) {
        const int j = fdiv(q, mnx);
        const int i = q - j * nx;
        T y = T(0);
#pragma unroll
        for (int bb = 0; bb < 2; ++bb) {
          const int ey = j - 1 + bb;
          const bool oky = ey >= 0 && ey < g.ey;
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const int ex = i - 1 + a;
            const bool ok = oky && ex >= 0 && ex < EX;
            const int el = ey * EX + ex;
            const int v = (1 - a) + 2 * (1 - bb);
            const T cv = lc[v * nse + (ok ? el : 0)];
            y += ok ? cv : T(0);
          }
        }
        const T xn = cur[q] + om * (lb[q] - y) * ld[q];
        if (s == nc) out[q] = xn;
        else nxt[q] = xn;
      }
      __syncthreads();
    }
  }

  __device__ __forceinline__ void residual_inner(int l, const TI* __restrict__ b, const TI* __restrict__ x, TI* __restrict__ out) const {
    const int n = L->g[l].n;
    bytes = uni(bytes + (4.0 * sizeof(TI) * n + dbytes(l)));
    const TI* __restrict__ w = mgW(l);
    staged<TI>(
        l, x, w, b, (const TI*)nullptr, KScale<TI>{TI(prm.theta)},
        [](TI a, TI ww) { return ww * a; }, [&](int idx, int, int, int, TI y, TI, TI, TI bo, TI) { gmem(out)[idx] = bo - y; });
  }

  // coarse[l+1] = P^T fine[l]  (full weighting, transpose of Q1 interpolation); G == 1 only
  __device__ __forceinline__ void restrict_to(int l, const TI* __restrict__ rf, TI* __restrict__ bc) const {
    const GridDev& gf = L->g[l];
    const GridDev& gc = L->g[l + 1];
    bytes = uni(bytes + (double(sizeof(TI)) * (gf.n + gc.n)));
    for (int idx = threadIdx.x; idx < gc.n; idx += BLOCK) {
      int I, J, K;
      decode<DIM>(gc, idx, I, J, K);
      TI acc = TI(0);
      const int kz0 = (DIM == 3) ? -1 : 0, kz1 = (DIM == 3) ? 1 : 0;
      for (int c = kz0; c <= kz1; ++c) {
        const int fk = 2 * K + c;
        if (DIM == 3 && (fk < 0 || fk >= gf.nz)) continue;
        const TI wz = (c == 0) ? TI(1) : TI(0.5);
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
          const int fj = 2 * J + b;
          if (fj < 0 || fj >= gf.ny) continue;
          const TI wy = (b == 0) ? TI(1) : TI(0.5);
#pragma unroll
          for (int a = -1; a <= 1; ++a) {
            const int fi = 2 * I + a;
            if (fi < 0 || fi >= gf.nx) continue;
            const TI wx = (a == 0) ? TI(1) : TI(0.5);
            acc += wx * wy * wz * rf[(DIM == 3 ? (fk * gf.ny + fj) : fj) * gf.nx + fi];
          }
        }
      }
      bc[idx] = acc;
    }
    __syncthreads();
  }

  // fine[l] += P coarse[l+1]  (Q1 interpolation of nested grids); G == 1 only
  __device__ __forceinline__ void prolong_add(int l, const TI* __restrict__ xc, TI* __restrict__ xf) const {
    const GridDev& gf = L->g[l];
    const GridDev& gc = L->g[l + 1];
    bytes = uni(bytes + (double(sizeof(TI)) * (2.0 * gf.n + gc.n)));
    for (int idx = threadIdx.x; idx < gf.n; idx += BLOCK) {
      int i, j, k;
      decode<DIM>(gf, idx, i, j, k);
      const int I = i >> 1, J = j >> 1, K = k >> 1;
      const int oi = i & 1, oj = j & 1, ok = (DIM == 3) ? (k & 1) : 0;
      const TI w = (oi ? TI(0.5) : TI(1)) * (oj ? TI(0.5) : TI(1)) * (ok ? TI(0.5) : TI(1));
      TI acc = TI(0);
      for (int c = 0; c <= ok; ++c)
        for (int b = 0; b <= oj; ++b)
          for (int a = 0; a <= oi; ++a) {
            const int q = (DIM == 3) ? (((K + c) * gc.ny + (J + b)) * gc.nx + (I + a)) : ((J + b) * gc.nx + (I + a));
            acc += w * xc[q];
          }
      xf[idx] += acc;
    }
    __syncthreads();
  }

  // weight of sweep s (0-based) of grid l
  __device__ __forceinline__ TI wgt(int l, int s) const {
    if (prm.smoother == 0) return TI(prm.smooth_omega);
    return TI(omega[l * kMaxSweeps + s]);
  }

  // out = V-cycle(b) on grid 0.  Pre- and post-smoothing sweeps alternate
  // between a level's two buffers so that buf[1] is the level's output for any
  // sweep count; the coarsest grid's sweeps start in the buffer that makes the
  // last one land in buf[1].
  __device__ __forceinline__ void vcycle(const TI* __restrict__ b0, TI* __restrict__ out0) const {
    if constexpr (!MG) {
      // sweep s (1-based) of nc writes buf[(nc - s + 1) % 2]: the last one out0
      TI* buf[2] = {mgT(0), out0};
      const int nc = L->sweeps;
      if constexpr (DIM == 3) {
        // sweep s (1-based) of nc writes buf[(nc - s + 1) % 2]: the last one out0
        jacobi(0, b0, nullptr, buf[nc % 2], wgt(0, 0));
        for (int s = 2; s <= nc; ++s) jacobi(0, b0, buf[(nc - s + 2) % 2], buf[(nc - s + 1) % 2], wgt(0, s - 1));
      } else {
        // A one-workgroup team whose grid fits one tile runs every sweep in one
        // pass.  Otherwise the sweeps after the first run as fused pairs (one
        // pass each), and a single sweep when one is left.  Pass t (1-based) of
        // P writes buf[(P - t + 1) % 2]: the last one out0.
        if (G == 1 && (sizeof(TI) == 8 ? L->tile_p8 : L->tile_p4) >= L->g[0].ny) {
          jacobi_resident(b0, out0, nc);
          return;
        }
        // With three or more sweeps the first pass runs sweeps 1 to 3 (the sweep
        // from zero formed while staging).
        const int np = (nc - 1) / 2;
        const int P = nc - np - (nc >= 3 ? 1 : 0);
        int s, t;
        if (nc >= 3) {
          jacobi_pair(nullptr, b0, buf[P % 2], wgt(0, 0), wgt(0, 1), wgt(0, 2));
          s = 4;
        } else {
          jacobi(0, b0, nullptr, buf[P % 2], wgt(0, 0));
          s = 2;
        }
        t = 2;
        for (; s + 1 <= nc; s += 2, ++t)
          jacobi_pair(buf[(P - t + 2) % 2], b0, buf[(P - t + 1) % 2], TI(0), wgt(0, s - 1), wgt(0, s));
        for (; s <= nc; ++s, ++t) jacobi(0, b0, buf[(P - t + 2) % 2], buf[(P - t + 1) % 2], wgt(0, s - 1));
      }
      return;
    }
    const int nmg = L->nmg;
    const int nu = prm.smooth_steps;
    for (int l = 0; l < nmg - 1; ++l) {
      TI* buf[2] = {mgT(l), l == 0 ? out0 : mgX(l)};
      const TI* b = (l == 0) ? b0 : mgB(l);
      jacobi(l, b, nullptr, buf[0], wgt(l, 0));
      for (int s = 2; s <= nu; ++s) jacobi(l, b, buf[s % 2], buf[(s - 1) % 2], wgt(l, s - 1));
      residual_inner(l, b, buf[(nu - 1) % 2], buf[nu % 2]);
      restrict_to(l, buf[nu % 2], mgB(l + 1));
    }
    {
      // coarsest grid: sweep s of nc writes buf[(nc - s + 1) % 2], the last buf[1]
      const int l = nmg - 1;
      TI* buf[2] = {mgT(l), l == 0 ? out0 : mgX(l)};
      const TI* b = (l == 0) ? b0 : mgB(l);
      const int nc = L->sweeps;
      jacobi(l, b, nullptr, buf[nc % 2], wgt(l, 0));
      for (int s = 2; s <= nc; ++s) jacobi(l, b, buf[(nc - s + 2) % 2], buf[(nc - s + 1) % 2], wgt(l, s - 1));
    }
    for (int l = nmg - 2; l >= 0; --l) {
      TI* buf[2] = {mgT(l), l == 0 ? out0 : mgX(l)};
      const TI* b = (l == 0) ? b0 : mgB(l);
      prolong_add(l, mgX(l + 1), buf[(nu - 1) % 2]);
      for (int t = 1; t <= nu; ++t) jacobi(l, b, buf[(nu - 2 + t) % 2], buf[(nu - 1 + t) % 2], wgt(l, nu - t));
    }
  }

  // lmax of D^-1 A_l by power iteration.
  // Uses buffers x0, x1 of grid l.  Returns the estimate (team-uniform).
  __device__ __forceinline__ double power_lmax(int l, TI* x0, TI* x1) const {
    const GridDev& g = L->g[l];
    const int nb = l == 0 ? nband() : g.n;  // coarse grids: one-workgroup teams own every node
    // Start: a constant plus per-node pseudo-random values in [-1/2, 1/2) (a
    // multiplicative hash of the node index, the same on every member).  When
    // the stiffness dominates A, the largest eigenvalues of D^-1 A belong to
    // modes that alternate along one axis only (Q1 in 2D and 3D); a start
    // without them, such as a checkerboard, underestimates lmax, and the
    // Chebyshev sweeps then amplify those modes.  Pseudo-random values contain
    // every mode.
    for (int q = threadIdx.x; q < nb; q += BLOCK) {
      const int idx = l == 0 ? bidx(q) : q;
      const unsigned hsh = (unsigned)idx * 2654435761u;
      x0[idx] = TI(1.0 + double(hsh >> 8) * (1.0 / 16777216.0) - 0.5);
    }
    sync();
    double lam = 0.0;
    const TI* __restrict__ w = mgW(l);
    const TI* __restrict__ di = mgI(l);
    for (int it = 0; it < prm.power_iters; ++it) {
      double nn[2] = {0.0, 0.0};
      staged<TI>(
          l, x0, w, di, (const TI*)nullptr, KScale<TI>{TI(prm.theta)},
          [](TI a, TI ww) { return ww * a; },
          [&](int idx, int, int, int, TI ax, TI xown, TI, TI dio, TI) {
            const TI y = ax * dio;
            gmem(x1)[idx] = y;
            nn[0] += double(y) * double(y);
            nn[1] += double(xown) * double(xown);
          });
      tsum<2>(nn);
      lam = sqrt(nn[0] / nn[1]);
      const TI scl = TI(1.0 / sqrt(nn[0]));
      for (int q = threadIdx.x; q < nb; q += BLOCK) {
        const int idx = l == 0 ? bidx(q) : q;
        x0[idx] = x1[idx] * scl;
      }
      sync();
    }
    bytes = uni(bytes + (prm.power_iters * (5.0 * sizeof(TI) * g.n + dbytes(l))));
    return lam;
  }
};

// Weights 1 / xi_s, xi_s the roots of the degree-K Chebyshev polynomial
// shifted to [a, b], ordered to alternate large and small roots.
__device__ inline void chebyshev_weights(double a, double b, int K, double* w) {
  const double th = 0.5 * (b + a), de = 0.5 * (b - a);
  const double PI = 3.14159265358979323846;
  for (int s = 0; s < K; ++s) {
    const int r = (s % 2 == 0) ? s / 2 : K - 1 - s / 2;
    const double xi = th + de * cos(PI * (2 * r + 1) / (2.0 * K));
    w[s] = 1.0 / xi;
  }
}

template <typename TI, int DIM, int BLOCK, bool MG>
__global__ __launch_bounds__(BLOCK) void st_team_kernel(const LevelDev* __restrict__ levels,
                                                        const TeamTask* __restrict__ tasks, SolverParams prm) {
  constexpr int NW = BLOCK / kWave;
  extern __shared__ __align__(16) unsigned char smem_dyn[];
  __shared__ double red[NW * 9];
  __shared__ double H[(kMaxRestart + 1) * kMaxRestart];
  __shared__ double cs_[kMaxRestart], sn_[kMaxRestart], gv[kMaxRestart + 1], sc[kMaxRestart + 1];
  __shared__ double yv[kMaxRestart], coef[kMaxRestart + 1];
  __shared__ double omega_tab[kMaxMG * kMaxSweeps];
  __shared__ double sh_resid;
#ifdef STM_PHASE_TIMERS
  __shared__ long long ph_acc[8];
  if (threadIdx.x < 8) ph_acc[threadIdx.x] = 0;
  __syncthreads();
#endif

  const TeamTask task = tasks[blockIdx.x];
  const LevelDev* L = levels + task.level;
  const int tid = threadIdx.x;

  Team<TI, DIM, BLOCK, MG> tm;
  tm.L = L;
  tm.prm = prm;
  tm.work = task.work;
  tm.smem = smem_dyn;
  tm.omega = omega_tab;
  tm.red = red;
  tm.bytes = 0.0;
  tm.rank = task.rank;
  tm.G = task.G;
  tm.bar = task.bar;
  tm.part = task.part;
  tm.fault = task.fault;
  tm.gen = 0;
  tm.rslot = 0;
  tm.broken = false;
#ifdef STM_PHASE_TIMERS
  tm.ph = ph_acc;
#endif
  const GridDev g0 = L->g[0];
  tm.set_box();
  const int n0 = g0.n;
  const int nb = tm.nband();
  double* __restrict__ u = reinterpret_cast<double*>(task.work + L->off_u);
  double* __restrict__ uprev = reinterpret_cast<double*>(task.work + L->off_uprev);
  double* __restrict__ wk1 = reinterpret_cast<double*>(task.work + L->off_wk1);
  double* __restrict__ tact = reinterpret_cast<double*>(task.work + L->off_tact);
  double* __restrict__ dlt = reinterpret_cast<double*>(task.work + L->off_dlt);
  tm.V = reinterpret_cast<TI*>(task.work + L->off_V);
  tm.kdiag0 = reinterpret_cast<double*>(task.work + L->off_kd);
  tm.dinv = reinterpret_cast<TI*>(task.work + L->off_dinv);
  tm.w0 = reinterpret_cast<TI*>(task.work + L->off_mgW[0]);
  tm.Z = reinterpret_cast<TI*>(task.work + L->off_Z);
  const int64_t vs = (int64_t)((n0 + 63) & ~63);
  tm.vstride = vs;
  double* ubuf = reinterpret_cast<double*>(task.work + L->off_U);

  const int m = L->m;
  const double dt = uni(L->dt), inv_dt = uni(1.0 / L->dt);
  const double kr = uni(prm.k_react), ar = uni(prm.a_react), tau = uni(prm.tau), thr = uni(prm.threshold);
  const double zr = uni(prm.zr);
  const double th = uni(prm.theta);
  const int restart = prm.restart;

  bool have_prev = false;
  const double* prevU = nullptr;

  for (int it_s = 0; it_s < task.count; ++it_s) {
    const int s = task.order ? task.order[task.first + it_s * task.stride] : task.first + it_s * task.stride;
    const long long t_start = wall_clock64();
    tm.bytes = 0.0;
    tm.sigma = task.sigma + (int64_t)s * g0.ne;
    double* Uout = task.u_out ? task.u_out + (int64_t)s * m * n0 : ubuf;
    const double* W = nullptr;
    if (task.u_guess) W = task.u_guess + (int64_t)s * m * n0;
    else if (have_prev) W = prevU;

    tm.setup_operator();
    // initial state, activation markers, warm-start history
    tm.bytes = uni(tm.bytes + ((24.0 + sizeof(TI) + 24.0) * n0));
    for (int q = tid; q < nb; q += BLOCK) {
      const int idx = tm.bidx(q);
      const double v = L->u0[idx];
      uprev[idx] = v;
      wk1[idx] = v;
      tact[idx] = (v >= thr) ? 0.0 : -1.0;
    }
    tm.sync();

    long long newton_total = 0, krylov_total = 0, damped = 0;
    int newton_max_slab = 0, status = 0;
    // bytes by the per-step word model: 4 float64 words per residual; per
    // Krylov iteration j, 4 (Jacobian product) + the preconditioner's words
    // (5 per sweep and per coarse-grid residual, weighted by the grid's nodes)
    // + 2j + 3 (Arnoldi step) inner words, per node
    double model_bytes = 0.0;
    const double krylov_words = 7.0 + L->pc_words;
    double worst_final = 0.0;
    bool weights_ready = (prm.smoother == 0);

    for (int k = 0; k < m; ++k) {
      // ---- initial iterate of slab k ----
      const double* Wk = W ? W + (int64_t)k * n0 : nullptr;
      tm.bytes = uni(tm.bytes + ((Wk ? 40.0 : 16.0) * n0));
      for (int q = tid; q < nb; q += BLOCK) {
        const int idx = tm.bidx(q);
        if (Wk) {
          const double w = Wk[idx];
          u[idx] = uprev[idx] + (w - wk1[idx]);
          wk1[idx] = w;
        } else {
          u[idx] = uprev[idx];
        }
      }
      tm.sync();

      double dprev = 0.0, eta = fmax(prm.gmres_rtol, 1e-5);
      int it = 0;
      bool conv = false;
      double dmax = 0.0;
      // damping: the residual 2-norm of the last accepted iterate and the
      // fraction of the last Newton step in u (halved while the residual grows)
      double beta_acc = 0.0, tstep = 1.0;
      for (; it < prm.newton_max; ++it) {
        // ---- residual (float64) -> V_0, Jacobian weights on every grid ----
        TI* V0 = tm.V;
        TI* w0 = tm.mgW(0);
        double rr[1] = {0.0};
        STM_T0(t_res);
        tm.bytes = uni(tm.bytes + (24.0 * n0 + 8.0 * g0.ne + 3.0 * sizeof(TI) * n0));
        for (int l = 1; l < L->nmg; ++l) tm.bytes = uni(tm.bytes + ((8.0 + sizeof(TI)) * L->g[l].n));
        {
          TI* __restrict__ di = tm.dinv;
          const double cmd = (DIM == 3) ? 8.0 * g0.hx * g0.hy * g0.hz / 216.0 : 4.0 * g0.hx * g0.hy / 36.0;
          tm.template staged<double>(
              0, u, uprev, tm.kdiag0, (const double*)nullptr,
              [th](double a, double b) { return th * a + (1.0 - th) * b; },
              [&](double a, double b) { return (a - b) * inv_dt - react(a, kr, ar); },
              [&](int idx, int i, int j, int k, double y, double uown, double, double kd, double) {
                const double r = -y;
                const double w = inv_dt - react_d(uown, kr, ar);
                gmem(V0)[idx] = TI(r);
                gmem(w0)[idx] = TI(w);
                gmem(di)[idx] = TI(1.0 / (th * kd + tm.nel(0, i, j, k) * cmd * w));
                rr[0] += r * r;
              });
        }
        tm.coarse_weights(u, inv_dt);
        tm.template tsum<1>(rr);  // its barriers also publish the writes above
        STM_T1(t_res, 0);
        model_bytes = uni(model_bytes + 32.0 * n0);
        const double beta = uni(sqrt(rr[0]));
        if (!isfinite(beta) && !(prm.damping && it > 0 && tstep > kMinStep)) {
          status = -5;
          break;
        }
        if (beta == 0.0) {
          conv = true;
          dmax = 0.0;
          break;
        }
        // the last step made the residual grow (or not finite): take half of
        // it back, u -= (t/2) delta, and evaluate again (Armijo-style halving
        // down to kMinStep; the pass counts as a Newton iteration)
        if (prm.damping && it > 0 && !(beta <= beta_acc) && tstep > kMinStep) {
          tstep = uni(0.5 * tstep);
          for (int q = tid; q < nb; q += BLOCK) {
            const int idx = tm.bidx(q);
            u[idx] -= tstep * dlt[idx];
          }
          tm.bytes = uni(tm.bytes + 24.0 * n0);
          dmax = uni(0.5 * dmax);
          ++damped;
          tm.sync();
          continue;
        }
        beta_acc = beta;
        tstep = 1.0;
        // ---- smoother weights: once per sample, from the first slab operator ----
        if (!weights_ready) {
          for (int l = 0; l < (MG ? L->nmg : 1); ++l) {
            TI* x0 = (l == 0) ? tm.V + vs : tm.mgX(l);
            TI* x1 = (l == 0) ? tm.V + 2 * vs : tm.mgT(l);
            const double lmax = 1.05 * tm.power_lmax(l, x0, x1);
            const int K = (l == L->nmg - 1) ? L->sweeps : prm.smooth_steps;
            if (tid == 0) chebyshev_weights(lmax / L->cheb_ratio, lmax, K, omega_tab + l * kMaxSweeps);
          }
          __syncthreads();
          weights_ready = true;
        }

        // ---- GMRES(restart), right-preconditioned by the V-cycle ----
        if (tid == 0) {
          sc[0] = 1.0 / beta;
          gv[0] = beta;
        }
        __syncthreads();
        const double tol_abs = uni(eta * beta);
        int jdim = 0;
        for (int j = 0; j < restart; ++j) {
          TI* Vj = tm.V + j * vs;
          TI* Zj = tm.Z + j * vs;
          TI* Vn = tm.V + (j + 1) * vs;
          model_bytes = uni(model_bytes + double(sizeof(TI)) * n0 * (krylov_words + 2.0 * j));
          STM_T0(t_vc);
          tm.vcycle(Vj, Zj);
          STM_T1(t_vc, 1);
          STM_T0(t_pa);
          // pass A: ws = A Z_j (into V_{j+1})
          tm.bytes = uni(tm.bytes + (3.0 * sizeof(TI) * n0 + tm.dbytes(0)));
          tm.template staged<TI>(
              0, Zj, tm.mgW(0), (const TI*)nullptr, (const TI*)nullptr, KScale<TI>{TI(prm.theta)},
              [](TI a, TI ww) { return ww * a; },
              [&](int idx, int, int, int, TI w, TI, TI, TI, TI) { gmem(Vn)[idx] = w; });
          STM_T1(t_pa, 2);
          // Classical Gram-Schmidt against V_0..V_j, done twice when the inner
          // vectors are float32 (CGS2: the second pass restores the orthogonality
          // the first loses to rounding); each pass adds its projections to
          // column j of H.
          double nn[1] = {0.0};
          constexpr int kPasses = sizeof(TI) == 4 ? 2 : 1;
          // dots of the next pass, accumulated by the first pass's update
          double dnext[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
          bool have_dots = false;
#pragma unroll 1
          for (int pass = 0; pass < kPasses; ++pass) {
            STM_T0(t_dot);
            // dots with V_0..V_min(j,7) over the owned nodes: batched loads
            double d[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) d[q] = have_dots ? dnext[q] : 0.0;
            const int nk0 = min(j + 1, 8);
            if (!have_dots) {
              tm.bytes = uni(tm.bytes + ((1.0 + nk0) * sizeof(TI) * n0));
              const TI* __restrict__ Vb = tm.V;
              const TI* __restrict__ Vr = Vn;
              for (int qb = tid; qb < nb; qb += BLOCK * 2) {
                TI wv[2], vv[2][8];
#pragma unroll
                for (int uu = 0; uu < 2; ++uu) {
                  const int q = qb + uu * BLOCK;
                  const int idx = q < nb ? tm.bidx(q) : 0;
                  wv[uu] = q < nb ? Vr[idx] : TI(0);
#pragma unroll
                  for (int p = 0; p < 8; ++p) vv[uu][p] = (p < nk0 && q < nb) ? Vb[p * vs + idx] : TI(0);
                }
#pragma unroll
                for (int uu = 0; uu < 2; ++uu)
#pragma unroll
                  for (int p = 0; p < 8; ++p) d[p] += double(vv[uu][p]) * double(wv[uu]);
              }
            }
            tm.template tsum<9>(d);
            if (tid == 0) {
#pragma unroll
              for (int q = 0; q < 8; ++q)
                if (q < nk0) coef[q] = d[q];
            }
            for (int k0 = 8; k0 <= j; k0 += 8) {  // remaining dot chunks
              const int nk = min(j + 1 - k0, 8);
              tm.bytes = uni(tm.bytes + ((1.0 + nk) * sizeof(TI) * n0));
#pragma unroll
              for (int q = 0; q < 9; ++q) d[q] = 0.0;
              for (int q = tid; q < nb; q += BLOCK) {
                const int idx = tm.bidx(q);
                const double wd = double(Vn[idx]);
#pragma unroll
                for (int p = 0; p < 8; ++p)
                  if (p < nk) d[p] += double(tm.V[(k0 + p) * vs + idx]) * wd;
              }
              tm.template tsum<9>(d);
              if (tid == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                  if (q < nk) coef[k0 + q] = d[q];
              }
            }
            // projections onto the normalised basis enter H; V_q is stored with
            // norm 1/sc[q], so w loses (sc[q]^2 <V_q, w>) V_q
            if (tid == 0)
              for (int q = 0; q <= j; ++q) {
                const double hq = sc[q] * sc[j] * coef[q];
                H[q * kMaxRestart + j] = (pass ? H[q * kMaxRestart + j] : 0.0) + hq;
                coef[q] = sc[q] * sc[q] * coef[q];
              }
            __syncthreads();
            STM_T1(t_dot, 3);
            STM_T0(t_pb);
            // pass B: V_{j+1} -= sum_q coef_q V_q over the owned nodes; norm
            nn[0] = 0.0;
            tm.bytes = uni(tm.bytes + ((j + 3.0) * sizeof(TI) * n0));
            // The first of two passes with at most 8 basis vectors also forms
            // the second pass's dots from the values it holds: the same nodes
            // per thread, the same operations in the same order as the
            // separate loops, one read of the vectors fewer.
            const bool fuse = pass + 1 < kPasses && j < 8;
            if (fuse) {
#pragma unroll
              for (int q = 0; q < 9; ++q) dnext[q] = 0.0;
              for (int qb = tid; qb < nb; qb += BLOCK * 2) {
                double w[2];
                int ix[2];
                TI vv[2][8];
#pragma unroll
                for (int uu = 0; uu < 2; ++uu) {
                  const int q = qb + uu * BLOCK;
                  ix[uu] = q < nb ? tm.bidx(q) : 0;
                  w[uu] = q < nb ? double(Vn[ix[uu]]) : 0.0;
#pragma unroll
                  for (int p = 0; p < 8; ++p) vv[uu][p] = (p <= j && q < nb) ? tm.V[p * vs + ix[uu]] : TI(0);
                }
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                  const double cq = p <= j ? coef[p] : 0.0;
#pragma unroll
                  for (int uu = 0; uu < 2; ++uu) w[uu] -= cq * double(vv[uu][p]);
                }
                TI wt[2];
#pragma unroll
                for (int uu = 0; uu < 2; ++uu) {
                  wt[uu] = TI(0);
                  if (qb + uu * BLOCK < nb) {
                    wt[uu] = TI(w[uu]);
                    Vn[ix[uu]] = wt[uu];
                  }
                }
#pragma unroll
                for (int uu = 0; uu < 2; ++uu)
#pragma unroll
                  for (int p = 0; p < 8; ++p) dnext[p] += double(vv[uu][p]) * double(wt[uu]);
              }
            } else {
              // vectors in chunks of 4, all loads of a chunk issued before use
              for (int qb = tid; qb < nb; qb += BLOCK * 2) {
                double w[2];
                int ix[2];
#pragma unroll
                for (int uu = 0; uu < 2; ++uu) {
                  const int q = qb + uu * BLOCK;
                  ix[uu] = q < nb ? tm.bidx(q) : 0;
                  w[uu] = q < nb ? double(Vn[ix[uu]]) : 0.0;
                }
                for (int q0 = 0; q0 <= j; q0 += 4) {
                  TI vv[4][2];
#pragma unroll
                  for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int uu = 0; uu < 2; ++uu)
                      vv[p][uu] = (q0 + p <= j) ? tm.V[(q0 + p) * vs + ix[uu]] : TI(0);
#pragma unroll
                  for (int p = 0; p < 4; ++p) {
                    const double cq = (q0 + p <= j) ? coef[q0 + p] : 0.0;
#pragma unroll
                    for (int uu = 0; uu < 2; ++uu) w[uu] -= cq * double(vv[p][uu]);
                  }
                }
#pragma unroll
                for (int uu = 0; uu < 2; ++uu) {
                  if (qb + uu * BLOCK < nb) {
                    const TI wt = TI(w[uu]);
                    Vn[ix[uu]] = wt;
                    nn[0] += double(wt) * double(wt);
                  }
                }
              }
            }
            // Only the last pass's norm is used.  A member reads V_{j+1} at
            // its own nodes only, and in the same thread-to-node order as it
            // wrote them, so the first pass ends with a workgroup barrier.
            have_dots = fuse;
            if (pass + 1 < kPasses)
              __syncthreads();
            else
              tm.template tsum<1>(nn);
            STM_T1(t_pb, 4);
          }
          const double hn = uni(sqrt(nn[0]));
          if (tid == 0) {
            const double hj1 = sc[j] * hn;
            sc[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
            for (int q = 0; q < j; ++q) {  // previous rotations on column j
              const double a = H[q * kMaxRestart + j], b = H[(q + 1) * kMaxRestart + j];
              H[q * kMaxRestart + j] = cs_[q] * a + sn_[q] * b;
              H[(q + 1) * kMaxRestart + j] = -sn_[q] * a + cs_[q] * b;
            }
            const double a = H[j * kMaxRestart + j];
            const double r = sqrt(a * a + hj1 * hj1);
            const double c = r > 0.0 ? a / r : 1.0, sn = r > 0.0 ? hj1 / r : 0.0;
            cs_[j] = c;
            sn_[j] = sn;
            H[j * kMaxRestart + j] = r;
            H[(j + 1) * kMaxRestart + j] = 0.0;
            gv[j + 1] = -sn * gv[j];
            gv[j] = c * gv[j];
            sh_resid = fabs(gv[j + 1]);
          }
          __syncthreads();
          jdim = j + 1;
          const double resid = uni(sh_resid);
          if (!(resid > tol_abs) || !(hn > 0.0)) break;
        }
        krylov_total += jdim;
        if (tid == 0) {
          for (int q = jdim - 1; q >= 0; --q) {
            double acc = gv[q];
            for (int p = q + 1; p < jdim; ++p) acc -= H[q * kMaxRestart + p] * yv[p];
            yv[q] = acc / H[q * kMaxRestart + q];
          }
          for (int q = 0; q < jdim; ++q) coef[q] = yv[q] * sc[q];
        }
        __syncthreads();
        // ---- u += sum_q y_q z_q (float64) over the owned nodes, max-norm of the step ----
        STM_T0(t_up);
        double dm = 0.0;
        tm.bytes = uni(tm.bytes + (double(jdim) * sizeof(TI) * n0 + 24.0 * n0));
        for (int qb = tid; qb < nb; qb += BLOCK * 2) {
          double dl[2] = {0.0, 0.0}, uo[2];
          int ix[2];
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            const int q = qb + v * BLOCK;
            ix[v] = q < nb ? tm.bidx(q) : 0;
            uo[v] = q < nb ? u[ix[v]] : 0.0;
          }
          for (int q0 = 0; q0 < jdim; q0 += 4) {
            TI zz[4][2];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
              for (int v = 0; v < 2; ++v) zz[p][v] = (q0 + p < jdim) ? tm.Z[(q0 + p) * vs + ix[v]] : TI(0);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
              const double cq = (q0 + p < jdim) ? coef[q0 + p] : 0.0;
#pragma unroll
              for (int v = 0; v < 2; ++v) dl[v] += cq * double(zz[p][v]);
            }
          }
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            if (qb + v * BLOCK < nb) {
              u[ix[v]] = uo[v] + dl[v];
              dlt[ix[v]] = dl[v];
              dm = fmax(dm, fabs(dl[v]));
            }
          }
        }
        dmax = uni(tm.tmax(dm));  // its barrier also publishes u to the other members
        STM_T1(t_up, 5);
        const double ach = sh_resid / beta;
        if (!isfinite(dmax)) {
          status = -5;
          break;
        }
        if (dmax <= prm.newton_tol) {
          conv = true;
          ++it;
          break;
        }
        if (it >= 1) {
          const double ratio = dmax / dprev;
          const double pred = dmax * fmax(ratio * ratio, 10.0 * ach);
          if (ratio < 0.5 && pred <= 0.1 * prm.newton_tol) {
            conv = true;
            ++it;
            break;
          }
        }
        dprev = uni(dmax);
        eta = uni(fmax(prm.gmres_rtol, fmin(1e-4, 0.01 * dmax)));
      }
      if (status == -5) break;
      if (!conv && status == 0) status = -4;
      newton_total += it;
      newton_max_slab = max(newton_max_slab, it);
      worst_final = uni(fmax(worst_final, dmax));

      // ---- accept slab k: store, activation crossing, shift history ----
      double* Uk = Uout + (int64_t)k * n0;
      const double tk = k * dt;
      tm.bytes = uni(tm.bytes + (40.0 * n0));
      for (int q = tid; q < nb; q += BLOCK) {
        const int idx = tm.bidx(q);
        const double un = u[idx], up = uprev[idx];
        Uk[idx] = un;
        if (tact[idx] < 0.0 && un >= thr) tact[idx] = tk + dt * (thr - up) / (un - up);
        uprev[idx] = un;
      }
      tm.sync();
    }

    // ---- finalize the sample ----
    double cen[1] = {0.0};
    for (int q = tid; q < nb; q += BLOCK) {
      const int idx = tm.bidx(q);
      double t = tact[idx];
      if (t < 0.0) {
        t = L->T;
        cen[0] += 1.0;
      }
      if (task.t_act) task.t_act[(int64_t)s * n0 + idx] = t;
    }
    tm.template tsum<1>(cen);
    if (tid == 0 && task.stats && task.rank == 0) {
      SampleStatsDev st;
      st.status = tm.broken ? -3 : status;
      st.newton_max_per_slab = newton_max_slab;
      st.newton_iters = newton_total;
      st.krylov_iters = krylov_total;
      st.final_step = worst_final;
      st.ticks = wall_clock64() - t_start;
      st.censored = (int)cen[0];
      st.damped = (int)damped;
      st.alg_bytes = tm.bytes;
      st.model_bytes = model_bytes;
      for (int q = 0; q < 8; ++q) st.phase_ticks[q] = 0;
#ifdef STM_PHASE_TIMERS
      for (int q = 0; q < 8; ++q) st.phase_ticks[q] = ph_acc[q];
#endif
      task.stats[s] = st;
    }
#ifdef STM_PHASE_TIMERS
    __syncthreads();
    if (threadIdx.x < 8) ph_acc[threadIdx.x] = 0;
#endif
    prevU = Uout;
    have_prev = (status == 0);
    tm.sync();
  }
}

// ---------------------------------------------------------------------------
// Global space-time solve (Sec. 3.2 eq. system_C, Sec. 3.5): Newton on the
// whole space-time system at once.  Each linear step J delta = -R is one GMRES
// over all m slabs, right-preconditioned by forward substitution in time in
// which every diagonal block is replaced by the slab preconditioner (one
// V-cycle, or the Chebyshev-weighted sweeps):
//   z_0 = P_0^-1 r_0,  z_k = P_k^-1 (r_k - B z_{k-1}),  B = -M/dt + (1 - theta) K.
// The residual and the product J x = (A_k x_k + B x_{k-1})_k treat every slab
// on its own (the parallel-in-time part of the method); the preconditioner
// sweeps the slabs in order.  The step is added in float64 and halved while
// the residual 2-norm grows, as in the slab solve; the first iterate is the
// lane's previous solution or the caller's guess, else the initial state at
// every time level.  Teams, tasks and statistics as in st_team_kernel
// (newton_max_per_slab is the number of global Newton steps).
// ---------------------------------------------------------------------------
template <typename TI, int DIM, int BLOCK, bool MG>
__global__ __launch_bounds__(BLOCK) void st_global_kernel(const LevelDev* __restrict__ levels,
                                                          const TeamTask* __restrict__ tasks, SolverParams prm) {
  constexpr int NW = BLOCK / kWave;
  extern __shared__ __align__(16) unsigned char smem_dyn[];
  __shared__ double red[NW * 9];
  __shared__ double H[(kMaxRestart + 1) * kMaxRestart];
  __shared__ double cs_[kMaxRestart], sn_[kMaxRestart], gv[kMaxRestart + 1], sc[kMaxRestart + 1];
  __shared__ double yv[kMaxRestart], coef[kMaxRestart + 1];
  __shared__ double omega_tab[kMaxMG * kMaxSweeps];
  __shared__ double sh_resid;
#ifdef STM_PHASE_TIMERS
  __shared__ long long ph_acc[8];
  if (threadIdx.x < 8) ph_acc[threadIdx.x] = 0;
  __syncthreads();
#endif

  const TeamTask task = tasks[blockIdx.x];
  const LevelDev* L = levels + task.level;
  const int tid = threadIdx.x;

  Team<TI, DIM, BLOCK, MG> tm;
  tm.L = L;
  tm.prm = prm;
  tm.work = task.work;
  tm.smem = smem_dyn;
  tm.omega = omega_tab;
  tm.red = red;
  tm.bytes = 0.0;
  tm.rank = task.rank;
  tm.G = task.G;
  tm.bar = task.bar;
  tm.part = task.part;
  tm.fault = task.fault;
  tm.gen = 0;
  tm.rslot = 0;
  tm.broken = false;
#ifdef STM_PHASE_TIMERS
  tm.ph = ph_acc;
#endif
  const GridDev g0 = L->g[0];
  tm.set_box();
  const int n0 = g0.n;
  const int nb = tm.nband();
  double* __restrict__ tact = reinterpret_cast<double*>(task.work + L->off_tact);
  tm.V = reinterpret_cast<TI*>(task.work + L->off_V);  // slab-sized scratch of the power iteration
  tm.Z = reinterpret_cast<TI*>(task.work + L->off_Z);
  tm.kdiag0 = reinterpret_cast<double*>(task.work + L->off_kd);
  tm.dinv = reinterpret_cast<TI*>(task.work + L->off_dinv);
  tm.w0 = reinterpret_cast<TI*>(task.work + L->off_mgW[0]);
  const int64_t vs = (int64_t)((n0 + 63) & ~63);
  tm.vstride = vs;
  const int m = L->m;
  const int64_t gs = (int64_t)m * vs;  // stride of space-time vectors
  TI* __restrict__ gV = reinterpret_cast<TI*>(task.work + L->off_gV);
  TI* __restrict__ gW = reinterpret_cast<TI*>(task.work + L->off_gW);
  TI* __restrict__ gD = reinterpret_cast<TI*>(task.work + L->off_gD);
  TI* __restrict__ gZ = reinterpret_cast<TI*>(task.work + L->off_gZ);
  TI* __restrict__ gT = reinterpret_cast<TI*>(task.work + L->off_gT);
  double* ubuf = reinterpret_cast<double*>(task.work + L->off_U);

  const double dt = uni(L->dt), inv_dt = uni(1.0 / L->dt);
  const double kr = uni(prm.k_react), ar = uni(prm.a_react), thr = uni(prm.threshold);
  const double th = uni(prm.theta);
  const double cmd = (DIM == 3) ? 8.0 * g0.hx * g0.hy * g0.hz / 216.0 : 4.0 * g0.hx * g0.hy / 36.0;
  const int restart = prm.restart;

  bool have_prev = false;
  const double* prevU = nullptr;

  for (int it_s = 0; it_s < task.count; ++it_s) {
    const int s = task.order ? task.order[task.first + it_s * task.stride] : task.first + it_s * task.stride;
    const long long t_start = wall_clock64();
    tm.bytes = 0.0;
    tm.sigma = task.sigma + (int64_t)s * g0.ne;
    double* __restrict__ U = task.u_out ? task.u_out + (int64_t)s * m * n0 : ubuf;
    const double* W = nullptr;
    if (task.u_guess) W = task.u_guess + (int64_t)s * m * n0;
    else if (have_prev) W = prevU;

    tm.setup_operator();
    // first iterate: the guess, else the initial state at every time level
    tm.bytes = uni(tm.bytes + 16.0 * (double)m * n0);
    for (int k = 0; k < m; ++k)
      for (int q = tid; q < nb; q += BLOCK) {
        const int idx = tm.bidx(q);
        U[(int64_t)k * n0 + idx] = W ? W[(int64_t)k * n0 + idx] : L->u0[idx];
      }
    tm.sync();

    // z = P^-1 r over the space-time vectors r, z: forward substitution in time
    auto precond = [&](const TI* __restrict__ r, TI* __restrict__ z) {
      for (int k = 0; k < m; ++k) {
        tm.w0 = gW + k * vs;
        tm.dinv = gD + k * vs;
        if (MG) tm.coarse_weights(U + (int64_t)k * n0, inv_dt);
        const TI* b = r + k * vs;
        if (k > 0) {
          tm.template staged<TI>(
              0, z + (k - 1) * vs, r + k * vs, (const TI*)nullptr, (const TI*)nullptr,
              KScale<TI>{TI(1.0 - th)}, [c0 = TI(-inv_dt)](TI a, TI) { return c0 * a; },
              [&](int idx, int, int, int, TI y, TI, TI ro, TI, TI) { gmem(gT)[idx] = ro - y; });
          b = gT;
        }
        tm.vcycle(b, z + k * vs);
      }
    };
    // y = J x: slab products and the coupling to the previous slab
    auto spmv = [&](const TI* __restrict__ x, TI* __restrict__ y) {
      for (int k = 0; k < m; ++k) {
        TI* yk = y + k * vs;
        tm.template staged<TI>(
            0, x + k * vs, gW + k * vs, (const TI*)nullptr, (const TI*)nullptr,
            KScale<TI>{TI(th)}, [](TI a, TI ww) { return ww * a; },
            [&](int idx, int, int, int, TI v, TI, TI, TI, TI) { gmem(yk)[idx] = v; });
        if (k > 0)
          // in place: f1 = y_k enters only the body (its own node), never the element terms
          tm.template staged<TI>(
              0, x + (k - 1) * vs, yk, (const TI*)nullptr, (const TI*)nullptr,
              KScale<TI>{TI(1.0 - th)}, [c0 = TI(-inv_dt)](TI a, TI) { return c0 * a; },
              [&](int idx, int, int, int, TI v, TI, TI yo, TI, TI) { gmem(yk)[idx] = yo + v; });
      }
    };

    long long krylov_total = 0, damped = 0;
    int status = 0;
    // per-step word model: 4 float64 words per node and slab per residual; per
    // Krylov iteration j, per node and slab: 4 (slab product) + 4 (coupling) +
    // 4 (coupling in the substitution) + the slab preconditioner's words +
    // 2j + 3 (Arnoldi step) inner words
    double model_bytes = 0.0;
    const double krylov_words = 15.0 + L->pc_words;
    const double nm = (double)m * n0;
    bool weights_ready = (prm.smoother == 0);
    double dprev = 0.0, eta = fmax(prm.gmres_rtol, 1e-5), dmax = 0.0;
    double beta_acc = 0.0, tstep = 1.0;
    bool conv = false;
    int it = 0;
    for (; it < prm.newton_max; ++it) {
      // ---- residual of every slab (float64) -> V_0 = -R, weights and inverse diagonals ----
      double rr[1] = {0.0};
      tm.bytes = uni(tm.bytes + (24.0 * nm + 8.0 * g0.ne * m + 3.0 * sizeof(TI) * nm));
      for (int k = 0; k < m; ++k) {
        const double* uk = U + (int64_t)k * n0;
        const double* up = k ? U + (int64_t)(k - 1) * n0 : L->u0;
        TI* Vk = gV + k * vs;
        TI* wk = gW + k * vs;
        TI* dk = gD + k * vs;
        tm.template staged<double>(
            0, uk, up, tm.kdiag0, (const double*)nullptr,
            [th](double a, double b) { return th * a + (1.0 - th) * b; },
            [&](double a, double b) { return (a - b) * inv_dt - react(a, kr, ar); },
            [&](int idx, int i, int j, int kk, double y, double uown, double, double kd, double) {
              const double r = -y;
              const double w = inv_dt - react_d(uown, kr, ar);
              gmem(Vk)[idx] = TI(r);
              gmem(wk)[idx] = TI(w);
              gmem(dk)[idx] = TI(1.0 / (th * kd + tm.nel(0, i, j, kk) * cmd * w));
              rr[0] += r * r;
            });
      }
      tm.template tsum<1>(rr);
      model_bytes = uni(model_bytes + 32.0 * nm);
      const double beta = uni(sqrt(rr[0]));
      if (!isfinite(beta) && !(prm.damping && it > 0 && tstep > kMinStep)) {
        status = -5;
        break;
      }
      if (beta == 0.0) {
        conv = true;
        dmax = 0.0;
        break;
      }
      // the last step made the residual grow: take half of it back
      if (prm.damping && it > 0 && !(beta <= beta_acc) && tstep > kMinStep) {
        tstep = uni(0.5 * tstep);
        for (int k = 0; k < m; ++k)
          for (int q = tid; q < nb; q += BLOCK) {
            const int idx = tm.bidx(q);
            U[(int64_t)k * n0 + idx] -= tstep * double(gZ[k * vs + idx]);
          }
        tm.bytes = uni(tm.bytes + (16.0 + sizeof(TI)) * nm);
        dmax = uni(0.5 * dmax);
        ++damped;
        tm.sync();
        continue;
      }
      beta_acc = beta;
      tstep = 1.0;
      // ---- smoother weights: once per sample, from the first slab operator ----
      if (!weights_ready) {
        tm.w0 = gW;
        tm.dinv = gD;
        if (MG) tm.coarse_weights(U, inv_dt);
        for (int l = 0; l < (MG ? L->nmg : 1); ++l) {
          TI* x0 = (l == 0) ? tm.V + vs : tm.mgX(l);
          TI* x1 = (l == 0) ? tm.V + 2 * vs : tm.mgT(l);
          const double lmax = 1.05 * tm.power_lmax(l, x0, x1);
          const int K = (l == L->nmg - 1) ? L->sweeps : prm.smooth_steps;
          if (tid == 0) chebyshev_weights(lmax / L->cheb_ratio, lmax, K, omega_tab + l * kMaxSweeps);
        }
        __syncthreads();
        weights_ready = true;
      }

      // ---- GMRES(restart) over the space-time vectors ----
      if (tid == 0) {
        sc[0] = 1.0 / beta;
        gv[0] = beta;
      }
      __syncthreads();
      const double tol_abs = uni(eta * beta);
      int jdim = 0;
      for (int j = 0; j < restart; ++j) {
        const TI* Vj = gV + j * gs;
        TI* Vn = gV + (j + 1) * gs;
        model_bytes = uni(model_bytes + double(sizeof(TI)) * nm * (krylov_words + 2.0 * j));
        precond(Vj, gZ);
        spmv(gZ, Vn);
        // Classical Gram-Schmidt against V_0..V_j, twice for float32 (CGS2)
        double nn[1] = {0.0};
        constexpr int kPasses = sizeof(TI) == 4 ? 2 : 1;
#pragma unroll 1
        for (int pass = 0; pass < kPasses; ++pass) {
          for (int k0 = 0; k0 <= j; k0 += 8) {
            const int nk = min(j + 1 - k0, 8);
            tm.bytes = uni(tm.bytes + ((1.0 + nk) * sizeof(TI) * nm));
            double d[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) d[q] = 0.0;
            for (int k = 0; k < m; ++k)
              for (int q = tid; q < nb; q += BLOCK) {
                const int64_t idx = k * vs + tm.bidx(q);
                const double wd = double(Vn[idx]);
#pragma unroll
                for (int p = 0; p < 8; ++p)
                  if (p < nk) d[p] += double(gV[(k0 + p) * gs + idx]) * wd;
              }
            tm.template tsum<9>(d);
            if (tid == 0) {
#pragma unroll
              for (int q = 0; q < 8; ++q)
                if (q < nk) coef[k0 + q] = d[q];
            }
          }
          // projections onto the normalised basis enter H; V_q is stored with
          // norm 1/sc[q], so w loses (sc[q]^2 <V_q, w>) V_q
          if (tid == 0)
            for (int q = 0; q <= j; ++q) {
              const double hq = sc[q] * sc[j] * coef[q];
              H[q * kMaxRestart + j] = (pass ? H[q * kMaxRestart + j] : 0.0) + hq;
              coef[q] = sc[q] * sc[q] * coef[q];
            }
          __syncthreads();
          nn[0] = 0.0;
          tm.bytes = uni(tm.bytes + ((j + 3.0) * sizeof(TI) * nm));
          for (int k = 0; k < m; ++k)
            for (int q = tid; q < nb; q += BLOCK) {
              const int64_t idx = k * vs + tm.bidx(q);
              double w = double(Vn[idx]);
              for (int p = 0; p <= j; ++p) w -= coef[p] * double(gV[p * gs + idx]);
              const TI wt = TI(w);
              Vn[idx] = wt;
              nn[0] += double(wt) * double(wt);
            }
          tm.template tsum<1>(nn);  // its barriers also publish V_{j+1}
        }
        const double hn = uni(sqrt(nn[0]));
        if (tid == 0) {
          const double hj1 = sc[j] * hn;
          sc[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
          for (int q = 0; q < j; ++q) {  // previous rotations on column j
            const double a = H[q * kMaxRestart + j], b = H[(q + 1) * kMaxRestart + j];
            H[q * kMaxRestart + j] = cs_[q] * a + sn_[q] * b;
            H[(q + 1) * kMaxRestart + j] = -sn_[q] * a + cs_[q] * b;
          }
          const double a = H[j * kMaxRestart + j];
          const double r = sqrt(a * a + hj1 * hj1);
          const double c = r > 0.0 ? a / r : 1.0, sn = r > 0.0 ? hj1 / r : 0.0;
          cs_[j] = c;
          sn_[j] = sn;
          H[j * kMaxRestart + j] = r;
          H[(j + 1) * kMaxRestart + j] = 0.0;
          gv[j + 1] = -sn * gv[j];
          gv[j] = c * gv[j];
          sh_resid = fabs(gv[j + 1]);
        }
        __syncthreads();
        jdim = j + 1;
        const double resid = uni(sh_resid);
        if (!(resid > tol_abs) || !(hn > 0.0)) break;
      }
      krylov_total += jdim;
      if (tid == 0) {
        for (int q = jdim - 1; q >= 0; --q) {
          double acc = gv[q];
          for (int p = q + 1; p < jdim; ++p) acc -= H[q * kMaxRestart + p] * yv[p];
          yv[q] = acc / H[q * kMaxRestart + q];
        }
        for (int q = 0; q < jdim; ++q) coef[q] = yv[q] * sc[q];
      }
      __syncthreads();
      // ---- delta = P^-1 (sum_q y_q v_q); U += delta (float64), max-norm ----
      TI* t = gV + jdim * gs;  // the last basis vector is no longer needed
      tm.bytes = uni(tm.bytes + (double(jdim) + 1.0) * sizeof(TI) * nm);
      for (int k = 0; k < m; ++k)
        for (int q = tid; q < nb; q += BLOCK) {
          const int64_t idx = k * vs + tm.bidx(q);
          double acc = 0.0;
          for (int p = 0; p < jdim; ++p) acc += coef[p] * double(gV[p * gs + idx]);
          t[idx] = TI(acc);
        }
      tm.sync();
      precond(t, gZ);
      double dm = 0.0;
      tm.bytes = uni(tm.bytes + (16.0 + sizeof(TI)) * nm);
      for (int k = 0; k < m; ++k)
        for (int q = tid; q < nb; q += BLOCK) {
          const int idx = tm.bidx(q);
          const double dl = double(gZ[k * vs + idx]);
          U[(int64_t)k * n0 + idx] += dl;
          dm = fmax(dm, fabs(dl));
        }
      dmax = uni(tm.tmax(dm));  // its barrier also publishes U to the other members
      const double ach = sh_resid / beta;
      if (!isfinite(dmax)) {
        status = -5;
        break;
      }
      if (dmax <= prm.newton_tol) {
        conv = true;
        ++it;
        break;
      }
      if (it >= 1) {
        const double ratio = dmax / dprev;
        const double pred = dmax * fmax(ratio * ratio, 10.0 * ach);
        if (ratio < 0.5 && pred <= 0.1 * prm.newton_tol) {
          conv = true;
          ++it;
          break;
        }
      }
      dprev = uni(dmax);
      eta = uni(fmax(prm.gmres_rtol, fmin(1e-4, 0.01 * dmax)));
    }
    if (!conv && status == 0) status = -4;

    // ---- activation map: first up-crossing in time at every owned node ----
    double cen[1] = {0.0};
    tm.bytes = uni(tm.bytes + 8.0 * nm + 16.0 * n0);
    for (int q = tid; q < nb; q += BLOCK) {
      const int idx = tm.bidx(q);
      double up = L->u0[idx];
      double t = (up >= thr) ? 0.0 : -1.0;
      for (int k = 0; k < m; ++k) {
        const double un = U[(int64_t)k * n0 + idx];
        if (t < 0.0 && un >= thr) t = k * dt + dt * (thr - up) / (un - up);
        up = un;
      }
      if (t < 0.0) {
        t = L->T;
        cen[0] += 1.0;
      }
      tact[idx] = t;
      if (task.t_act) task.t_act[(int64_t)s * n0 + idx] = t;
    }
    tm.template tsum<1>(cen);
    if (tid == 0 && task.stats && task.rank == 0) {
      SampleStatsDev st;
      st.status = tm.broken ? -3 : status;
      st.newton_max_per_slab = it;
      st.newton_iters = it;
      st.krylov_iters = krylov_total;
      st.final_step = dmax;
      st.ticks = wall_clock64() - t_start;
      st.censored = (int)cen[0];
      st.damped = (int)damped;
      st.alg_bytes = tm.bytes;
      st.model_bytes = model_bytes;
      for (int q = 0; q < 8; ++q) st.phase_ticks[q] = 0;
#ifdef STM_PHASE_TIMERS
      for (int q = 0; q < 8; ++q) st.phase_ticks[q] = ph_acc[q];
#endif
      task.stats[s] = st;
    }
#ifdef STM_PHASE_TIMERS
    __syncthreads();
    if (threadIdx.x < 8) ph_acc[threadIdx.x] = 0;
#endif
    prevU = U;
    have_prev = (status == 0);
    tm.sync();
  }
}

// ---------------------------------------------------------------------------
// host launcher
// ---------------------------------------------------------------------------
template <typename TI, int DIM, bool MG>
static const void* kernel_for_block(int block, bool global) {
  if (global) {
    switch (block) {
      case 256: return (const void*)st_global_kernel<TI, DIM, 256, MG>;
      case 512: return (const void*)st_global_kernel<TI, DIM, 512, MG>;
      default: return nullptr;
    }
  }
  switch (block) {
    case 256: return (const void*)st_team_kernel<TI, DIM, 256, MG>;
    case 512: return (const void*)st_team_kernel<TI, DIM, 512, MG>;
    case 1024: return (const void*)st_team_kernel<TI, DIM, 1024, MG>;
    default: return nullptr;
  }
}

// The multi-grid kernel variant (MG = true) serves launches with a level
// whose V-cycle has coarse grids; the others take the single-grid variant,
// which compiles none of the coarse-grid code.
template <int DIM>
static const void* kernel_for_dim(bool fp32, bool mg, int block, bool global) {
  if (mg)
    return fp32 ? kernel_for_block<float, DIM, true>(block, global) : kernel_for_block<double, DIM, true>(block, global);
  return fp32 ? kernel_for_block<float, DIM, false>(block, global) : kernel_for_block<double, DIM, false>(block, global);
}

static const void* solver_kernel(int dim, bool fp32, bool mg, int block, bool global) {
  return dim == 2 ? kernel_for_dim<2>(fp32, mg, block, global) : kernel_for_dim<3>(fp32, mg, block, global);
}

hipError_t launch_team_solver(int dim, bool inner_fp32, bool mg, const LevelDev* levels, const TeamTask* tasks,
                              int n_blocks, SolverParams prm, int block, size_t lds_bytes, bool cooperative,
                              hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  const void* f = solver_kernel(dim, inner_fp32, mg, block, prm.global_st != 0);
  if (!f) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&levels, (void*)&tasks, (void*)&prm};
  if (cooperative) return hipLaunchCooperativeKernel(f, dim3(n_blocks), dim3(block), args, (unsigned)lds_bytes, st);
  return hipLaunchKernel(f, dim3(n_blocks), dim3(block), args, lds_bytes, st);
}

// Co-resident workgroups per CU for a launch configuration (0 on error).
int team_solver_occupancy(int dim, bool inner_fp32, bool mg, bool global, int block, size_t lds_bytes) {
  int nb = 0;
  const void* f = solver_kernel(dim, inner_fp32, mg, block, global);
  if (!f) return 0;
  if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, block, lds_bytes) != hipSuccess) return 0;
  return nb;
}

}  // namespace stm
