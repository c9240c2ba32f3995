// Matrix-free Q1 operators on structured grids (node-centred gather).
//
// For an axis-aligned box element with sides (hx, hy[, hz]) and a constant
// tensor D, the element mass and stiffness matrices are tensor products of the
// 1D matrices  m = h/6 [2 1; 1 2],  k = 1/h [1 -1; -1 1],  g = int phi_a' phi_b = s_a / 2
// (s_0 = -1, s_1 = +1).  Contracting them with the element's vertex values in
// closed form gives the row of node v of  M_e mv + K_e kv  with a few dozen
// flops; a node sums the rows of its 4 (2D) or 8 (3D) adjacent elements.  The
// result is y = M mv + K kv for two nodal fields mv, kv -- the Jacobian slab
// operator uses mv = (1/dt - f'(u)) x, kv = x; the residual uses
// mv = (u_k - u_{k-1})/dt - f(u_k), kv = u_k.
//
// Field accessors take node coordinates (ii, jj[, kk]), already clamped to the
// grid, so the same code reads global memory or an LDS tile.
#pragma once

#include "stm_device.h"

namespace stm {

template <typename T>
struct Tensor2 { T xx, yy, xy; };

template <typename T>
struct Tensor3 { T xx, yy, zz, xy; };  // fibres lie in the x-y plane: xz = yz = 0

// y for node (i, j).  fm(ii, jj), fk(ii, jj): nodal values; fd(ex, ey): Tensor2.
// diag (optional): diagonal of  M diag(w) + K  at the node, w = wself there.
template <typename T, typename FM, typename FK, typename FD>
__device__ __forceinline__ T q1_apply_2d(const GridDev& g, int i, int j, FM fm, FK fk, FD fd, T wself, T* diag) {
  T mv[3][3], kv[3][3];
#pragma unroll
  for (int dj = 0; dj < 3; ++dj) {
    const int jj = min(max(j + dj - 1, 0), g.ny - 1);
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const int ii = min(max(i + di - 1, 0), g.nx - 1);
      mv[dj][di] = fm(ii, jj);
      kv[dj][di] = fk(ii, jj);
    }
  }
  const T cxx = T(g.hy / (6.0 * g.hx));
  const T cyy = T(g.hx / (6.0 * g.hy));
  const T cm = T(g.hx * g.hy / 36.0);
  T y = T(0), dg = T(0);
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int ey = j - 1 + b;
    if (ey < 0 || ey >= g.ey) continue;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int ex = i - 1 + a;
      if (ex < 0 || ex >= g.ex) continue;
      const Tensor2<T> D = fd(ex, ey);
      const T sx = T(1 - 2 * a), sy = T(1 - 2 * b);
      // differences along x on the node's row and the opposite row
      const T dxv = kv[1][a + 1] - kv[1][a];
      const T dxo = kv[2 * b][a + 1] - kv[2 * b][a];
      // differences along y on the node's column and the opposite column
      const T dyv = kv[b + 1][1] - kv[b][1];
      const T dyo = kv[b + 1][2 * a] - kv[b][2 * a];
      T acc = cxx * D.xx * sx * (T(2) * dxv + dxo);
      acc += cyy * D.yy * sy * (T(2) * dyv + dyo);
      acc += T(0.25) * D.xy * (sx * (dyv + dyo) + sy * (dxv + dxo));
      acc += cm * (T(4) * mv[1][1] + T(2) * mv[1][2 * a] + T(2) * mv[2 * b][1] + mv[2 * b][2 * a]);
      y += acc;
      if (diag) dg += T(2) * cxx * D.xx + T(2) * cyy * D.yy + T(0.5) * D.xy * sx * sy + T(4) * cm * wself;
    }
  }
  if (diag) *diag = dg;
  return y;
}

// 3D: node (i, j, k).  Element vertex (wx, wy, wz) of the element at offset
// (a, b, c) (ex = i-1+a ...) sits at stencil position (a+wx, b+wy, c+wz).
// The 1D factors along each axis: mass m(v,w) = h/6 (2 if v==w else 1),
// stiffness k(v,w) = s_v s_w / h, mixed g(v,w) = s_v / 2.
template <typename T, typename FM, typename FK, typename FD>
__device__ __forceinline__ T q1_apply_3d(const GridDev& g, int i, int j, int k, FM fm, FK fk, FD fd, T wself,
                                         T* diag) {
  T mv[3][3][3], kv[3][3][3];
#pragma unroll
  for (int dk = 0; dk < 3; ++dk) {
    const int kk = min(max(k + dk - 1, 0), g.nz - 1);
#pragma unroll
    for (int dj = 0; dj < 3; ++dj) {
      const int jj = min(max(j + dj - 1, 0), g.ny - 1);
#pragma unroll
      for (int di = 0; di < 3; ++di) {
        const int ii = min(max(i + di - 1, 0), g.nx - 1);
        mv[dk][dj][di] = fm(ii, jj, kk);
        kv[dk][dj][di] = fk(ii, jj, kk);
      }
    }
  }
  const T hx = T(g.hx), hy = T(g.hy), hz = T(g.hz);
  const T cxx = hy * hz / (T(36) * hx), cyy = hx * hz / (T(36) * hy), czz = hx * hy / (T(36) * hz);
  const T cxy = hz / T(24), cm = hx * hy * hz / T(216);
  T y = T(0), dg = T(0);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int ez = k - 1 + c;
    if (ez < 0 || ez >= g.ez) continue;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int ey = j - 1 + b;
      if (ey < 0 || ey >= g.ey) continue;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ex = i - 1 + a;
        if (ex < 0 || ex >= g.ex) continue;
        const Tensor3<T> D = fd(ex, ey, ez);
        // local vertex of the node: (1-a, 1-b, 1-c); signs s = 2v - 1
        const T sx = T(1 - 2 * a), sy = T(1 - 2 * b), sz = T(1 - 2 * c);
        // Sum over the 8 element vertices w of  A_vw x_w  with
        //   xx: (sx sw_x / hx) (hy/6 my) (hz/6 mz),  likewise yy, zz
        //   xy + yx: (sx/2)(sw_y/2)(hz/6 mz) + (sw_x/2)(sy/2)(hz/6 mz)
        //   mass: (hx/6 mx)(hy/6 my)(hz/6 mz)
        T sxx = T(0), syy = T(0), szz = T(0), sxy = T(0), smm = T(0);
#pragma unroll
        for (int wz = 0; wz < 2; ++wz) {
#pragma unroll
          for (int wy = 0; wy < 2; ++wy) {
#pragma unroll
            for (int wx = 0; wx < 2; ++wx) {
              const T xk = kv[c + wz][b + wy][a + wx];
              const T xm = mv[c + wz][b + wy][a + wx];
              const T mx = (wx == 1 - a) ? T(2) : T(1);
              const T my = (wy == 1 - b) ? T(2) : T(1);
              const T mz = (wz == 1 - c) ? T(2) : T(1);
              const T swx = T(2 * wx - 1), swy = T(2 * wy - 1), swz = T(2 * wz - 1);
              sxx += swx * my * mz * xk;
              syy += swy * mx * mz * xk;
              szz += swz * mx * my * xk;
              sxy += (sx * swy + swx * sy) * mz * xk;
              smm += mx * my * mz * xm;
            }
          }
        }
        T acc = D.xx * sx * sxx * cxx;
        acc += D.yy * sy * syy * cyy;
        acc += D.zz * sz * szz * czz;
        acc += D.xy * sxy * cxy;
        acc += smm * cm;
        y += acc;
        if (diag) {
          dg += T(4) * (D.xx * cxx + D.yy * cyy + D.zz * czz) + T(4) * D.xy * sx * sy * cxy +
                T(8) * cm * wself;
        }
      }
    }
  }
  if (diag) *diag = dg;
  return y;
}

}  // namespace stm

namespace stm {

// ---------------------------------------------------------------------------
// Element-centred evaluation: the contributions of one element to its
// vertices, out[v] = (M_e m + K_e k)_v, with the 1D factors applied axis by
// axis (sum factorisation).  Vertex v = bx + 2 by (+ 4 bz).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void elem_apply_2d(const T (&k)[4], const T (&m)[4], const Tensor2<T>& D, T cxx, T cyy,
                                              T cm, T (&out)[4]) {
  const T dx0 = k[1] - k[0], dx1 = k[3] - k[2];
  const T dy0 = k[2] - k[0], dy1 = k[3] - k[1];
  const T p0 = cxx * D.xx * (T(2) * dx0 + dx1), p1 = cxx * D.xx * (T(2) * dx1 + dx0);
  const T q0 = cyy * D.yy * (T(2) * dy0 + dy1), q1 = cyy * D.yy * (T(2) * dy1 + dy0);
  const T A = T(0.25) * D.xy * (dy0 + dy1), B = T(0.25) * D.xy * (dx0 + dx1);
  const T r00 = T(2) * m[0] + m[1], r01 = m[0] + T(2) * m[1];  // row by=0: vx = 0, 1
  const T r10 = T(2) * m[2] + m[3], r11 = m[2] + T(2) * m[3];  // row by=1
  out[0] = -p0 - q0 - A - B + cm * (T(2) * r00 + r10);
  out[1] = p0 - q1 + A - B + cm * (T(2) * r01 + r11);
  out[2] = -p1 + q0 - A + B + cm * (T(2) * r10 + r00);
  out[3] = p1 + q1 + A + B + cm * (T(2) * r11 + r01);
}

// 1D factor [[2,1],[1,2]] along one axis of a 2x2x2 block given by index stride
template <typename T>
__device__ __forceinline__ void m1_axis(T (&f)[8], int stride) {
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    if (v & stride) continue;
    const T a = f[v], b = f[v + stride];
    f[v] = T(2) * a + b;
    f[v + stride] = a + T(2) * b;
  }
}

template <typename T>
__device__ __forceinline__ void elem_apply_3d(const T (&k)[8], const T (&m)[8], const Tensor3<T>& D, T cxx, T cyy,
                                              T czz, T cxy, T cm, T (&out)[8]) {
  T fx[8], fy[8], fz[8], fm[8], gxy[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    // s_a (f1 - f0) along each axis
    const int bx = v & 1, by = (v >> 1) & 1, bz = (v >> 2) & 1;
    const T dxv = k[v | 1] - k[v & ~1];
    const T dyv = k[v | 2] - k[v & ~2];
    const T dzv = k[v | 4] - k[v & ~4];
    fx[v] = bx ? dxv : -dxv;
    fy[v] = by ? dyv : -dyv;
    fz[v] = bz ? dzv : -dzv;
    fm[v] = m[v];
  }
  // xy coupling: s_vx (h_y(0) + h_y(1)) + s_vy (h_x(0) + h_x(1)), h = differences
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int bx = v & 1, by = (v >> 1) & 1;
    const int base = v & 4;  // same z layer
    const T hy = (k[base | 2] - k[base]) + (k[base | 3] - k[base | 1]);
    const T hx = (k[base | 1] - k[base]) + (k[base | 3] - k[base | 2]);
    gxy[v] = (bx ? hy : -hy) + (by ? hx : -hx);
  }
  m1_axis(fx, 2); m1_axis(fx, 4);
  m1_axis(fy, 1); m1_axis(fy, 4);
  m1_axis(fz, 1); m1_axis(fz, 2);
  m1_axis(gxy, 4);
  m1_axis(fm, 1); m1_axis(fm, 2); m1_axis(fm, 4);
  const T ax = D.xx * cxx, ay = D.yy * cyy, az = D.zz * czz, axy = D.xy * cxy;
#pragma unroll
  for (int v = 0; v < 8; ++v) out[v] = ax * fx[v] + ay * fy[v] + az * fz[v] + axy * gxy[v] + cm * fm[v];
}

}  // namespace stm
