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

// The 3D element: with vertex v = bx + 2 by + 4 bz and s = 2 b - 1 per axis,
//   (K_e k)_v = s_x A(by, bz) + s_y B(bx, bz) + s_z C(bx, by)
//   A = ax [M_y M_z dx] + axy [M_z hy],  B = ay [M_x M_z dy] + axy [M_z hx],
//   C = az [M_x M_y dz],
//   (M_e m)_v = cm [M_x M_y M_z m]_v
// where dx(by, bz) are the four x-edge differences of k (likewise dy, dz),
// hx(bz), hy(bz) the sums of a z-layer's two x- resp. y-edge differences, and
// M = [[2, 1], [1, 2]] along the named axis; ax = D_xx h_y h_z / (36 h_x),
// ay, az likewise, axy = D_xy h_z / 24, cm = h_x h_y h_z / 216 (an element
// with a constant tensor whose fibres lie in the x-y plane).  Only the unique
// factors are formed, which keeps few values live.
template <typename T>
__device__ __forceinline__ void m1_pair(T& a, T& b) {
  const T x = a, y = b;
  a = T(2) * x + y;
  b = x + T(2) * y;
}

template <typename T>
__device__ __forceinline__ void elem_apply_3d(const T (&k)[8], const T (&m)[8], T ax, T ay, T az, T axy, T cm,
                                              T (&out)[8]) {
  // edge differences: index (the two other axes' bits) = first + 2 second
  T dx[4], dy[4], dz[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int b1 = u & 1, b2 = u >> 1;
    dx[u] = k[1 + 2 * b1 + 4 * b2] - k[2 * b1 + 4 * b2];  // (by, bz)
    dy[u] = k[b1 + 2 + 4 * b2] - k[b1 + 4 * b2];          // (bx, bz)
    dz[u] = k[b1 + 2 * b2 + 4] - k[b1 + 2 * b2];          // (bx, by)
  }
  T hx[2] = {dx[0] + dx[1], dx[2] + dx[3]};  // per bz
  T hy[2] = {dy[0] + dy[1], dy[2] + dy[3]};
  m1_pair(hx[0], hx[1]);
  m1_pair(hy[0], hy[1]);
  // M along both other axes of each difference set
  m1_pair(dx[0], dx[1]);
  m1_pair(dx[2], dx[3]);
  m1_pair(dx[0], dx[2]);
  m1_pair(dx[1], dx[3]);
  m1_pair(dy[0], dy[1]);
  m1_pair(dy[2], dy[3]);
  m1_pair(dy[0], dy[2]);
  m1_pair(dy[1], dy[3]);
  m1_pair(dz[0], dz[1]);
  m1_pair(dz[2], dz[3]);
  m1_pair(dz[0], dz[2]);
  m1_pair(dz[1], dz[3]);
  T fm[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) fm[v] = m[v];
#pragma unroll
  for (int v = 0; v < 8; v += 2) m1_pair(fm[v], fm[v + 1]);
#pragma unroll
  for (int v = 0; v < 8; ++v)
    if (!(v & 2)) m1_pair(fm[v], fm[v + 2]);
#pragma unroll
  for (int v = 0; v < 4; ++v) m1_pair(fm[v], fm[v + 4]);
  T A[4], B[4], C[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    A[u] = ax * dx[u] + axy * hy[u >> 1];
    B[u] = ay * dy[u] + axy * hx[u >> 1];
    C[u] = az * dz[u];
  }
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int bx = v & 1, by = (v >> 1) & 1, bz = v >> 2;
    const T a = A[by + 2 * bz], b = B[bx + 2 * bz], c = C[bx + 2 * by];
    T acc = bx ? a : -a;
    acc += by ? b : -b;
    acc += bz ? c : -c;
    out[v] = acc + cm * fm[v];
  }
}

template <typename T>
__device__ __forceinline__ void elem_apply_3d(const T (&k)[8], const T (&m)[8], const Tensor3<T>& D, T cxx, T cyy,
                                              T czz, T cxy, T cm, T (&out)[8]) {
  elem_apply_3d<T>(k, m, D.xx * cxx, D.yy * cyy, D.zz * czz, D.xy * cxy, cm, out);
}

}  // namespace stm
