// Device building blocks of the element loop for gfx950 (wave64).
//
// Layout of the work: eight consecutive lanes own one element.  For gather
// and scatter lane l stands for corner c(l); for the pointwise physics the
// same lane stands for the Gauss point with the same sign pattern.  The lane
// to corner map is l = bx ^ 2*by ^ 7*bz, so that the corner partner along x,
// y and z is the lane l^1, l^2 and l^7: all three exchanges are DPP moves
// (quad_perm for ^1 and ^2, row_half_mirror for ^7) and never touch LDS.
//
// Trilinear (Q1) fields on [-1,1]^3 are tensor products, so evaluation at the
// 2x2x2 Gauss points (+-1/sqrt(3), weight 1) is one 2x2 butterfly per axis:
//   value:      v <- A*mine + B*partner,  A = (1+g)/2, B = (1-g)/2, g = 1/sqrt(3)
//   derivative: d <- s*(mine - partner)/h  (s = +1 for the upper corner)
// and the test-function contraction sum_q [N_a(q) c_q + grad N_a(q) . F_q] is
// the transposed butterfly.  Gradients are physical: d/dx = (2/h) d/dxi.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace chns {
namespace dev {

constexpr double kGauss = 0.57735026918962576451;  // 1/sqrt(3)
constexpr double kA = 0.5 * (1.0 + kGauss);
constexpr double kB = 0.5 * (1.0 - kGauss);

// DPP controls (gfx9): quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror
constexpr int kXor1 = 0xB1;
constexpr int kXor2 = 0x4E;
constexpr int kXor7 = 0x141;

template <int CTRL>
__device__ __forceinline__ float xchg(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double xchg(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Per-lane geometry of the element and of the lane's corner / Gauss point.
template <class T>
struct Lane {
  int c;          // corner index i + 2j + 4k
  T sxh, syh, szh;  // corner sign along each axis divided by h
  T h, wdet;      // side and Gauss weight * det J = h^3/8
  __device__ void init(int lane8, int level) {
    const int bz = lane8 >> 2;
    const int t = bz ? (lane8 ^ 7) : lane8;
    const int bx = t & 1, by = (t >> 1) & 1;
    c = bx + 2 * by + 4 * bz;
    h = (T)ldexp(1.0, -level);
    const T ih = (T)1 / h;
    sxh = bx ? ih : -ih;
    syh = by ? ih : -ih;
    szh = bz ? ih : -ih;
    wdet = h * h * h * (T)0.125;
  }
};

template <class T>
struct VG {  // value and gradient at the lane's Gauss point
  T v, dx, dy, dz;
};
template <class T>
struct VGH {  // value, gradient and mixed second derivatives
  T v, dx, dy, dz, dxy, dxz, dyz;
};

template <class T>
__device__ __forceinline__ T eval_v(T u) {
  const T A = (T)kA, B = (T)kB;
  T v = A * u + B * xchg<kXor1>(u);
  v = A * v + B * xchg<kXor2>(v);
  return A * v + B * xchg<kXor7>(v);
}

template <class T>
__device__ __forceinline__ VG<T> eval_vg(T u, const Lane<T>& L) {
  const T A = (T)kA, B = (T)kB;
  T p = xchg<kXor1>(u);
  T v = A * u + B * p;
  T dx = L.sxh * (u - p);
  T pv = xchg<kXor2>(v), pdx = xchg<kXor2>(dx);
  T v2 = A * v + B * pv;
  T dy = L.syh * (v - pv);
  T dx2 = A * dx + B * pdx;
  T qv = xchg<kXor7>(v2), qdx = xchg<kXor7>(dx2), qdy = xchg<kXor7>(dy);
  VG<T> r;
  r.v = A * v2 + B * qv;
  r.dz = L.szh * (v2 - qv);
  r.dx = A * dx2 + B * qdx;
  r.dy = A * dy + B * qdy;
  return r;
}

template <class T>
__device__ __forceinline__ VGH<T> eval_vgh(T u, const Lane<T>& L) {
  const T A = (T)kA, B = (T)kB;
  T p = xchg<kXor1>(u);
  T v = A * u + B * p;
  T dx = L.sxh * (u - p);
  T pv = xchg<kXor2>(v), pdx = xchg<kXor2>(dx);
  T v2 = A * v + B * pv;
  T dy = L.syh * (v - pv);
  T dxy = L.syh * (dx - pdx);
  T dx2 = A * dx + B * pdx;
  T qv = xchg<kXor7>(v2), qdx = xchg<kXor7>(dx2), qdy = xchg<kXor7>(dy), qdxy = xchg<kXor7>(dxy);
  VGH<T> r;
  r.v = A * v2 + B * qv;
  r.dz = L.szh * (v2 - qv);
  r.dx = A * dx2 + B * qdx;
  r.dy = A * dy + B * qdy;
  r.dxy = A * dxy + B * qdxy;
  r.dxz = L.szh * (dx2 - qdx);
  r.dyz = L.szh * (dy - qdy);
  return r;
}

// sum over the element's Gauss points of N_a c + dN_a/dx Fx + dN_a/dy Fy +
// dN_a/dz Fz, returned on the lane of corner a.
template <class T>
__device__ __forceinline__ T test_contract(T c, T Fx, T Fy, T Fz, const Lane<T>& L) {
  const T A = (T)kA, B = (T)kB;
  T pc = xchg<kXor7>(c), pFz = xchg<kXor7>(Fz), pFx = xchg<kXor7>(Fx), pFy = xchg<kXor7>(Fy);
  T c1 = A * c + B * pc + L.szh * (Fz + pFz);
  T Fx1 = A * Fx + B * pFx;
  T Fy1 = A * Fy + B * pFy;
  T pc1 = xchg<kXor2>(c1), pFy1 = xchg<kXor2>(Fy1), pFx1 = xchg<kXor2>(Fx1);
  T c2 = A * c1 + B * pc1 + L.syh * (Fy1 + pFy1);
  T Fx2 = A * Fx1 + B * pFx1;
  T pc2 = xchg<kXor1>(c2), pFx2 = xchg<kXor1>(Fx2);
  return A * c2 + B * pc2 + L.sxh * (Fx2 + pFx2);
}

// Sum of a value over the 8 lanes of an element (every lane gets the sum).
template <class T>
__device__ __forceinline__ T group_sum(T v) {
  v += xchg<kXor1>(v);
  v += xchg<kXor2>(v);
  v += xchg<kXor7>(v);
  return v;
}

// --------------------------------------------------------- mesh access ----
struct MeshView {
  const int32_t* elem;   // E*8 corner refs: id >= 0, or -1-h
  const uint8_t* level;  // E
  const int32_t* hoff;   // NH+1
  const int32_t* hids;   // constraint parents
  const double* hw;      // constraint weights (FP64)
  const float* hw32;     // constraint weights (FP32)
  int64_t E;
};

template <class W>
__device__ __forceinline__ const W* weights(const MeshView& m);
template <>
__device__ __forceinline__ const double* weights<double>(const MeshView& m) { return m.hw; }
template <>
__device__ __forceinline__ const float* weights<float>(const MeshView& m) { return m.hw32; }

// Physical parameters in kernel form.
struct PhysView {
  double dt, inv_dt;
  double Cn, inv_PeCn, Cn2;          // CH block
  double alpha, beta, gamma, xi;     // rho = alpha phi* + beta, eta = gamma phi* + xi
  double kappa;                      // J = kappa grad mu~
  double inv_Pe, inv_Re, inv_We, inv_Fr, CnWe;  // CnWe = Cn/We
  double g[3];
  double C_I;
};

}  // namespace dev
}  // namespace chns
