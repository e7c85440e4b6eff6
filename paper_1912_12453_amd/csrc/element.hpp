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

// Every lane of the wave is active whenever these run (all row and bank masks
// set), and every source lane of these controls lies in the lane's own row,
// so the moved value never falls back to the "old" operand or to bound_ctrl's
// zero.  The FP32 form is written as update_dpp with bound_ctrl set because
// then the compiler folds the move into the VOP2 that consumes it
// (v_sub_f32_dpp, v_add_f32_dpp): one VALU instruction instead of two.  The
// 64-bit moves stay separate (no DPP form of the FP64 arithmetic with these
// controls).
template <int CTRL>
__device__ __forceinline__ float xchg(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double xchg(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Per-lane geometry of the element and of the lane's corner / Gauss point.
template <class T>
struct Lane {
  int c;          // corner index i + 2j + 4k
  T sxh, syh, szh;  // corner sign along each axis divided by h
  T h, wdet;      // side and Gauss weight * det J = h^3/8
  T ih, Gh;       // 1/h and 4/h^2 (exact: h is a power of two)
  __device__ void init(int lane8, int level) {
    const int bz = lane8 >> 2;
    const int t = bz ? (lane8 ^ 7) : lane8;
    const int bx = t & 1, by = (t >> 1) & 1;
    c = bx + 2 * by + 4 * bz;
    h = (T)ldexp(1.0, -level);
    ih = (T)ldexp(1.0, level);
    Gh = (T)ldexp(1.0, 2 * level + 2);
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

// One axis of the butterfly with d = partner - mine:
//   value at the lane's Gauss point  mine + B*d   (A*mine + B*partner, A + B = 1)
//   derivative along the axis       -s*d/h        (s*(mine - partner)/h)
template <class T>
__device__ __forceinline__ T eval_v(T u) {
  const T B = (T)kB;
  T v = u + B * (xchg<kXor1>(u) - u);
  v = v + B * (xchg<kXor2>(v) - v);
  return v + B * (xchg<kXor7>(v) - v);
}

template <class T>
__device__ __forceinline__ VG<T> eval_vg(T u, const Lane<T>& L) {
  const T B = (T)kB;
  const T d1 = xchg<kXor1>(u) - u;
  const T v = u + B * d1;
  const T dx = -L.sxh * d1;
  const T d2 = xchg<kXor2>(v) - v, e2 = xchg<kXor2>(dx) - dx;
  const T v2 = v + B * d2;
  const T dy = -L.syh * d2;
  const T dx2 = dx + B * e2;
  const T d3 = xchg<kXor7>(v2) - v2, e3 = xchg<kXor7>(dx2) - dx2, f3 = xchg<kXor7>(dy) - dy;
  VG<T> r;
  r.v = v2 + B * d3;
  r.dz = -L.szh * d3;
  r.dx = dx2 + B * e3;
  r.dy = dy + B * f3;
  return r;
}

template <class T>
__device__ __forceinline__ VGH<T> eval_vgh(T u, const Lane<T>& L) {
  const T B = (T)kB;
  const T d1 = xchg<kXor1>(u) - u;
  const T v = u + B * d1;
  const T dx = -L.sxh * d1;
  const T d2 = xchg<kXor2>(v) - v, e2 = xchg<kXor2>(dx) - dx;
  const T v2 = v + B * d2;
  const T dy = -L.syh * d2;
  const T dxy = -L.syh * e2;
  const T dx2 = dx + B * e2;
  const T d3 = xchg<kXor7>(v2) - v2, e3 = xchg<kXor7>(dx2) - dx2, f3 = xchg<kXor7>(dy) - dy,
          g3 = xchg<kXor7>(dxy) - dxy;
  VGH<T> r;
  r.v = v2 + B * d3;
  r.dz = -L.szh * d3;
  r.dx = dx2 + B * e3;
  r.dy = dy + B * f3;
  r.dxy = dxy + B * g3;
  r.dxz = -L.szh * e3;
  r.dyz = -L.szh * f3;
  return r;
}

// sum over the element's Gauss points of N_a c + dN_a/dx Fx + dN_a/dy Fy +
// dN_a/dz Fz, returned on the lane of corner a (the transposed butterfly:
// per axis c <- A*c + B*c_partner + s*(F + F_partner)/h).
template <class T>
__device__ __forceinline__ T test_contract(T c, T Fx, T Fy, T Fz, const Lane<T>& L) {
  const T B = (T)kB;
  const T c1 = c + B * (xchg<kXor7>(c) - c) + L.szh * (Fz + xchg<kXor7>(Fz));
  const T Fx1 = Fx + B * (xchg<kXor7>(Fx) - Fx);
  const T Fy1 = Fy + B * (xchg<kXor7>(Fy) - Fy);
  const T c2 = c1 + B * (xchg<kXor2>(c1) - c1) + L.syh * (Fy1 + xchg<kXor2>(Fy1));
  const T Fx2 = Fx1 + B * (xchg<kXor2>(Fx1) - Fx1);
  return c2 + B * (xchg<kXor1>(c2) - c2) + L.sxh * (Fx2 + xchg<kXor1>(Fx2));
}

// FP64: each 64-bit exchange is two DPP moves, so the partner's share of a
// stage is formed on the partner and moved once.  Across an axis the two
// lanes differ only in that axis' sign s, so B c_P + s (F_P) = B c_P - s_P F_P:
// per contraction 6 exchanges instead of 9, the same arithmetic count.
template <>
__device__ __forceinline__ double test_contract<double>(double c, double Fx, double Fy, double Fz,
                                                        const Lane<double>& L) {
  const double A = kA, B = kB;
  const double c1 = A * c + L.szh * Fz + xchg<kXor7>(B * c - L.szh * Fz);
  const double Fx1 = A * Fx + xchg<kXor7>(B * Fx);
  const double Fy1 = A * Fy + xchg<kXor7>(B * Fy);
  const double c2 = A * c1 + L.syh * Fy1 + xchg<kXor2>(B * c1 - L.syh * Fy1);
  const double Fx2 = A * Fx1 + xchg<kXor2>(B * Fx1);
  return A * c2 + L.sxh * Fx2 + xchg<kXor1>(B * c2 - L.sxh * Fx2);
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

// Scatter plan on the device (see ScatterPlan in internal.hpp).
struct PlanView {
  const int32_t* tgt_off;     // per chunk
  const int32_t* tgt;         // per target slot: node id
  const int32_t* inc_off;     // per target slot
  const int32_t* chunk_inc;   // per chunk: inc_off of its first target
  const uint8_t* inc_corner;  // local element * 8 + corner
  const float* inc_w;
  const int32_t* node_off;    // per node
  const int32_t* node_slot;
  const int64_t* touch_off;   // per element
  const int32_t* touch_node;  // per element touch: the node
  const int64_t* ntouch_off;  // per node
  const int64_t* ntouch_slot;
  const uint8_t* bflags;      // per node
  const int32_t* cmap;        // per element corner: target-list position, or -1 - hanging entry
  const int32_t* hmap;        // per hanging entry: kHMapDev ints (row start, count, 16-bit positions)
};
constexpr int kHMapDev = 8;

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
