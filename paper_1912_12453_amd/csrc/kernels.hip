// HIP kernels of the CHNS element loop for gfx950.
//
// Cahn-Hilliard block (Def. 1 of Sec. 3 with the Crank-Nicolson averages,
// cG(1) form of Def. 2): for test function q = N_a
//   R_phi,a = (q, (phi^{k+1}-phi^k)/dt) - (dq/dx_i, v~_i phi~) + 1/(Pe Cn) (dq/dx_i, dmu~/dx_i)
//   R_mu,a  = -(q, mu~) + (q, phi~^3 - phi~) + Cn^2 (dq/dx_i, dphi~/dx_i)
// Navier-Stokes block (Def. 2 of Sec. 3.4, residual-based VMS with tau_m,
// tau_c and the strong residuals R_m, R_c), coarse velocity and pressure at the
// midpoint, rho and eta from phi^{k+1} pulled back to [-1,1].
//
// Every element integral is evaluated at the 2x2x2 Gauss points; the
// pointwise integrand is written as a pair (c, F) such that the contribution to
// row a is sum_q wdet (N_a c + grad N_a . F), which test_contract performs.
#include <hip/hip_runtime.h>

#include "element.hpp"
#include "dual.hpp"

namespace chns {
namespace dev {

constexpr int kChunkThreads = 256;  // 32 elements x 8 lanes per workgroup

// ------------------------------------------------------------- helpers ----
// Gathers NF fields of a node-major array for the lane's corner straight from
// global memory (used by the kernels that do not stage the chunk).
template <class TS, class T, int NF>
__device__ __forceinline__ void gather(const MeshView& m, int ref, const TS* __restrict__ X,
                                       int ld, int f0, T (&out)[NF]) {
  if (ref >= 0) {
    const TS* p = X + (int64_t)ref * ld + f0;
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f] = (T)p[f];
    return;
  }
  const int h = -1 - ref;
  const int t0 = m.hoff[h], t1 = m.hoff[h + 1];
#pragma unroll
  for (int f = 0; f < NF; ++f) out[f] = (T)0;
  const auto* w = weights<T>(m);
  for (int t = t0; t < t1; ++t) {
    const T wt = w[t];
    const TS* p = X + (int64_t)m.hids[t] * ld + f0;
#pragma unroll
    for (int f = 0; f < NF; ++f) out[f] += wt * (T)p[f];
  }
}

template <class T>
__device__ __forceinline__ T clamp1(T x) {
  return x > (T)1 ? (T)1 : (x < (T)-1 ? (T)-1 : x);
}

// Chunk staging in dynamic LDS.  A workgroup owns one chunk of 32 leaves.
// Before any arithmetic it copies, with coalesced loads, the records of the
// chunk's target nodes (NU fields of U^{k+1} and U^k, ND of the direction),
// the sorted target list and the chunk's incidence lists; lanes then read
// their corners from LDS.  Capacities come from the largest chunk of the
// mesh.  Layout: val[cap_t][SV] (T) | res[256][SF] (T) | tgt[cap_t] |
// ioff[cap_t+1] | iw[cap_i] (float) | icor[cap_i] (byte).
struct ChunkCaps {
  int cap_t, cap_i;
};

template <class T, int NU, int ND, int NF>
struct ChunkLDS {
  static constexpr int NV = 2 * NU + ND;
  // record strides padded to an odd number of words so that lanes reading the
  // same field of different records hit different LDS banks
  static constexpr int SV = NV | 1;
  static constexpr int SF = NF | 1;
  T* val;
  T* res;
  int* tgt;
  int* ioff;
  float* iw;
  uint8_t* icor;
  int s0, cnt;
  __host__ __device__ static size_t bytes(ChunkCaps c) {
    return sizeof(T) * ((size_t)c.cap_t * SV + kChunkThreads * SF) + sizeof(int) * (2 * (size_t)c.cap_t + 1) +
           5 * (size_t)c.cap_i;
  }
  __device__ __forceinline__ void carve(char* smem, ChunkCaps c) {
    val = (T*)smem;
    res = val + (size_t)c.cap_t * SV;
    tgt = (int*)(res + kChunkThreads * SF);
    ioff = tgt + c.cap_t;
    iw = (float*)(ioff + c.cap_t + 1);
    icor = (uint8_t*)(iw + c.cap_i);
  }
  template <class TS, class TD>
  __device__ __forceinline__ void stage(const PlanView& pl, const TS* __restrict__ U1, const TS* __restrict__ U0,
                        const TD* __restrict__ dU, int ldD, int offD) {
    stage_chunk(pl, (int)blockIdx.x, U1, U0, dU, ldD, offD);
  }
  template <class TS, class TD>
  __device__ __forceinline__ void stage_chunk(const PlanView& pl, int chunk, const TS* __restrict__ U1,
                                              const TS* __restrict__ U0, const TD* __restrict__ dU, int ldD,
                                              int offD) {
    s0 = pl.tgt_off[chunk];
    cnt = pl.tgt_off[chunk + 1] - s0;
    const int i0 = pl.inc_off[s0];
    const int ni = pl.inc_off[s0 + cnt] - i0;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) tgt[i] = pl.tgt[s0 + i];
    for (int i = threadIdx.x; i <= cnt; i += blockDim.x) ioff[i] = pl.inc_off[s0 + i] - i0;
    for (int i = threadIdx.x; i < ni; i += blockDim.x) {
      iw[i] = pl.inc_w[i0 + i];
      icor[i] = pl.inc_corner[i0 + i];
    }
    for (int i = threadIdx.x; i < cnt * NV; i += blockDim.x) {
      const int j = i / NV, f = i - j * NV;
      const int64_t g = pl.tgt[s0 + j];
      T v;
      if constexpr (NU > 0) {
        if (f < NU) {
          v = (T)U1[g * 6 + f];
        } else if (ND == 0 || f < 2 * NU) {
          v = (T)U0[g * 6 + f - NU];
        } else {
          if constexpr (ND > 0) v = (T)dU[g * ldD + offD + f - 2 * NU];
        }
      } else {
        v = (T)dU[g * ldD + offD + f];  // direction only
      }
      val[j * SV + f] = v;
    }
  }
  // position of node g in the sorted target list
  __device__ __forceinline__ int find(int g) const {
    int lo = 0, hi = cnt;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (tgt[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
  }
  // the lane's corner record (2NU+ND values), through the constraint when the
  // corner hangs
  __device__ __forceinline__ void corner(const MeshView& m, int ref, T (&out)[NV]) const {
    if (ref >= 0) {
      const T* p = val + find(ref) * SV;
#pragma unroll
      for (int f = 0; f < NV; ++f) out[f] = p[f];
      return;
    }
#pragma unroll
    for (int f = 0; f < NV; ++f) out[f] = (T)0;
    const int h = -1 - ref;
    const auto* w = weights<T>(m);
    for (int t = m.hoff[h]; t < m.hoff[h + 1]; ++t) {
      const T wt = w[t];
      const T* p = val + find(m.hids[t]) * SV;
#pragma unroll
      for (int f = 0; f < NV; ++f) out[f] += wt * p[f];
    }
  }
  // Element-loop epilogue: stage the corner results, then every target sums
  // its incident corner results times the constraint weight in the plan's
  // fixed order and writes one partial row.  No atomics, so results do not
  // depend on scheduling.
  __device__ __forceinline__ void finish(int corner_slot, const T (&r)[NF], T* __restrict__ partial) {
#pragma unroll
    for (int f = 0; f < NF; ++f) res[corner_slot * SF + f] = r[f];
    __syncthreads();
    for (int i = threadIdx.x; i < cnt * NF; i += blockDim.x) {
      const int j = i / NF, f = i - j * NF;
      T acc = 0;
      for (int k = ioff[j]; k < ioff[j + 1]; ++k) acc += (T)iw[k] * res[icor[k] * SF + f];
      partial[(int64_t)(s0 + j) * NF + f] = acc;
    }
  }
};

// ------------------------------------------------------------ CH block ----
// CH residual rows at the lane's Gauss point, contracted against the test
// functions of the lane's corner; a / b: the corner's phi, mu, u, v, w at
// k+1 / k.
template <class T>
__device__ __forceinline__ void ch_residual_point(const PhysView& p, const Lane<T>& L, const T (&a)[5],
                                                  const T (&b)[5], T (&r)[2]) {
  const VG<T> ph = eval_vg<T>((T)0.5 * (a[0] + b[0]), L);
  const VG<T> mu = eval_vg<T>((T)0.5 * (a[1] + b[1]), L);
  const T dphi = eval_v<T>(a[0] - b[0]);
  const T vx = eval_v<T>((T)0.5 * (a[2] + b[2]));
  const T vy = eval_v<T>((T)0.5 * (a[3] + b[3]));
  const T vz = eval_v<T>((T)0.5 * (a[4] + b[4]));
  const T w = L.wdet, kd = (T)p.inv_PeCn, cn2 = (T)p.Cn2;
  r[0] = test_contract<T>(w * dphi * (T)p.inv_dt, w * (kd * mu.dx - vx * ph.v),
                          w * (kd * mu.dy - vy * ph.v), w * (kd * mu.dz - vz * ph.v), L);
  r[1] = test_contract<T>(w * (ph.v * ph.v * ph.v - ph.v - mu.v), w * cn2 * ph.dx,
                          w * cn2 * ph.dy, w * cn2 * ph.dz, L);
}

template <class T>
__global__ __launch_bounds__(256) void k_ch_residual(MeshView m, PlanView pl, PhysView p,
                                                     ChunkCaps caps,
                                                     const double* __restrict__ U1,
                                                     const double* __restrict__ U0,
                                                     T* __restrict__ partial) {
  extern __shared__ double smem_d[];
  using CL = ChunkLDS<T, 5, 0, 2>;
  CL S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int64_t e = e0 < m.E ? e0 : m.E - 1;
  Lane<T> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int ref = m.elem[e * 8 + L.c];
  S.stage(pl, U1, U0, (const double*)nullptr, 0, 0);
  __syncthreads();
  T c[CL::NV];  // phi, mu, u, v, w at k+1, then at k
  S.corner(m, ref, c);
  const T a[5] = {c[0], c[1], c[2], c[3], c[4]};
  const T b[5] = {c[5], c[6], c[7], c[8], c[9]};
  T r[2];
  ch_residual_point<T>(p, L, a, b, r);
  S.finish((threadIdx.x >> 3) * 8 + L.c, r, partial);
}

// psi''(phi~) = 3 phi~^2 - 1, the derivative of phi~^3 - phi~
template <class T>
__device__ __forceinline__ T ch_dpsi(T pt) {
  return (T)3 * pt * pt - (T)1;
}

// CH Jacobian rows at the lane's Gauss point in the direction (dp, dm) of
// (phi^{k+1}, mu^{k+1}) (values and gradients; the midpoint fields move by
// half of them).  The linearisation point enters through psi''(phi~) and v~.
template <class T>
__device__ __forceinline__ void ch_jvp_point(const PhysView& p, const Lane<T>& L, T dpsi, T vx, T vy, T vz,
                                             const VG<T>& dp, const VG<T>& dm, T (&r)[2]) {
  const T w = L.wdet, hk = (T)0.5 * (T)p.inv_PeCn, hc = (T)0.5 * (T)p.Cn2, hp = (T)0.5 * dp.v;
  r[0] = test_contract<T>(w * dp.v * (T)p.inv_dt, w * (hk * dm.dx - vx * hp),
                          w * (hk * dm.dy - vy * hp), w * (hk * dm.dz - vz * hp), L);
  r[1] = test_contract<T>(w * dpsi * hp - w * (T)0.5 * dm.v, w * hc * dp.dx, w * hc * dp.dy,
                          w * hc * dp.dz, L);
}

template <class T, class TS, class TD>
__global__ __launch_bounds__(256) void k_ch_jvp(MeshView m, PlanView pl, PhysView p, ChunkCaps caps,
                                                const TS* __restrict__ U1, const TS* __restrict__ U0,
                                                const TD* __restrict__ dU, int ldD, int offD,
                                                T* __restrict__ partial, const int* skip) {
  if (skip && *skip) return;  // GMRES control: this step is not needed
  extern __shared__ double smem_d[];
  using CL = ChunkLDS<T, 5, 2, 2>;
  CL S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int64_t e = e0 < m.E ? e0 : m.E - 1;
  Lane<T> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int ref = m.elem[e * 8 + L.c];
  S.stage(pl, U1, U0, dU, ldD, offD);
  __syncthreads();
  T c[CL::NV];  // phi, mu, u, v, w at k+1 and at k, then d phi, d mu
  S.corner(m, ref, c);
  const T pt = eval_v<T>((T)0.5 * (c[0] + c[5]));
  const T vx = eval_v<T>((T)0.5 * (c[2] + c[7]));
  const T vy = eval_v<T>((T)0.5 * (c[3] + c[8]));
  const T vz = eval_v<T>((T)0.5 * (c[4] + c[9]));
  const VG<T> dp = eval_vg<T>(c[10], L);  // d phi^{k+1}; d phi~ = dp/2
  const VG<T> dm = eval_vg<T>(c[11], L);  // d mu^{k+1};  d mu~  = dm/2
  T r[2];
  ch_jvp_point<T>(p, L, ch_dpsi<T>(pt), vx, vy, vz, dp, dm, r);
  S.finish((threadIdx.x >> 3) * 8 + L.c, r, partial);
}

// ------------------------------------------------------------ NS block ----
// Quantities of the linearisation point at one Gauss point.
template <class T>
struct NSPoint {
  T ps;              // phi^{k+1} pulled back to [-1,1]
  T rho, eta, inv_rho;
  T vt[3], G[3][3];  // v~ and its gradient G[i][j] = dv~_i/dx_j
  T J[3];            // mass flux kappa grad mu~
  T adv[3];          // rho v~_j + J_j/Pe - (deta/dx_j)/Re: transport velocity of R_m
  T tg[3];           // rho (v^{k+1}-v^k)_i/dt - rho g_i/Fr
  T Rm[3], Rc;       // strong residuals
  T tau_m, tau_c, Gh;  // Gh = 4/h^2 (G_ij = Gh delta_ij)
  T sbr;               // 1/tau_m, the square root of the bracket
  T gpht[3];         // grad phi~
  T pt;              // p~
  bool ok;           // tau_m bracket positive
};

// 1/x and 1/sqrt(x) for the point quantities (x > 0 and far from the
// exponent limits here).  FP64: the hardware estimate (v_rcp_f64, v_rsq_f64)
// refined by two Newton steps, r <- r + r (1 - x r) and y <- y + y (1/2 -
// (x/2) y^2), each of which squares the relative error; the result is within
// about an ulp of the rounded quotient, where a correctly rounded division or
// square root takes two to three times the instructions.  FP32: the
// hardware's 1-ulp instructions; dual numbers (the coupled rows) take the
// derivative of the same value.
template <class T>
__device__ __forceinline__ T recip_nr(const T& x) {
  return (T)1 / x;
}
template <class T>
__device__ __forceinline__ T rsqrt_nr(const T& x) {
  return (T)1 / sqrt(x);
}
__device__ __forceinline__ double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip_nr(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  double t = fma(-hx * y, y, 0.5);
  y = fma(y, t, y);
  t = fma(-hx * y, y, 0.5);
  return fma(y, t, y);
}
__device__ __forceinline__ float rsqrt_nr(float x) { return __builtin_amdgcn_rsqf(x); }
// dual numbers: (1/x)' = -x'/x^2, (x^-1/2)' = -x' x^-3/2 / 2
template <class T>
__device__ __forceinline__ Dual<T> recip_nr(const Dual<T>& x) {
  const T r = recip_nr(x.v);
  return Dual<T>(r, -x.d * r * r);
}
template <class T>
__device__ __forceinline__ Dual<T> rsqrt_nr(const Dual<T>& x) {
  const T y = rsqrt_nr(x.v);
  return Dual<T>(y, (T)-0.5 * x.d * y * y * y);
}

// rho, eta (linear in the pulled-back phi) and 1/rho.  The point evaluation
// and the cached linearisation share this code, so both get the same values.
template <class T>
__device__ __forceinline__ void ns_material(const PhysView& p, T ps, NSPoint<T>& P) {
  P.ps = ps;
  P.rho = (T)p.alpha * ps + (T)p.beta;
  P.eta = (T)p.gamma * ps + (T)p.xi;
  P.inv_rho = recip_nr(P.rho);
}

// R_c, the metric Gh = 4/h^2 and the stabilisation parameters tau_m, tau_c
// from v~, its gradient, J, rho and eta (shared as ns_material is).
template <class T>
__device__ __forceinline__ void ns_stab(const PhysView& p, const Lane<T>& L, NSPoint<T>& P) {
  const T iPe = (T)p.inv_Pe, iRe = (T)p.inv_Re, idt = (T)p.inv_dt;
  P.Rc = P.G[0][0] + P.G[1][1] + P.G[2][2];
  P.Gh = L.Gh;
  const T vv = P.vt[0] * P.vt[0] + P.vt[1] * P.vt[1] + P.vt[2] * P.vt[2];
  const T vJ = P.vt[0] * P.J[0] + P.vt[1] * P.J[1] + P.vt[2] * P.J[2];
  const T nu = P.eta * P.inv_rho * iRe;
  const T br = (T)4 * idt * idt + P.Gh * vv + P.Gh * vJ * P.inv_rho * iPe +
               (T)p.C_I * nu * nu * (T)3 * P.Gh * P.Gh;
  P.ok = br > (T)0;
  P.tau_m = rsqrt_nr(br);
  P.sbr = br * P.tau_m;  // 1/tau_m
  P.tau_c = P.sbr * recip_nr((T)3 * P.Gh);
}

// Linearisation point from the lane's corner values of U^{k+1} (a) and U^k (b),
// 6 fields each (phi, mu, u, v, w, p).
template <class T>
__device__ __forceinline__ void ns_point(const PhysView& p, const Lane<T>& L, const T (&a)[6],
                                         const T (&b)[6], NSPoint<T>& P) {
  const VG<T> ph1 = eval_vg<T>(a[0], L);
  const VGH<T> pht = eval_vgh<T>((T)0.5 * (a[0] + b[0]), L);
  const VG<T> mut = eval_vg<T>((T)0.5 * (a[1] + b[1]), L);
  const VG<T> pt = eval_vg<T>((T)0.5 * (a[5] + b[5]), L);
  T dv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const VG<T> v = eval_vg<T>((T)0.5 * (a[2 + i] + b[2 + i]), L);
    P.vt[i] = v.v;
    P.G[i][0] = v.dx;
    P.G[i][1] = v.dy;
    P.G[i][2] = v.dz;
    dv[i] = eval_v<T>(a[2 + i] - b[2 + i]);
  }
  ns_material<T>(p, clamp1(ph1.v), P);
  const bool inside = ph1.v <= (T)1 && ph1.v >= (T)-1;
  const T gg = inside ? (T)p.gamma : (T)0;  // grad eta, zero where phi* is pulled back
  const T kap = (T)p.kappa;
  P.J[0] = kap * mut.dx;
  P.J[1] = kap * mut.dy;
  P.J[2] = kap * mut.dz;
  const T iPe = (T)p.inv_Pe, iRe = (T)p.inv_Re, iWe = (T)p.inv_We;
  P.adv[0] = P.rho * P.vt[0] + iPe * P.J[0] - iRe * gg * ph1.dx;
  P.adv[1] = P.rho * P.vt[1] + iPe * P.J[1] - iRe * gg * ph1.dy;
  P.adv[2] = P.rho * P.vt[2] + iPe * P.J[2] - iRe * gg * ph1.dz;
  P.gpht[0] = pht.dx;
  P.gpht[1] = pht.dy;
  P.gpht[2] = pht.dz;
  P.pt = pt.v;
  // capillary divergence (Cn/We) d/dx_j (dphi~/dx_i dphi~/dx_j): on trilinear
  // cells the Laplacian vanishes and only the mixed derivatives remain
  const T cw = (T)p.CnWe;
  const T cap[3] = {cw * (pht.dy * pht.dxy + pht.dz * pht.dxz),
                    cw * (pht.dx * pht.dxy + pht.dz * pht.dyz),
                    cw * (pht.dx * pht.dxz + pht.dy * pht.dyz)};
  const T gpt[3] = {pt.dx, pt.dy, pt.dz};
  const T ifr = (T)p.inv_Fr, idt = (T)p.inv_dt;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    P.tg[i] = P.rho * (dv[i] * idt - (T)p.g[i] * ifr);
    P.Rm[i] = P.tg[i] + P.adv[0] * P.G[i][0] + P.adv[1] * P.G[i][1] + P.adv[2] * P.G[i][2] +
              cap[i] + iWe * gpt[i];
  }
  ns_stab<T>(p, L, P);
}

// Residual rows of the NS block (momentum i = 0..2, continuity 3) at the point,
// contracted against the test functions of the lane's corner.
template <class T>
__device__ __forceinline__ void ns_residual_point(const PhysView& p, const Lane<T>& L,
                                                  const NSPoint<T>& P, T (&r)[4]) {
  const T w = L.wdet, iPe = (T)p.inv_Pe, iWe = (T)p.inv_We, tm = P.tau_m;
  const T er = P.eta * (T)p.inv_Re, cw = (T)p.CnWe;
  T W[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) W[j] = P.vt[j] + (P.J[j] * iPe - tm * P.Rm[j]) * P.inv_rho;
  const T dgl = iWe * (P.rho * P.tau_c * P.Rc - P.pt);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T c = P.tg[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) c += (P.rho * P.vt[j] + iPe * P.J[j] - tm * P.Rm[j]) * P.G[i][j];
    T F[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      F[j] = P.Rm[i] * tm * W[j] - cw * P.gpht[i] * P.gpht[j] + er * P.G[i][j];
    F[i] += dgl;
    r[i] = test_contract<T>(w * c, w * F[0], w * F[1], w * F[2], L);
  }
  const T q = tm * P.inv_rho * w;
  r[3] = test_contract<T>(w * P.Rc, q * P.Rm[0], q * P.Rm[1], q * P.Rm[2], L);
}

// Derivative of the NS integrand in the direction (dv, dp) of (v^{k+1},
// p^{k+1}) at the point: dvt = dv/2 (value and gradient), ddv = dv (value),
// dpt = dp/2.  Returns the coefficients (c, F) of the momentum rows i = 0..2
// and the continuity row 3, before the Gauss weight.
// LAP: the direction's v~ has a Laplacian (dlap, already halved) whose
// viscous part -(eta/Re) lap dv~_i enters dR_m (triquadratic leaves; on
// trilinear leaves it vanishes and the term is compiled out).
template <class T, bool LAP = false>
__device__ __forceinline__ void ns_jvp_coef(const PhysView& p, const NSPoint<T>& P,
                                            const VG<T> (&dvt)[3], const T (&ddv)[3],
                                            const VG<T>& dpt, T (&c)[4], T (&F)[4][3],
                                            const T* dlap = nullptr) {
  const T iPe = (T)p.inv_Pe, iWe = (T)p.inv_We, tm = P.tau_m, ir = P.inv_rho;
  const T er = P.eta * (T)p.inv_Re, idt = (T)p.inv_dt;
  T dG[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    dG[i][0] = dvt[i].dx;
    dG[i][1] = dvt[i].dy;
    dG[i][2] = dvt[i].dz;
  }
  const T dgp[3] = {dpt.dx, dpt.dy, dpt.dz};
  T dRm[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T t = P.rho * ddv[i] * idt + iWe * dgp[i];
#pragma unroll
    for (int j = 0; j < 3; ++j) t += P.adv[j] * dG[i][j] + P.rho * dvt[j].v * P.G[i][j];
    if constexpr (LAP) t -= P.eta * (T)p.inv_Re * dlap[i];
    dRm[i] = t;
  }
  const T dRc = dG[0][0] + dG[1][1] + dG[2][2];
  const T vdv = P.vt[0] * dvt[0].v + P.vt[1] * dvt[1].v + P.vt[2] * dvt[2].v;
  const T Jdv = P.J[0] * dvt[0].v + P.J[1] * dvt[1].v + P.J[2] * dvt[2].v;
  const T dbr = (T)2 * P.Gh * vdv + P.Gh * Jdv * ir * iPe;
  const T dtm = (T)-0.5 * tm * tm * tm * dbr;
  const T dtc = -P.tau_c * dtm * P.sbr;  // tau_c' = -tau_c tau_m' / tau_m
  T W[3], dW[3], dTR[3];  // dTR_j = d(tau_m R_m,j)
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    W[j] = P.vt[j] + (P.J[j] * iPe - tm * P.Rm[j]) * ir;
    dTR[j] = dtm * P.Rm[j] + tm * dRm[j];
    dW[j] = dvt[j].v - dTR[j] * ir;
  }
  const T dgl = iWe * (P.rho * (dtc * P.Rc + P.tau_c * dRc) - dpt.v);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T ci = P.rho * ddv[i] * idt;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      ci += (P.rho * P.vt[j] + iPe * P.J[j] - tm * P.Rm[j]) * dG[i][j] +
            (P.rho * dvt[j].v - dTR[j]) * P.G[i][j];
    c[i] = ci;
#pragma unroll
    for (int j = 0; j < 3; ++j) F[i][j] = dTR[i] * W[j] + P.Rm[i] * tm * dW[j] + er * dG[i][j];
    F[i][i] += dgl;
  }
  c[3] = dRc;
#pragma unroll
  for (int j = 0; j < 3; ++j) F[3][j] = dTR[j] * ir;
}

template <class T>
__device__ __forceinline__ void ns_jvp_point(const PhysView& p, const Lane<T>& L,
                                             const NSPoint<T>& P, const VG<T> (&dvt)[3],
                                             const T (&ddv)[3], const VG<T>& dpt, T (&r)[4]) {
  T c[4], F[4][3];
  ns_jvp_coef<T>(p, P, dvt, ddv, dpt, c, F);
  // the contraction is linear and wdet = h^3/8 is a power of two, so scaling
  // its result instead of its 16 inputs gives the same bits
  const T w = L.wdet;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = w * test_contract<T>(c[i], F[i][0], F[i][1], F[i][2], L);
}

template <class T>
__global__ __launch_bounds__(256) void k_ns_residual(MeshView m, PlanView pl, PhysView p,
                                                     ChunkCaps caps,
                                                     const double* __restrict__ U1,
                                                     const double* __restrict__ U0,
                                                     T* __restrict__ partial, int* __restrict__ flag) {
  extern __shared__ double smem_d[];
  using CL = ChunkLDS<T, 6, 0, 4>;
  CL S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const bool valid = e0 < m.E;
  const int64_t e = valid ? e0 : m.E - 1;
  Lane<T> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int ref = m.elem[e * 8 + L.c];
  S.stage(pl, U1, U0, (const double*)nullptr, 0, 0);
  __syncthreads();
  T c[CL::NV];
  S.corner(m, ref, c);
  const T a[6] = {c[0], c[1], c[2], c[3], c[4], c[5]};
  const T b[6] = {c[6], c[7], c[8], c[9], c[10], c[11]};
  NSPoint<T> P;
  ns_point<T>(p, L, a, b, P);
  T r[4];
  ns_residual_point<T>(p, L, P, r);
  if (valid && !P.ok) atomicOr(flag, 1);
  S.finish((threadIdx.x >> 3) * 8 + L.c, r, partial);
}

template <class T, class TS, class TD>
__global__ __launch_bounds__(256) void k_ns_jvp(MeshView m, PlanView pl, PhysView p, ChunkCaps caps,
                                                const TS* __restrict__ U1, const TS* __restrict__ U0,
                                                const TD* __restrict__ dU, int ldD, int offD,
                                                T* __restrict__ partial, const int* skip) {
  if (skip && *skip) return;  // GMRES control: this step is not needed
  extern __shared__ double smem_d[];
  using CL = ChunkLDS<T, 6, 4, 4>;
  CL S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int64_t e = e0 < m.E ? e0 : m.E - 1;
  Lane<T> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int ref = m.elem[e * 8 + L.c];
  S.stage(pl, U1, U0, dU, ldD, offD);
  __syncthreads();
  T c[CL::NV];
  S.corner(m, ref, c);
  const T a[6] = {c[0], c[1], c[2], c[3], c[4], c[5]};
  const T b[6] = {c[6], c[7], c[8], c[9], c[10], c[11]};
  NSPoint<T> P;
  ns_point<T>(p, L, a, b, P);
  VG<T> dvt[3];
  T ddv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const VG<T> g = eval_vg<T>(c[12 + i], L);
    ddv[i] = g.v;
    dvt[i].v = (T)0.5 * g.v;
    dvt[i].dx = (T)0.5 * g.dx;
    dvt[i].dy = (T)0.5 * g.dy;
    dvt[i].dz = (T)0.5 * g.dz;
  }
  const VG<T> dpt = eval_vg<T>((T)0.5 * c[15], L);
  T r[4];
  ns_jvp_point<T>(p, L, P, dvt, ddv, dpt, r);
  S.finish((threadIdx.x >> 3) * 8 + L.c, r, partial);
}

// ------------------------------------------ cached linearisation points ----
// Within one Newton iteration the state is fixed, so the quantities of the
// linearisation point at every Gauss point can be computed once and reused by
// every Jacobian-vector product of the linear solve.  Layout (structure of
// arrays per chunk, coalesced for the 256 lanes of the chunk's workgroup):
// lin[(chunk * NL + k) * 256 + lane] for the NL values of a block.
//
// NS block: 7 values per Gauss point, phi^{k+1} pulled back to [-1,1], the
// transport velocity of R_m and R_m itself, and 4 values per node, the
// midpoints u~, v~, w~, mu~ (mid[node * 4 + f]).  The JVP stages the nodal
// midpoints of the chunk's targets next to the direction and rebuilds v~, its
// gradient and J at the point with the evaluation the element loop runs
// anyway; that costs four butterflies per lane instead of 15 cached values
// (960 B per element in FP64).  rho, eta, 1/rho, R_c, tau_m and tau_c are
// recomputed too (ns_material, ns_stab).  What needs second derivatives (R_m)
// or the state at both time levels (the transport velocity) stays cached.
// CH block: 4 values, psi''(phi~) and v~.
constexpr int kNSLin = 7;
constexpr int kNSMid = 4;
constexpr int kCHLin = 4;

template <class T>
__device__ __forceinline__ void ns_lin_store(const NSPoint<T>& P, T* __restrict__ q) {
  q[0] = P.ps;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    q[(1 + i) * kChunkThreads] = P.adv[i];
    q[(4 + i) * kChunkThreads] = P.Rm[i];
  }
}

// The linearisation point from the cached values q and the lane's corner
// midpoints cm (u~, v~, w~, mu~).
template <class T>
__device__ __forceinline__ void ns_lin_unpack(const PhysView& p, const T (&q)[kNSLin], const T (&cm)[kNSMid],
                                              const Lane<T>& L, NSPoint<T>& P) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    P.adv[i] = q[1 + i];
    P.Rm[i] = q[4 + i];
    const VG<T> v = eval_vg<T>(cm[i], L);
    P.vt[i] = v.v;
    P.G[i][0] = v.dx;
    P.G[i][1] = v.dy;
    P.G[i][2] = v.dz;
  }
  const VG<T> mut = eval_vg<T>(cm[3], L);
  const T kap = (T)p.kappa;
  P.J[0] = kap * mut.dx;
  P.J[1] = kap * mut.dy;
  P.J[2] = kap * mut.dz;
  ns_material<T>(p, q[0], P);
  ns_stab<T>(p, L, P);
}

// Nodal midpoints of the NS linearisation point: u~, v~, w~, mu~ per node,
// with the arithmetic of the element loop's staging (both levels converted to
// T, then averaged).
template <class T, class TS>
__global__ __launch_bounds__(256) void k_ns_mid(int64_t n, const TS* __restrict__ U1, const TS* __restrict__ U0,
                                                T* __restrict__ mid) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * kNSMid;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = i / kNSMid;
    const int f = (int)(i - g * kNSMid), src = f < 3 ? 2 + f : 1;
    mid[i] = (T)0.5 * ((T)U1[g * 6 + src] + (T)U0[g * 6 + src]);
  }
}

// Linearisation points of every Gauss point of the mesh (one workgroup per
// chunk, as the element loop).
template <class T, class TS>
__global__ __launch_bounds__(256) void k_ns_lin(MeshView m, PlanView pl, PhysView p, ChunkCaps caps,
                                                const TS* __restrict__ U1, const TS* __restrict__ U0,
                                                T* __restrict__ lin) {
  extern __shared__ double smem_d[];
  using CL = ChunkLDS<T, 6, 0, 4>;
  CL S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int64_t e = e0 < m.E ? e0 : m.E - 1;
  Lane<T> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int ref = m.elem[e * 8 + L.c];
  S.stage(pl, U1, U0, (const TS*)nullptr, 0, 0);
  __syncthreads();
  T c[CL::NV];
  S.corner(m, ref, c);
  const T a[6] = {c[0], c[1], c[2], c[3], c[4], c[5]};
  const T b[6] = {c[6], c[7], c[8], c[9], c[10], c[11]};
  NSPoint<T> P;
  ns_point<T>(p, L, a, b, P);
  ns_lin_store<T>(P, lin + (int64_t)blockIdx.x * kNSLin * kChunkThreads + threadIdx.x);
}

template <class T, class TS>
__global__ __launch_bounds__(256) void k_ch_lin(MeshView m, PlanView pl, PhysView p, ChunkCaps caps,
                                                const TS* __restrict__ U1, const TS* __restrict__ U0,
                                                T* __restrict__ lin) {
  extern __shared__ double smem_d[];
  using CL = ChunkLDS<T, 5, 0, 2>;
  CL S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int64_t e = e0 < m.E ? e0 : m.E - 1;
  Lane<T> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int ref = m.elem[e * 8 + L.c];
  S.stage(pl, U1, U0, (const TS*)nullptr, 0, 0);
  __syncthreads();
  T c[CL::NV];  // phi, mu, u, v, w at k+1 and at k
  S.corner(m, ref, c);
  T* q = lin + (int64_t)blockIdx.x * kCHLin * kChunkThreads + threadIdx.x;
  q[0] = ch_dpsi<T>(eval_v<T>((T)0.5 * (c[0] + c[5])));
  q[kChunkThreads] = eval_v<T>((T)0.5 * (c[2] + c[7]));
  q[2 * kChunkThreads] = eval_v<T>((T)0.5 * (c[3] + c[8]));
  q[3 * kChunkThreads] = eval_v<T>((T)0.5 * (c[4] + c[9]));
}

// Prologue of the JVPs from cached linearisation points: stages, per target
// of the chunk, the ND-field direction followed by NM cached nodal values
// (mid[node * NM + f]), and the chunk's lists; loads the lane's NL cached
// values and returns the lane's corner record, ND + NM values (after the
// barrier).  The corner's record is found through the plan's corner map
// (cw = cmap[element * 8 + corner]): its position in the staged target list,
// or for a hanging corner the positions of its constraint parents, so no
// search of the target list is needed.  Vector memory counters retire in the
// order the loads were issued, so they are issued in the order they are
// needed: (1) the chunk's target and incidence lists and the lane's
// hanging-corner entry, (2) the cached values, which carry most of the bytes,
// (3) what depends on (1): the targets' records and the constraint weights of
// a hanging corner.  The LDS stores of (1) and (3) wait only for their own
// loads and (2) streams meanwhile.  The fixed per-thread counts cover chunks
// of up to 128 targets and 512 incidences; loops take anything beyond.
template <class T, class TD, int ND, int NM, int NL>
__device__ __forceinline__ void lin_prologue(ChunkLDS<T, 0, ND + NM, ND>& S, const MeshView& m,
                                             const PlanView& pl, int ch, int cw, const T* __restrict__ lin,
                                             const T* __restrict__ mid, const TD* __restrict__ dU, int ldD,
                                             int offD, T (&q)[NL], T (&c)[ND + NM]) {
  constexpr int NV = ND + NM;
  constexpr int SV = ChunkLDS<T, 0, NV, ND>::SV, KI = 2, KH = 4;
  // the direction and the nodal values are staged by separate passes over
  // (target, field) pairs, so that the lanes of a wave load from one array
  constexpr int KD = (128 * ND + kChunkThreads - 1) / kChunkThreads;
  constexpr int KM = NM > 0 ? (128 * NM + kChunkThreads - 1) / kChunkThreads : 0;
  static_assert(kChunkThreads % ND == 0 && (NM == 0 || kChunkThreads % NM == 0), "field counts");
  const int t = threadIdx.x;
  const int s0 = pl.tgt_off[ch], cnt = pl.tgt_off[ch + 1] - s0;
  const int i0 = pl.chunk_inc[ch], ni = pl.chunk_inc[ch + 1] - i0;
  S.s0 = s0;
  S.cnt = cnt;
  // (1) lists; indices past the end are clamped and their values dropped
  const int tg = pl.tgt[s0 + min(t, cnt - 1)];
  const int io = pl.inc_off[s0 + min(t, cnt)];
  int gd[KD], gm[KM > 0 ? KM : 1], icv[KI];
  float iwv[KI];
#pragma unroll
  for (int k = 0; k < KD; ++k) gd[k] = pl.tgt[s0 + min((t + k * kChunkThreads) / ND, cnt - 1)];
  if constexpr (KM > 0) {
#pragma unroll
    for (int k = 0; k < KM; ++k) gm[k] = pl.tgt[s0 + min((t + k * kChunkThreads) / NM, cnt - 1)];
  }
#pragma unroll
  for (int k = 0; k < KI; ++k) {
    const int i = i0 + min(t + k * kChunkThreads, ni - 1);
    iwv[k] = pl.inc_w[i];
    icv[k] = pl.inc_corner[i];
  }
  int4 he0 = {0, 0, -1, -1}, he1 = {-1, -1, 0, 0};  // hanging entry: row start, count, positions
  if (cw < 0) {
    const int4* he = reinterpret_cast<const int4*>(pl.hmap + (int64_t)(-1 - cw) * kHMapDev);
    he0 = he[0];
    he1 = he[1];
  }
  __builtin_amdgcn_sched_barrier(0);
  // (2)
  const T* ql = lin + (int64_t)ch * NL * kChunkThreads + t;
#pragma unroll
  for (int k = 0; k < NL; ++k) q[k] = ql[k * kChunkThreads];
  __builtin_amdgcn_sched_barrier(0);
  // (3)
  T dv[KD], mv[KM > 0 ? KM : 1];
#pragma unroll
  for (int k = 0; k < KD; ++k) dv[k] = (T)dU[(int64_t)gd[k] * ldD + offD + t % ND];
  if constexpr (KM > 0) {
#pragma unroll
    for (int k = 0; k < KM; ++k) mv[k] = mid[(int64_t)gm[k] * NM + t % NM];
  }
  const int h0 = he0.x, h1 = he0.x + he0.y;
  T hwt[KH];
  if (cw < 0) {
    const auto* w = weights<T>(m);
#pragma unroll
    for (int k = 0; k < KH; ++k) hwt[k] = w[min(h0 + k, h1 - 1)];
  }
  if (t < cnt) S.tgt[t] = tg;
  if (t <= cnt) S.ioff[t] = io - i0;
#pragma unroll
  for (int k = 0; k < KI; ++k)
    if (t + k * kChunkThreads < ni) {
      S.iw[t + k * kChunkThreads] = iwv[k];
      S.icor[t + k * kChunkThreads] = (uint8_t)icv[k];
    }
#pragma unroll
  for (int k = 0; k < KD; ++k) {
    const int i = t + k * kChunkThreads;
    if (i < cnt * ND) S.val[(i / ND) * SV + i % ND] = dv[k];
  }
  if constexpr (KM > 0) {
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const int i = t + k * kChunkThreads;
      if (i < cnt * NM) S.val[(i / NM) * SV + ND + i % NM] = mv[k];
    }
  }
  // chunks beyond the fixed counts
  for (int i = t + kChunkThreads; i <= cnt; i += kChunkThreads) {
    if (i < cnt) S.tgt[i] = pl.tgt[s0 + i];
    S.ioff[i] = pl.inc_off[s0 + i] - i0;
  }
  for (int i = t + KI * kChunkThreads; i < ni; i += kChunkThreads) {
    S.iw[i] = pl.inc_w[i0 + i];
    S.icor[i] = pl.inc_corner[i0 + i];
  }
  for (int i = t + KD * kChunkThreads; i < cnt * ND; i += kChunkThreads)
    S.val[(i / ND) * SV + i % ND] = (T)dU[(int64_t)pl.tgt[s0 + i / ND] * ldD + offD + i % ND];
  if constexpr (KM > 0) {
    for (int i = t + KM * kChunkThreads; i < cnt * NM; i += kChunkThreads)
      S.val[(i / NM) * SV + ND + i % NM] = mid[(int64_t)pl.tgt[s0 + i / NM] * NM + i % NM];
  }
  __syncthreads();
  // the lane's corner: its node, or its constraint's parents in row order
  if (cw >= 0) {
    const T* v = S.val + cw * SV;
#pragma unroll
    for (int f = 0; f < NV; ++f) c[f] = v[f];
  } else {
    const int pk[8] = {he0.z & 0xFFFF, (int)((unsigned)he0.z >> 16), he0.w & 0xFFFF, (int)((unsigned)he0.w >> 16),
                       he1.x & 0xFFFF, (int)((unsigned)he1.x >> 16), he1.y & 0xFFFF, (int)((unsigned)he1.y >> 16)};
#pragma unroll
    for (int f = 0; f < NV; ++f) c[f] = (T)0;
#pragma unroll
    for (int k = 0; k < KH; ++k)
      if (h0 + k < h1) {
        const T* v = S.val + pk[k] * SV;
#pragma unroll
        for (int f = 0; f < NV; ++f) c[f] += hwt[k] * v[f];
      }
    const auto* w = weights<T>(m);
#pragma unroll
    for (int k = KH; k < 8; ++k)
      if (h0 + k < h1) {
        const T wk = w[h0 + k];
        const T* v = S.val + pk[k] * SV;
#pragma unroll
        for (int f = 0; f < NV; ++f) c[f] += wk * v[f];
      }
  }
}

// The NS Jacobian-vector product from the cached linearisation points.
template <class T, class TD>
__global__ __launch_bounds__(256) void k_ns_jvp_lin(MeshView m, PlanView pl, PhysView p, ChunkCaps caps,
                                                    const T* __restrict__ lin, const T* __restrict__ mid,
                                                    const TD* __restrict__ dU, int ldD, int offD,
                                                    T* __restrict__ partial, const int* skip) {
  if (skip && *skip) return;  // GMRES control: this step is not needed
  extern __shared__ double smem_d[];
  ChunkLDS<T, 0, 4 + kNSMid, 4> S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * kChunkThreads + threadIdx.x) >> 3;
  const int64_t e = e0 < m.E ? e0 : m.E - 1;
  Lane<T> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int cw = pl.cmap[e * 8 + L.c];
  T q[kNSLin], c[4 + kNSMid];  // direction dv, dp, then the midpoints u~, v~, w~, mu~
  lin_prologue<T, TD, 4, kNSMid, kNSLin>(S, m, pl, blockIdx.x, cw, lin, mid, dU, ldD, offD, q, c);
  NSPoint<T> P;
  const T cm[kNSMid] = {c[4], c[5], c[6], c[7]};
  ns_lin_unpack<T>(p, q, cm, L, P);
  VG<T> dvt[3];
  T ddv[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const VG<T> g = eval_vg<T>(c[i], L);
    ddv[i] = g.v;
    dvt[i].v = (T)0.5 * g.v;
    dvt[i].dx = (T)0.5 * g.dx;
    dvt[i].dy = (T)0.5 * g.dy;
    dvt[i].dz = (T)0.5 * g.dz;
  }
  const VG<T> dpt = eval_vg<T>((T)0.5 * c[3], L);
  T r[4];
  ns_jvp_point<T>(p, L, P, dvt, ddv, dpt, r);
  S.finish((threadIdx.x >> 3) * 8 + L.c, r, partial);
}

// The CH Jacobian-vector product from the cached linearisation points.
template <class T, class TD>
__global__ __launch_bounds__(256) void k_ch_jvp_lin(MeshView m, PlanView pl, PhysView p, ChunkCaps caps,
                                                    const T* __restrict__ lin, const TD* __restrict__ dU,
                                                    int ldD, int offD, T* __restrict__ partial,
                                                    const int* skip) {
  if (skip && *skip) return;  // GMRES control: this step is not needed
  extern __shared__ double smem_d[];
  ChunkLDS<T, 0, 2, 2> S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * kChunkThreads + threadIdx.x) >> 3;
  const int64_t e = e0 < m.E ? e0 : m.E - 1;
  Lane<T> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int cw = pl.cmap[e * 8 + L.c];
  T q[kCHLin], c[2];
  lin_prologue<T, TD, 2, 0, kCHLin>(S, m, pl, blockIdx.x, cw, lin, (const T*)nullptr, dU, ldD, offD, q, c);
  const VG<T> dp = eval_vg<T>(c[0], L);
  const VG<T> dm = eval_vg<T>(c[1], L);
  T r[2];
  ch_jvp_point<T>(p, L, q[0], q[1], q[2], q[3], dp, dm, r);
  S.finish((threadIdx.x >> 3) * 8 + L.c, r, partial);
}

// ---------------------------------------------- coupled Jacobian rows ----
// Rows of one block of the coupled Jacobian applied to dU (all six fields of
// U^{k+1}): the block's residual evaluated in dual numbers whose derivative
// parts carry dU, so every dependence (the other block's fields included) is
// differentiated exactly.
template <class T, class TS, class TD>
__global__ __launch_bounds__(256) void k_ch_jvp_full(MeshView m, PlanView pl, PhysView p, ChunkCaps caps,
                                                     const TS* __restrict__ U1, const TS* __restrict__ U0,
                                                     const TD* __restrict__ dU, T* __restrict__ partial,
                                                     const int* skip) {
  if (skip && *skip) return;
  using D = Dual<T>;
  extern __shared__ double smem_d[];
  using CL = ChunkLDS<T, 5, 5, 2>;
  CL S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int64_t e = e0 < m.E ? e0 : m.E - 1;
  Lane<D> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int ref = m.elem[e * 8 + L.c];
  S.stage(pl, U1, U0, dU, 6, 0);
  __syncthreads();
  T c[CL::NV];  // phi, mu, u, v, w at k+1, at k, then their directions
  S.corner(m, ref, c);
  D a[5], b[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    a[f] = D(c[f], c[10 + f]);
    b[f] = D(c[5 + f]);
  }
  D r[2];
  ch_residual_point<D>(p, L, a, b, r);
  const T rt[2] = {r[0].d, r[1].d};
  S.finish((threadIdx.x >> 3) * 8 + L.c, rt, partial);
}

template <class T, class TS, class TD>
__global__ __launch_bounds__(256) void k_ns_jvp_full(MeshView m, PlanView pl, PhysView p, ChunkCaps caps,
                                                     const TS* __restrict__ U1, const TS* __restrict__ U0,
                                                     const TD* __restrict__ dU, T* __restrict__ partial,
                                                     const int* skip) {
  if (skip && *skip) return;
  using D = Dual<T>;
  extern __shared__ double smem_d[];
  using CL = ChunkLDS<T, 6, 6, 4>;
  CL S;
  S.carve((char*)smem_d, caps);
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int64_t e = e0 < m.E ? e0 : m.E - 1;
  Lane<D> L;
  L.init(threadIdx.x & 7, m.level[e]);
  const int ref = m.elem[e * 8 + L.c];
  S.stage(pl, U1, U0, dU, 6, 0);
  __syncthreads();
  T c[CL::NV];
  S.corner(m, ref, c);
  D a[6], b[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    a[f] = D(c[f], c[12 + f]);
    b[f] = D(c[6 + f]);
  }
  NSPoint<D> P;
  ns_point<D>(p, L, a, b, P);
  D r[4];
  ns_residual_point<D>(p, L, P, r);
  const T rt[4] = {r[0].d, r[1].d, r[2].d, r[3].d};
  S.finish((threadIdx.x >> 3) * 8 + L.c, rt, partial);
}

// -------------------------------------------------------- node gather ----
// acc[f] = the sum over node i's target slots k = node_off[i] .. node_off[i+1]-1,
// in that order, of partial[node_slot[k] * NF + f].  The ids of the first four
// slots, then their rows, are loaded before the first add, so a node waits
// for three loads in sequence instead of two per slot (past its last slot a
// node loads that slot again and does not add it).  Slots beyond the fourth
// follow in a loop.
template <int NF, class TP>
__device__ __forceinline__ void gather_node(const PlanView& pl, int64_t i, const TP* __restrict__ partial,
                                            TP (&acc)[NF]) {
  constexpr int U = 4;
  const int k0 = pl.node_off[i], k1 = pl.node_off[i + 1];
#pragma unroll
  for (int f = 0; f < NF; ++f) acc[f] = 0;
  if (k1 <= k0) return;
  int64_t sl[U];
#pragma unroll
  for (int u = 0; u < U; ++u) sl[u] = pl.node_slot[min(k0 + u, k1 - 1)];
  TP v[U][NF];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int f = 0; f < NF; ++f) v[u][f] = partial[sl[u] * NF + f];
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (k0 + u < k1)
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[f] += v[u][f];
  for (int k = k0 + U; k < k1; ++k) {
    const int64_t s = pl.node_slot[k];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] += partial[s * NF + f];
  }
}

// Every node sums its target slots in slot order and writes its rows of the
// output (ld values per node starting at off; with ld = 6 the other block's
// entries are set to 0).  Boundary rows of the NS block are written here too:
// MODE 1 (residual) velocity rows v^{k+1} - v^k on boundary nodes and the
// pressure row p^{k+1} - p^k of the pinned node; MODE 2 (JVP) the identity
// rows dU.
template <int NF, class TP, class TO, int MODE, bool KEEP = false>
__global__ void k_gather(PlanView pl, int64_t n, const TP* __restrict__ partial,
                         TO* __restrict__ out, int ld, int off, const double* __restrict__ U1,
                         const double* __restrict__ U0, const TO* __restrict__ dU, int ldD,
                         int offD, const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    TP acc[NF];
    gather_node<NF, TP>(pl, i, partial, acc);
    TO v[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] = (TO)acc[f];
    if constexpr (MODE != 0) {
      const uint8_t b = pl.bflags[i];
      if (b & 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
          v[d] = MODE == 1 ? (TO)(U1[i * 6 + 2 + d] - U0[i * 6 + 2 + d]) : dU[i * ldD + offD + d];
      }
      if (b & 2) v[3] = MODE == 1 ? (TO)(U1[i * 6 + 5] - U0[i * 6 + 5]) : dU[i * ldD + offD + 3];
    }
    TO* o = out + i * ld;
    if (ld == NF || KEEP) {  // KEEP: the other block's entries are left as they are
#pragma unroll
      for (int f = 0; f < NF; ++f) o[off + f] = v[f];
    } else {
      for (int f = 0; f < ld; ++f) o[f] = (f >= off && f < off + NF) ? v[f - off] : (TO)0;
    }
  }
}

// Node-block diagonal: node n sums its element touches; NS boundary rows
// become identity rows.
template <int NF>
__global__ void k_gather_diag(PlanView pl, int64_t n, const double* __restrict__ tbuf,
                              double* __restrict__ D) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc[NF * NF];
#pragma unroll
    for (int f = 0; f < NF * NF; ++f) acc[f] = 0;
    for (int64_t k = pl.ntouch_off[i]; k < pl.ntouch_off[i + 1]; ++k) {
      const int64_t t = pl.ntouch_slot[k];
#pragma unroll
      for (int f = 0; f < NF * NF; ++f) acc[f] += tbuf[t * NF * NF + f];
    }
    if (NF == 4) {
      const uint8_t b = pl.bflags[i];
      if (b & 1)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[r * 4 + c] = r == c ? 1.0 : 0.0;
      if (b & 2)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[12 + c] = c == 3 ? 1.0 : 0.0;
    }
#pragma unroll
    for (int f = 0; f < NF * NF; ++f) D[i * NF * NF + f] = acc[f];
  }
}

// ------------------------------------------------- node-block diagonal ----
// Diagonal block of node n: sum over elements of sum_{c,c'} P_cn P_c'n J_e[c][c'],
// where P_cn is 1 when corner c is node n, the constraint weight of n when c
// hangs on n, and 0 otherwise.  The element Jacobian is bilinear in (test,
// trial) function, so an element's share is the linearised integrand with
// the element's restriction of node n's shape function, s_n = sum_c P_cn N_c,
// as both the seed of field f and the test function of row i.  Each element
// visits the nodes it touches in the plan's order (touch_node); the lane
// evaluates s_n and its gradient at its Gauss point from its own corner's
// weight, and the 8 lanes sum.

// The NS linearised integrand (ns_jvp_coef) for a seed s in field FLD only
// (velocity component FLD < 3: dvt_FLD = s/2, ddv_FLD = s.v; pressure FLD == 3:
// dpt = s/2).  The terms of the other fields, which are zero, are left out.
template <class T, int FLD>
__device__ __forceinline__ void ns_seed_coef(const PhysView& p, const NSPoint<T>& P, const VG<T>& s,
                                             T (&c)[4], T (&F)[4][3]) {
  const T iPe = (T)p.inv_Pe, iWe = (T)p.inv_We, tm = P.tau_m, ir = P.inv_rho;
  const T er = P.eta * (T)p.inv_Re, idt = (T)p.inv_dt;
  const T g[3] = {s.dx, s.dy, s.dz};
  const T hv = (T)0.5 * s.v;
  T W[3], dTR[3], dW[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) W[j] = P.vt[j] + (P.J[j] * iPe - tm * P.Rm[j]) * ir;
  if constexpr (FLD < 3) {
    constexpr int f = FLD;
    T dRm[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) dRm[i] = P.rho * hv * P.G[i][f];
    dRm[f] += P.rho * s.v * idt + (T)0.5 * (P.adv[0] * g[0] + P.adv[1] * g[1] + P.adv[2] * g[2]);
    const T dRc = (T)0.5 * g[f];
    const T dbr = (T)2 * P.Gh * (P.vt[f] * hv) + P.Gh * (P.J[f] * hv) * ir * iPe;
    const T dtm = (T)-0.5 * tm * tm * tm * dbr;
    const T dtc = -P.tau_c * dtm * P.sbr;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      dTR[j] = dtm * P.Rm[j] + tm * dRm[j];
      dW[j] = -dTR[j] * ir;
    }
    dW[f] += hv;
    const T dgl = iWe * (P.rho * (dtc * P.Rc + P.tau_c * dRc));
    const T A[3] = {P.rho * P.vt[0] + iPe * P.J[0] - tm * P.Rm[0], P.rho * P.vt[1] + iPe * P.J[1] - tm * P.Rm[1],
                    P.rho * P.vt[2] + iPe * P.J[2] - tm * P.Rm[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T ci = P.rho * hv * P.G[i][f] - (dTR[0] * P.G[i][0] + dTR[1] * P.G[i][1] + dTR[2] * P.G[i][2]);
      if (i == f) ci += P.rho * s.v * idt + (T)0.5 * (A[0] * g[0] + A[1] * g[1] + A[2] * g[2]);
      c[i] = ci;
#pragma unroll
      for (int j = 0; j < 3; ++j) F[i][j] = dTR[i] * W[j] + P.Rm[i] * tm * dW[j];
      if (i == f)
#pragma unroll
        for (int j = 0; j < 3; ++j) F[i][j] += er * (T)0.5 * g[j];
      F[i][i] += dgl;
    }
    c[3] = dRc;
  } else {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      dTR[j] = tm * (iWe * (T)0.5 * g[j]);
      dW[j] = -dTR[j] * ir;
    }
    const T dgl = -iWe * hv;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      c[i] = -(dTR[0] * P.G[i][0] + dTR[1] * P.G[i][1] + dTR[2] * P.G[i][2]);
#pragma unroll
      for (int j = 0; j < 3; ++j) F[i][j] = dTR[i] * W[j] + P.Rm[i] * tm * dW[j];
      F[i][i] += dgl;
    }
    c[3] = (T)0;
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) F[3][j] = dTR[j] * ir;
}

// The CH linearised integrand (ch_jvp_point before the test functions) for a
// seed s in phi (FLD 0) or in mu (FLD 1) only.
template <class T, int FLD>
__device__ __forceinline__ void ch_seed_coef(const PhysView& p, T dpsi, const T (&v)[3], const VG<T>& s,
                                             T (&c)[2], T (&F)[2][3]) {
  const T g[3] = {s.dx, s.dy, s.dz};
  if constexpr (FLD == 0) {
    const T hp = (T)0.5 * s.v, hc = (T)0.5 * (T)p.Cn2;
    c[0] = s.v * (T)p.inv_dt;
    c[1] = dpsi * hp;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      F[0][j] = -v[j] * hp;
      F[1][j] = hc * g[j];
    }
  } else {
    const T hk = (T)0.5 * (T)p.inv_PeCn;
    c[0] = (T)0;
    c[1] = (T)-0.5 * s.v;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      F[0][j] = hk * g[j];
      F[1][j] = (T)0;
    }
  }
}

// Column FF of the NS node block at the lane's Gauss point: the seed s_n in
// field FF tested against s_n in every row i, v[i * 4 + FF].
template <class T, int FF>
__device__ __forceinline__ void ns_diag_column(const PhysView& p, const NSPoint<T>& P, const VG<T>& s, T w,
                                               T (&v)[16]) {
  T c[4], F[4][3];
  ns_seed_coef<T, FF>(p, P, s, c, F);
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i * 4 + FF] = w * (s.v * c[i] + s.dx * F[i][0] + s.dy * F[i][1] + s.dz * F[i][2]);
}

// Sum of 16 values over the 8 lanes of an element, scattered: lane l gets the
// sums of values 2l and 2l+1.  Three exchange stages (partners l^7, l^2, l^1)
// each halve the values a lane keeps; the order of the additions is fixed.
template <class T>
__device__ __forceinline__ void group_reduce_scatter16(T (&v)[16], int lane8, T& out0, T& out1) {
  T a[8], b[4];
  const bool u2 = (lane8 >> 2) & 1, u1 = (lane8 >> 1) & 1, u0 = lane8 & 1;
  // value k belongs to lane k >> 1: values 0..7 to lanes 0..3 (bit 2 clear),
  // 8..15 to lanes 4..7; each lane keeps the half its bit 2 selects
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const T send = u2 ? v[j] : v[j + 8];
    const T keep = u2 ? v[j + 8] : v[j];
    a[j] = keep + xchg<kXor7>(send);
  }
  // a[j]: value (u2 ? 8 : 0) + j; owners differ in bit 1 for j >> 2
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const T send = u1 ? a[j] : a[j + 4];
    const T keep = u1 ? a[j + 4] : a[j];
    b[j] = keep + xchg<kXor2>(send);
  }
  // b[j]: value (u2 ? 8 : 0) + (u1 ? 4 : 0) + j; owners differ in bit 0 for j >> 1
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const T send = u0 ? b[j] : b[j + 2];
    const T keep = u0 ? b[j + 2] : b[j];
    const T r = keep + xchg<kXor1>(send);
    if (j == 0) out0 = r; else out1 = r;
  }
}

template <class T, int BLOCK>
__global__ __launch_bounds__(256) void k_diag(MeshView m, PlanView pl, PhysView p,
                                              const double* __restrict__ U1,
                                              const double* __restrict__ U0,
                                              double* __restrict__ tbuf) {
  constexpr int NF = BLOCK == 0 ? 2 : 4;
  constexpr int KH = 4;
  const int64_t e0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const bool valid = e0 < m.E;
  const int64_t e = valid ? e0 : m.E - 1;
  const int lane8 = threadIdx.x & 7;
  Lane<T> L;
  L.init(lane8, m.level[e]);
  const int ref = m.elem[e * 8 + L.c];
  T a[6], b[6];
  gather<double, T, 6>(m, ref, U1, 6, 0, a);
  gather<double, T, 6>(m, ref, U0, 6, 0, b);
  NSPoint<T> P;
  T dpsi = 0, ch_v[3] = {0, 0, 0};
  if (BLOCK == 1) {
    ns_point<T>(p, L, a, b, P);
  } else {
    dpsi = ch_dpsi<T>(eval_v<T>((T)0.5 * (a[0] + b[0])));
#pragma unroll
    for (int d = 0; d < 3; ++d) ch_v[d] = eval_v<T>((T)0.5 * (a[2 + d] + b[2 + d]));
  }
  // the lane's corner: its node, or the parents and weights of its constraint
  int hid[KH];
  T hwt[KH];
  int h0 = 0, h1 = 0;
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    hid[k] = -1;
    hwt[k] = (T)0;
  }
  const auto* wts = weights<T>(m);
  if (ref < 0) {
    h0 = m.hoff[-1 - ref];
    h1 = m.hoff[-ref];
#pragma unroll
    for (int k = 0; k < KH; ++k)
      if (h0 + k < h1) {
        hid[k] = m.hids[h0 + k];
        hwt[k] = wts[h0 + k];
      }
  }
  const T w = L.wdet;
  const int64_t t0 = pl.touch_off[e], t1 = pl.touch_off[e + 1];  // the same for the element's 8 lanes
  for (int64_t t = t0; t < t1; ++t) {
    const int n = pl.touch_node[t];
    // P_cn of the lane's corner, then s_n at the lane's Gauss point
    T pw = (T)0;
    if (ref >= 0) {
      pw = ref == n ? (T)1 : (T)0;
    } else {
#pragma unroll
      for (int k = 0; k < KH; ++k)
        if (hid[k] == n) pw += hwt[k];
      for (int j = h0 + KH; j < h1; ++j)
        if (m.hids[j] == n) pw += wts[j];
    }
    const VG<T> sg = eval_vg<T>(pw, L);
    T v[NF * NF];
    if constexpr (BLOCK == 1) {
      ns_diag_column<T, 0>(p, P, sg, w, v);
      ns_diag_column<T, 1>(p, P, sg, w, v);
      ns_diag_column<T, 2>(p, P, sg, w, v);
      ns_diag_column<T, 3>(p, P, sg, w, v);
      T r0, r1;
      group_reduce_scatter16<T>(v, lane8, r0, r1);
      if (valid) {
        tbuf[t * 16 + 2 * lane8] = (double)r0;
        tbuf[t * 16 + 2 * lane8 + 1] = (double)r1;
      }
    } else {
      T c[2], F[2][3];
      ch_seed_coef<T, 0>(p, dpsi, ch_v, sg, c, F);
#pragma unroll
      for (int i = 0; i < 2; ++i) v[i * 2] = w * (sg.v * c[i] + sg.dx * F[i][0] + sg.dy * F[i][1] + sg.dz * F[i][2]);
      ch_seed_coef<T, 1>(p, dpsi, ch_v, sg, c, F);
#pragma unroll
      for (int i = 0; i < 2; ++i)
        v[i * 2 + 1] = w * (sg.v * c[i] + sg.dx * F[i][0] + sg.dy * F[i][1] + sg.dz * F[i][2]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const T sum = group_sum<T>(v[k]);
        if (valid && lane8 == k) tbuf[t * 4 + k] = (double)sum;
      }
    }
  }
}

// ------------------------------------------------------- diagnostics ----
// Sums of phi and of the energy density over the Gauss points.  A workgroup
// takes 32 elements at a time (8 lanes each) and walks the mesh with stride
// 32 * gridDim.x; each lane group adds its element totals in element order,
// then lane 0 adds the 32 groups in order: part[b] (mass) and
// part[gridDim.x + b] (energy) for workgroup b, summed by k_finish_sum.
constexpr int kDiagBlocks = 2048;  // most workgroups of k_diagnostics
__host__ __device__ inline int diag_blocks(int64_t E) {
  return (int)(E < (int64_t)kDiagBlocks * 32 ? (E + 31) / 32 : kDiagBlocks);
}

__global__ __launch_bounds__(256) void k_diagnostics(MeshView m, PhysView p,
                                                     const int32_t* __restrict__ anchor,
                                                     double unit, const double* __restrict__ U,
                                                     double* __restrict__ part) {
  __shared__ double sh[2][32];
  double am = 0, ae = 0;
  // the loop bound is the same for the whole workgroup: every lane takes part
  // in the exchanges of group_sum
  for (int64_t base = (int64_t)blockIdx.x * 32; base < m.E; base += (int64_t)gridDim.x * 32) {
    const int64_t e0 = base + (threadIdx.x >> 3);
    const bool valid = e0 < m.E;
    const int64_t e = valid ? e0 : m.E - 1;
    Lane<double> L;
    L.init(threadIdx.x & 7, m.level[e]);
    const int ref = m.elem[e * 8 + L.c];
    double a[5];
    gather<double, double, 5>(m, ref, U, 6, 0, a);
    const VG<double> ph = eval_vg<double>(a[0], L);
    const double vx = eval_v<double>(a[2]), vy = eval_v<double>(a[3]), vz = eval_v<double>(a[4]);
    // Gauss point position: anchor + h (1 + s g)/2 per axis
    const double x = anchor[e * 3 + 0] * unit + 0.5 * L.h * (1.0 + (L.sxh > 0 ? kGauss : -kGauss));
    const double y = anchor[e * 3 + 1] * unit + 0.5 * L.h * (1.0 + (L.syh > 0 ? kGauss : -kGauss));
    const double z = anchor[e * 3 + 2] * unit + 0.5 * L.h * (1.0 + (L.szh > 0 ? kGauss : -kGauss));
    const double rho = p.alpha * clamp1(ph.v) + p.beta;
    const double psi = 0.25 * (ph.v * ph.v - 1.0) * (ph.v * ph.v - 1.0);
    const double g2 = ph.dx * ph.dx + ph.dy * ph.dy + ph.dz * ph.dz;
    const double en = 0.5 * rho * (vx * vx + vy * vy + vz * vz) +
                      p.inv_Fr * rho * -(p.g[0] * x + p.g[1] * y + p.g[2] * z);
    const double fe = (psi + 0.5 * p.Cn2 * g2) * p.inv_We / p.Cn;
    const double mass = group_sum<double>(L.wdet * ph.v);
    const double energy = group_sum<double>(L.wdet * (en + fe));
    if (valid) {
      am += mass;
      ae += energy;
    }
  }
  if ((threadIdx.x & 7) == 0) {
    sh[0][threadIdx.x >> 3] = am;
    sh[1][threadIdx.x >> 3] = ae;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0;
    for (int g = 0; g < 32; ++g) t += sh[threadIdx.x][g];
    part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

}  // namespace dev
}  // namespace chns
