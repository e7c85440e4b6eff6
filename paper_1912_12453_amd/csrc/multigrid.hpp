// Device kernels of the octree multigrid V-cycle: state injection, residual
// restriction (P^T), correction prolongation (P) and damped node-block
// Jacobi smoothing.  Transfers are gathers over host-built CSR lists, so
// every result is summed in a fixed order.  Rows that the Navier-Stokes
// block holds by Dirichlet conditions (velocity on the boundary, pressure at
// the pinned node) take no coarse-grid correction and are smoothed exactly.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace chns {
namespace dev {

__device__ __forceinline__ bool dirichlet_row(uint8_t b, int block, int f) {
  return block == 1 && ((f < 3 && (b & 1)) || (f == 3 && (b & 2)));
}

// Uc[j] = Uf[inj[j]] for the 6 fields (and an FP32 copy when Uc32 is set)
__global__ void k_inject6(const double* __restrict__ Uf, const int32_t* __restrict__ inj, int64_t nc,
                          double* __restrict__ Uc, float* __restrict__ Uc32) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nc * 6;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / 6;
    const int f = (int)(t - j * 6);
    const double v = Uf[(int64_t)inj[j] * 6 + f];
    Uc[t] = v;
    if (Uc32) Uc32[t] = (float)v;
  }
}

// rc[j] = sum over the fine nodes i of node j's list of w * rf[i], coarse
// Dirichlet rows zero (the fine Dirichlet rows of rf are zero, as the residual
// gather writes them).  The lists are padded column-major (entry k of node j
// at k * nc + j) so that the lanes of a wave read consecutive entries; the
// dyadic weights are exact in FP32.  With xc set, the coarse level's first
// Jacobi step xc = omega Dic rc follows in the same kernel (as k_jacobi
// without Ax, same arithmetic).
template <int NF, class TV, class TM>
__global__ void k_restrict(const TV* __restrict__ rf, const int32_t* __restrict__ r_off,
                           const int32_t* __restrict__ r_eidx, const float* __restrict__ r_ew, int64_t nc,
                           const uint8_t* __restrict__ bf_c, int block, TV* __restrict__ rc,
                           const TM* __restrict__ Dic, double omega, TV* __restrict__ xc, const int* skip) {
  if (skip && *skip) return;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nc;
       j += (int64_t)gridDim.x * blockDim.x) {
    double acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0;
    const int cnt = r_off[j + 1] - r_off[j];
    // groups of U entries: ids and weights, then the rows, then the adds in
    // list order (entries past the end load the last one and are not added)
    constexpr int U = 8;
    for (int k = 0; k < cnt; k += U) {
      int64_t ii[U];
      double ww[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t q = (int64_t)min(k + u, cnt - 1) * nc + j;
        ii[u] = r_eidx[q];
        ww[u] = (double)r_ew[q];
      }
      TV vv[U][NF];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int f = 0; f < NF; ++f) vv[u][f] = rf[ii[u] * NF + f];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k + u < cnt)
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f] += ww[u] * (double)vv[u][f];
    }
    const uint8_t b = bf_c[j];
    TV v[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      v[f] = dirichlet_row(b, block, f) ? (TV)0 : (TV)acc[f];
      rc[j * NF + f] = v[f];
    }
    if (xc) {
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        TM sum = 0;
#pragma unroll
        for (int c = 0; c < NF; ++c) sum += Dic[j * NF * NF + f * NF + c] * (TM)v[c];
        const TM om = dirichlet_row(b, block, f) ? (TM)1 : (TM)omega;
        xc[j * NF + f] = (TV)(om * sum);
      }
    }
  }
}

// xf[i] += sum over coarse nodes j of node i's list of w * ec[j], Dirichlet
// rows untouched
template <int NF, class TV>
__global__ void k_prolong_add(TV* __restrict__ xf, const uint8_t* __restrict__ bf_f,
                              const int32_t* __restrict__ p_off, const int32_t* __restrict__ p_idx,
                              const double* __restrict__ p_w, int64_t nfn, const TV* __restrict__ ec,
                              int block, const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nfn;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0;
    const int k0 = p_off[i], k1 = p_off[i + 1];
    constexpr int U = 8;  // as in k_restrict
    for (int k = k0; k < k1; k += U) {
      int64_t jj[U];
      double ww[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = min(k + u, k1 - 1);
        jj[u] = p_idx[q];
        ww[u] = p_w[q];
      }
      TV vv[U][NF];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int f = 0; f < NF; ++f) vv[u][f] = ec[jj[u] * NF + f];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k + u < k1)
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f] += ww[u] * (double)vv[u][f];
    }
    const uint8_t b = bf_f[i];
#pragma unroll
    for (int f = 0; f < NF; ++f)
      if (!dirichlet_row(b, block, f)) xf[i * NF + f] = (TV)((double)xf[i * NF + f] + acc[f]);
  }
}

// Damped node-block Jacobi: x = omega Di b (Ax == nullptr, x starts at 0),
// else x += omega Di (b - Ax).  Dirichlet rows use omega = 1: their rows of
// the operator and of the diagonal block are identity rows, so they are then
// solved exactly.
template <int NF, class TV, class TM>
__global__ void k_jacobi(const TM* __restrict__ Di, const TV* __restrict__ b, const TV* __restrict__ Ax,
                         TV* __restrict__ x, const uint8_t* __restrict__ bf, int block, double omega,
                         int64_t n, const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    TM r[NF];
#pragma unroll
    for (int c = 0; c < NF; ++c) r[c] = Ax ? (TM)b[i * NF + c] - (TM)Ax[i * NF + c] : (TM)b[i * NF + c];
    const uint8_t bb = bf[i];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      TM s = 0;
#pragma unroll
      for (int c = 0; c < NF; ++c) s += Di[i * NF * NF + f * NF + c] * r[c];
      const TM om = dirichlet_row(bb, block, f) ? (TM)1 : (TM)omega;
      x[i * NF + f] = Ax ? (TV)((TM)x[i * NF + f] + om * s) : (TV)(om * s);
    }
  }
}

// The node gather of a V-cycle JVP v = A x (block vectors, NF fields per
// node; NS boundary rows are the identity rows of x) fused with what the
// cycle does next with v:
//   EPI 1  damped node-block Jacobi x += omega Di (b - v), omega = 1 on the
//          Dirichlet rows (as k_jacobi, same arithmetic);
//   EPI 2  the residual r = b - v (as k_rsub), zero on the Dirichlet rows.
template <int NF, class TV, class TM, int EPI>
__global__ void k_gather_vcycle(PlanView pl, int64_t n, const TV* __restrict__ partial, int block,
                                TV* __restrict__ x, const TV* __restrict__ b, const TM* __restrict__ Di,
                                double omega, TV* __restrict__ r, const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    TV acc[NF];
    gather_node<NF, TV>(pl, i, partial, acc);
    const uint8_t bb = pl.bflags[i];
    if (NF == 4 && block == 1) {
      if (bb & 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[d] = x[i * NF + d];
      if (bb & 2) acc[3] = x[i * NF + 3];
    }
    if constexpr (EPI == 1) {
      TM rr[NF];
#pragma unroll
      for (int c = 0; c < NF; ++c) rr[c] = (TM)b[i * NF + c] - (TM)acc[c];
      TV xn[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        TM sum = 0;
#pragma unroll
        for (int c = 0; c < NF; ++c) sum += Di[i * NF * NF + f * NF + c] * rr[c];
        const TM om = dirichlet_row(bb, block, f) ? (TM)1 : (TM)omega;
        xn[f] = (TV)((TM)x[i * NF + f] + om * sum);
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) x[i * NF + f] = xn[f];
    } else {  // Dirichlet rows take no coarse correction: their residual is zero
#pragma unroll
      for (int f = 0; f < NF; ++f) r[i * NF + f] = dirichlet_row(bb, block, f) ? (TV)0 : b[i * NF + f] - acc[f];
    }
  }
}

// Ut[i] = sum_k w[k] * Uf[idx[k]] for the 6 fields of node i (intergrid
// transfer, in the list's fixed order)
__global__ void k_interp6(const double* __restrict__ Uf, const int32_t* __restrict__ off,
                          const int32_t* __restrict__ idx, const double* __restrict__ w, int64_t n,
                          double* __restrict__ Ut) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int k = off[i]; k < off[i + 1]; ++k) {
      const int64_t j = idx[k];
      const double wk = w[k];
#pragma unroll
      for (int f = 0; f < 6; ++f) acc[f] += wk * Uf[j * 6 + f];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) Ut[i * 6 + f] = acc[f];
  }
}

// U[i][0] += c for every node (a constant shift of phi)
__global__ void k_shift_phi(double* __restrict__ U, int64_t n, const double* __restrict__ c) {
  const double s = *c;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    U[i * 6] += s;
}

}  // namespace dev
}  // namespace chns
