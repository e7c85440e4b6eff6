// Vector kernels of the Newton-Krylov solver: fills, block extraction,
// (block) Jacobi, multi-vector dot products and updates for classical
// Gram-Schmidt GMRES.  Dot products accumulate in FP64 whatever the storage
// type; reductions go through per-block partials summed in a fixed order, so
// results do not depend on timing.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace chns {
namespace dev {

constexpr int kMaxBasis = 32;  // restart length + 1 fits the by-value coefficient block
struct Coef {
  double c[kMaxBasis];
};

template <class T>
__global__ void k_fill(T* __restrict__ x, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

template <class TA, class TB>
__global__ void k_convert(const TA* __restrict__ a, TB* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (TB)a[i];
}

// U[n*6 + f0 + f] += s * x[n*nf + f]
template <class TX>
__global__ void k_add_block(double* __restrict__ U, const TX* __restrict__ x, int64_t nn, int f0,
                            int nf, double s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn * nf;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = i / nf;
    const int f = (int)(i - n * nf);
    U[n * 6 + f0 + f] += s * (double)x[i];
  }
}

__device__ __forceinline__ double block_reduce_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;  // valid on thread 0
}

// max that lets a NaN through (fmax would drop it)
__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ double block_reduce_max(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = nan_max(r, sh[i]);
  __syncthreads();
  return r;
}

// part[j * gridDim.x + b] = partial sum over block b of V_j . w, j < k
template <class TV>
__global__ __launch_bounds__(256) void k_multidot(const TV* __restrict__ V, int64_t stride, int k,
                                                  const TV* __restrict__ w, int64_t n,
                                                  double* __restrict__ part) {
  __shared__ double sh[4];
  double acc[kMaxBasis];
#pragma unroll
  for (int j = 0; j < kMaxBasis; ++j) acc[j] = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = (double)w[i];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j)
      if (j < k) acc[j] += (double)V[j * stride + i] * wi;
  }
  for (int j = 0; j < k; ++j) {
    const double s = block_reduce_sum(acc[j], sh);
    if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = s;
  }
}

// out[j] = sum_b part[j * nb + b] in block order
__global__ void k_finish_sum(const double* __restrict__ part, int nb, int k, double* __restrict__ out) {
  __shared__ double sh[4];
  for (int j = blockIdx.x; j < k; j += gridDim.x) {
    double s = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(int64_t)j * nb + b];
    s = block_reduce_sum(s, sh);
    if (threadIdx.x == 0) out[j] = s;
  }
}

__global__ void k_finish_max(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sh[4];
  double s = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s = nan_max(s, part[b]);
  s = block_reduce_max(s, sh);
  if (threadIdx.x == 0) out[0] = s;
}

// w -= sum_{j<k} c_j V_j
template <class TV>
__global__ void k_multi_axpy(TV* __restrict__ w, const TV* __restrict__ V, int64_t stride, int k,
                             Coef c, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = (double)w[i];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j)
      if (j < k) s -= c.c[j] * (double)V[j * stride + i];
    w[i] = (TV)s;
  }
}

// w -= sum_{j<k} c_j V_j and the partial sums of w . w (slot 0)
template <class TV>
__global__ __launch_bounds__(256) void k_axpy_norm(TV* __restrict__ w, const TV* __restrict__ V,
                                                   int64_t stride, int k, Coef c, int64_t n,
                                                   double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = (double)w[i];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j)
      if (j < k) s -= c.c[j] * (double)V[j * stride + i];
    const TV st = (TV)s;
    w[i] = st;
    acc += (double)st * (double)st;
  }
  const double t = block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// x += sum_{j<k} c_j Z_j  (x in FP64)
template <class TV>
__global__ void k_multi_update(double* __restrict__ x, const TV* __restrict__ Z, int64_t stride,
                               int k, Coef c, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = x[i];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j)
      if (j < k) s += c.c[j] * (double)Z[j * stride + i];
    x[i] = s;
  }
}

// y = a * x
template <class TA, class TB>
__global__ void k_scale(TB* __restrict__ y, const TA* __restrict__ x, double a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (TB)(a * (double)x[i]);
}

// r = b - r  (r holds J x on entry)
template <class TV>
__global__ void k_rsub(TV* __restrict__ r, const TV* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - r[i];
}

// Inverts the nf x nf node blocks (Gauss-Jordan with partial pivoting), or
// keeps the reciprocal of their diagonal (point Jacobi).  A zero pivot leaves
// the identity and raises *flag.
template <int NF>
__global__ void k_invert_blocks(const double* __restrict__ D, double* __restrict__ Di,
                                float* __restrict__ Di32, int64_t nn, int point,
                                int* __restrict__ flag) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  double A[NF][NF], B[NF][NF];
  for (int r = 0; r < NF; ++r)
    for (int c = 0; c < NF; ++c) {
      A[r][c] = D[n * NF * NF + r * NF + c];
      B[r][c] = r == c ? 1.0 : 0.0;
    }
  bool ok = true;
  if (point) {
    for (int r = 0; r < NF; ++r)
      for (int c = 0; c < NF; ++c) {
        if (r != c) continue;
        if (A[r][r] == 0.0) ok = false;
        B[r][r] = A[r][r] != 0.0 ? 1.0 / A[r][r] : 1.0;
      }
  } else {
    for (int c = 0; c < NF; ++c) {
      int piv = c;
      for (int r = c + 1; r < NF; ++r)
        if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
      if (A[piv][c] == 0.0) {
        ok = false;
        break;
      }
      if (piv != c)
        for (int k = 0; k < NF; ++k) {
          double t = A[c][k];
          A[c][k] = A[piv][k];
          A[piv][k] = t;
          t = B[c][k];
          B[c][k] = B[piv][k];
          B[piv][k] = t;
        }
      const double ip = 1.0 / A[c][c];
      for (int k = 0; k < NF; ++k) {
        A[c][k] *= ip;
        B[c][k] *= ip;
      }
      for (int r = 0; r < NF; ++r) {
        if (r == c) continue;
        const double f = A[r][c];
        for (int k = 0; k < NF; ++k) {
          A[r][k] -= f * A[c][k];
          B[r][k] -= f * B[c][k];
        }
      }
    }
    if (!ok)
      for (int r = 0; r < NF; ++r)
        for (int c = 0; c < NF; ++c) B[r][c] = r == c ? 1.0 : 0.0;
  }
  if (!ok) atomicOr(flag, 2);
  for (int r = 0; r < NF; ++r)
    for (int c = 0; c < NF; ++c) {
      Di[n * NF * NF + r * NF + c] = B[r][c];
      Di32[n * NF * NF + r * NF + c] = (float)B[r][c];
    }
}

// z = Dinv v, node by node
template <int NF, class TV, class TM>
__global__ void k_precond(const TM* __restrict__ Di, const TV* __restrict__ v, TV* __restrict__ z,
                          int64_t nn) {
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn;
       n += (int64_t)gridDim.x * blockDim.x) {
    TM x[NF];
#pragma unroll
    for (int c = 0; c < NF; ++c) x[c] = (TM)v[n * NF + c];
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      TM s = 0;
#pragma unroll
      for (int c = 0; c < NF; ++c) s += Di[n * NF * NF + r * NF + c] * x[c];
      z[n * NF + r] = (TV)s;
    }
  }
}

// part[b] = max over block b of |a - b|
__global__ void k_maxabs_diff(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                              double* __restrict__ part) {
  __shared__ double sh[4];
  double m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = nan_max(m, fabs(a[i] - b[i]));
  m = block_reduce_max(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

}  // namespace dev
}  // namespace chns
