// Vector kernels of the Newton-Krylov solver: fills, block extraction,
// (block) Jacobi, multi-vector dot products and updates for classical
// Gram-Schmidt GMRES.  Dot products accumulate in FP64 whatever the storage
// type; reductions go through per-block partials summed in a fixed order, so
// results do not depend on timing.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace chns {
namespace dev {

constexpr int kMaxBasis = 128;  // restart length + 1
constexpr int kDotTile = 32;    // basis vectors per multi-dot workgroup

// Kernels that run inside a GMRES cycle take a skip flag (device int): when
// it is set the whole grid returns at once.  The host can then enqueue a full
// restart cycle without reading anything back; the cycle's control kernels
// raise the flag once the iteration has stopped.
__device__ __forceinline__ bool skipped(const int* skip) { return skip && *skip; }

template <class T>
__global__ void k_fill(T* __restrict__ x, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

template <class TA, class TB>
__global__ void k_convert(const TA* __restrict__ a, TB* __restrict__ b, int64_t n, const int* skip) {
  if (skipped(skip)) return;
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

// out[j * stride] = the block's sum of v[j], for j < kk: for every j the wave
// butterfly and the in-order sum over waves of block_reduce_sum (so the bits
// are those of kk calls of it), behind one barrier instead of 2 kk.
// sh holds (blockDim.x / 64) * K doubles.
template <int K>
__device__ __forceinline__ void block_reduce_sums(const double (&v)[K], int kk, double* sh,
                                                  double* __restrict__ out, int64_t stride) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < kk) {
      double x = v[j];
      for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
      if (l == 0) sh[w * K + j] = x;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < kk) {
    double r = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i * K + threadIdx.x];
    out[(int64_t)threadIdx.x * stride] = r;
  }
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

// f(std::integral_constant<int, kk>) for 1 <= kk <= K: the loops below get
// compile-time trip counts, so a row's loads of all kk basis vectors are
// issued before the first wait (a loop over a runtime count with a guarded
// load per vector waits for each load before issuing the next).
template <int K, class F>
__device__ __forceinline__ void with_count(int kk, F&& f) {
  if constexpr (K > 0) {
    if (kk == K)
      f(std::integral_constant<int, K>{});
    else
      with_count<K - 1>(kk, f);
  }
}

template <class TV, int K>
__device__ __forceinline__ void multidot_rows(const TV* __restrict__ Vt, int64_t stride,
                                              const TV* __restrict__ w, int64_t n, double (&acc)[kDotTile]) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = (double)w[i];
    TV v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = Vt[j * stride + i];
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] += (double)v[j] * wi;
  }
}

// w -= sum_j c_j V_j row by row, then the dots of the updated w with the same
// K basis entries of the row, kept in registers.
template <class TV, int K>
__device__ __forceinline__ void axpy_multidot_rows(TV* __restrict__ w, const TV* __restrict__ V, int64_t stride,
                                                   const double* cc, int64_t n, double (&acc)[kDotTile]) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    TV v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = V[j * stride + i];
    double s = (double)w[i];
#pragma unroll
    for (int j = 0; j < K; ++j) s -= cc[j] * (double)v[j];
    const TV st = (TV)s;
    w[i] = st;
    const double wi = (double)st;
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] += (double)v[j] * wi;
  }
}

// part[j * gridDim.x + b] = partial sum over block b of V_j . w, j < k.
// blockIdx.y picks a tile of kDotTile basis vectors (grid.y = ceil(k / kDotTile)).
template <class TV>
__global__ __launch_bounds__(256) void k_multidot(const TV* __restrict__ V, int64_t stride, int k,
                                                  const TV* __restrict__ w, int64_t n,
                                                  double* __restrict__ part, const int* skip) {
  if (skipped(skip)) return;
  __shared__ double shm[4 * kDotTile];
  const int j0 = blockIdx.y * kDotTile;
  const int kk = min(kDotTile, k - j0);
  const TV* __restrict__ Vt = V + (int64_t)j0 * stride;
  double acc[kDotTile];
#pragma unroll
  for (int j = 0; j < kDotTile; ++j) acc[j] = 0;
  with_count<kDotTile>(kk, [&](auto KC) { multidot_rows<TV, decltype(KC)::value>(Vt, stride, w, n, acc); });
  block_reduce_sums<kDotTile>(acc, kk, shm, part + (int64_t)j0 * gridDim.x + blockIdx.x, gridDim.x);
}

// w -= sum_{j<k} c_j V_j, then part[j * gridDim.x + b] = partial sum over
// block b of V_j . w (the updated w), for k <= kDotTile: the multi-axpy of
// one Gram-Schmidt pass and the multi-dot of the next in one sweep over the
// basis.  Row assignment, rounding of w and summation order are those of
// k_multi_axpy followed by k_multidot, so the results are the same.
template <class TV>
__global__ __launch_bounds__(256) void k_axpy_multidot(TV* __restrict__ w, const TV* __restrict__ V,
                                                       int64_t stride, int k, const double* __restrict__ c,
                                                       int64_t n, double* __restrict__ part, const int* skip) {
  if (skipped(skip)) return;
  __shared__ double shm[4 * kDotTile];
  __shared__ double cc[kDotTile];
  for (int j = threadIdx.x; j < k; j += blockDim.x) cc[j] = c[j];
  __syncthreads();
  double acc[kDotTile];
#pragma unroll
  for (int j = 0; j < kDotTile; ++j) acc[j] = 0;
  with_count<kDotTile>(k, [&](auto KC) { axpy_multidot_rows<TV, decltype(KC)::value>(w, V, stride, cc, n, acc); });
  block_reduce_sums<kDotTile>(acc, k, shm, part + blockIdx.x, gridDim.x);
}

// sum over b = threadIdx.x, threadIdx.x + blockDim.x, ... < nb of p[b], added
// in that order; the first four loads are issued before the first add (the
// partial counts here are at most 4 per thread).  Lanes past the end load
// p[nb - 1] and do not add it; nb <= 0 gives 0 and reads nothing.
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int nb) {
  if (nb <= 0) return 0.0;
  const int t = threadIdx.x, d = blockDim.x;
  double v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = p[min(t + u * d, nb - 1)];
  double s = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (t + u * d < nb) s += v[u];
  for (int b = t + 4 * d; b < nb; b += d) s += p[b];
  return s;
}

// out[j] = sum_b part[j * nb + b] in block order
__global__ void k_finish_sum(const double* __restrict__ part, int nb, int k, double* __restrict__ out,
                             const int* skip) {
  if (skipped(skip)) return;
  __shared__ double sh[4];
  for (int j = blockIdx.x; j < k; j += gridDim.x) {
    double s = strided_sum(part + (int64_t)j * nb, nb);
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

// w -= sum_{j<k} c_j V_j  (c in device memory, staged in LDS)
template <class TV>
__global__ __launch_bounds__(256) void k_multi_axpy(TV* __restrict__ w, const TV* __restrict__ V,
                                                    int64_t stride, int k, const double* __restrict__ c,
                                                    int64_t n, const int* skip) {
  if (skipped(skip)) return;
  __shared__ double cc[kMaxBasis];
  for (int j = threadIdx.x; j < k; j += blockDim.x) cc[j] = c[j];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = (double)w[i];
#pragma unroll 8
    for (int j = 0; j < k; ++j) s -= cc[j] * (double)V[j * stride + i];
    w[i] = (TV)s;
  }
}

// w -= sum_{j<k} c_j V_j and the partial sums of w . w (slot 0)
template <class TV>
__global__ __launch_bounds__(256) void k_axpy_norm(TV* __restrict__ w, const TV* __restrict__ V,
                                                   int64_t stride, int k, const double* __restrict__ c,
                                                   int64_t n, double* __restrict__ part,
                                                   const int* skip) {
  if (skipped(skip)) return;
  __shared__ double sh[4];
  __shared__ double cc[kMaxBasis];
  for (int j = threadIdx.x; j < k; j += blockDim.x) cc[j] = c[j];
  __syncthreads();
  double acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = (double)w[i];
#pragma unroll 8
    for (int j = 0; j < k; ++j) s -= cc[j] * (double)V[j * stride + i];
    const TV st = (TV)s;
    w[i] = st;
    acc += (double)st * (double)st;
  }
  const double t = block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// x += sum_{j<*kp} c_j Z_j  (x in FP64; count and coefficients in device memory)
template <class TV>
__global__ __launch_bounds__(256) void k_multi_update(double* __restrict__ x, const TV* __restrict__ Z,
                                                      int64_t stride, const int* __restrict__ kp,
                                                      const double* __restrict__ c, int64_t n) {
  const int k = *kp;
  if (k == 0) return;
  __shared__ double cc[kMaxBasis];
  for (int j = threadIdx.x; j < k; j += blockDim.x) cc[j] = c[j];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = x[i];
#pragma unroll 8
    for (int j = 0; j < k; ++j) s += cc[j] * (double)Z[j * stride + i];
    x[i] = s;
  }
}

// y = (*a) * x
template <class TV>
__global__ void k_scale_dev(TV* __restrict__ y, const TV* __restrict__ x, const double* __restrict__ a,
                            int64_t n, const int* skip) {
  if (skipped(skip)) return;
  const double s = *a;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (TV)(s * (double)x[i]);
}

// ------------------------------------------------------ GMRES control ----
// State of one right-preconditioned restarted GMRES run, kept in device
// memory and advanced by single-workgroup kernels.  The host reads the first
// five ints after each cycle.
struct GmresCtl {
  int idle;      // 1: the Arnoldi steps still queued in this cycle do nothing
  int finished;  // 1: stopped (converged, breakdown, iteration cap or error)
  int its;       // Arnoldi steps taken
  int err;       // 1: a norm was not finite
  int kcols;     // Arnoldi columns of the current cycle
  int ncols;     // columns used by the last solution update
  int max_it, mres;
  double rtol, bn, beta;
  double inv_scale;  // 1/beta for V_0, then 1/h_{k+1,k} for V_{k+1}
  double h1[kMaxBasis], h2[kMaxBasis];
  double H[kMaxBasis * kMaxBasis];  // column k: H[i * kMaxBasis + k]
  double cs[kMaxBasis], sn[kMaxBasis], g[kMaxBasis + 1], y[kMaxBasis];
};

// fixed-order sum of nb partials, valid on thread 0
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nb) {
  __shared__ double sh[4];
  return block_reduce_sum(strided_sum(part, nb), sh);
}

// Starts a run from the partial sums of b . b (x_0 = 0, so r_0 = b).
__global__ void k_gmres_begin(GmresCtl* __restrict__ C, const double* __restrict__ part, int nb,
                              int max_it, int mres, double rtol) {
  const double bb = sum_partials(part, nb);
  if (threadIdx.x != 0) return;
  const double bn = sqrt(bb);
  C->its = 0;
  C->err = 0;
  C->kcols = 0;
  C->ncols = 0;
  C->max_it = max_it;
  C->mres = mres;
  C->rtol = rtol;
  C->bn = bn;
  C->beta = bn;
  C->inv_scale = 0.0;
  C->g[0] = bn;
  if (!isfinite(bn)) C->err = 1;
  const bool stop = C->err || bn == 0.0 || max_it <= 0;
  C->finished = stop ? 1 : 0;
  C->idle = stop ? 1 : 0;
  if (!stop) C->inv_scale = 1.0 / bn;
}

// Closes Arnoldi step k: column k of H from the two Gram-Schmidt passes, the
// new norm h_{k+1,k} from the partial sums of w . w, the Givens rotations and
// the stopping test.  One workgroup; the rotation chain runs on thread 0 over
// the column staged in LDS.
__global__ __launch_bounds__(256) void k_arnoldi_close(GmresCtl* __restrict__ C, int k,
                                                       const double* __restrict__ part, int nb) {
  if (C->idle) return;
  __shared__ double col[kMaxBasis + 1];
  for (int j = threadIdx.x; j <= k; j += blockDim.x) col[j] = C->h1[j] + C->h2[j];
  const double hh = sum_partials(part, nb);  // synchronises the workgroup
  if (threadIdx.x != 0) return;
  const int ld = kMaxBasis;
  double* H = C->H;
  const double hn = sqrt(hh);
  C->its += 1;
  C->kcols = k + 1;
  if (!isfinite(hn)) {
    C->err = 1;
    C->finished = 1;
    C->idle = 1;
    return;
  }
  C->inv_scale = hn > 0 ? 1.0 / hn : 0.0;
  col[k + 1] = hn;
  for (int j = 0; j < k; ++j) {
    const double a = col[j], b = col[j + 1];
    col[j] = C->cs[j] * a + C->sn[j] * b;
    col[j + 1] = -C->sn[j] * a + C->cs[j] * b;
  }
  const double a = col[k], b = col[k + 1];
  const double den = hypot(a, b);
  C->cs[k] = den > 0 ? a / den : 1.0;
  C->sn[k] = den > 0 ? b / den : 0.0;
  col[k] = den;
  for (int j = 0; j <= k; ++j) H[j * ld + k] = col[j];
  H[(k + 1) * ld + k] = 0.0;
  C->g[k + 1] = -C->sn[k] * C->g[k];
  C->g[k] = C->cs[k] * C->g[k];
  if (fabs(C->g[k + 1]) <= C->rtol * C->bn || den == 0.0 || hn == 0.0 || C->its >= C->max_it) {
    C->finished = 1;
    C->idle = 1;
  } else if (k + 1 >= C->mres) {
    C->idle = 1;
  }
}

// Back substitution H y = g over the cycle's columns, column by column (one
// workgroup: y_i on thread 0, then every thread updates the rows above).
__global__ __launch_bounds__(256) void k_gmres_solve(GmresCtl* __restrict__ C) {
  __shared__ double gg[kMaxBasis + 1];
  __shared__ double yi;
  const int k = C->kcols, ld = kMaxBasis;
  for (int i = threadIdx.x; i < k; i += blockDim.x) gg[i] = C->g[i];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const double d = C->H[i * ld + i];
      yi = d != 0 ? gg[i] / d : 0.0;
      C->y[i] = yi;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < i; j += blockDim.x) gg[j] -= C->H[j * ld + i] * yi;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    C->ncols = k;
    C->kcols = 0;
  }
}

// New cycle from the partial sums of r . r, r = b - J x.
__global__ void k_gmres_restart(GmresCtl* __restrict__ C, const double* __restrict__ part, int nb) {
  if (C->finished) return;
  const double rr = sum_partials(part, nb);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(rr);
  C->beta = beta;
  if (!isfinite(beta)) {
    C->err = 1;
    C->finished = 1;
    return;
  }
  if (beta <= C->rtol * C->bn) {
    C->finished = 1;
    return;
  }
  C->g[0] = beta;
  C->inv_scale = 1.0 / beta;
  C->idle = 0;
}

// out[i*nf + f] = v[i*ld + off + f]: one block's part of a node-major vector
template <class TV>
__global__ void k_pack(const TV* __restrict__ v, int ld, int off, int nf, int64_t n, TV* __restrict__ out,
                       const int* skip) {
  if (skipped(skip)) return;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * nf;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / nf;
    out[t] = v[i * ld + off + (t - i * nf)];
  }
}

// z[i*ld + off + f] = in[i*nf + f]
template <class TV>
__global__ void k_unpack(const TV* __restrict__ in, int nf, int64_t n, TV* __restrict__ z, int ld, int off,
                         const int* skip) {
  if (skipped(skip)) return;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * nf;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / nf;
    z[i * ld + off + (t - i * nf)] = in[t];
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
__global__ void k_rsub(TV* __restrict__ r, const TV* __restrict__ b, int64_t n, const int* skip) {
  if (skipped(skip)) return;
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
                          int64_t nn, const int* skip) {
  if (skipped(skip)) return;
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
