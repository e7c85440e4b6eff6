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

// k_finish_sum over a count held in device memory (*kn sums).
__global__ void k_finish_sum_n(const double* __restrict__ part, int nb, const int* __restrict__ kn,
                               double* __restrict__ out, const int* skip) {
  if (skipped(skip)) return;
  __shared__ double sh[4];
  const int k = *kn;
  for (int j = blockIdx.x; j < k; j += gridDim.x) {
    double s = strided_sum(part + (int64_t)j * nb, nb);
    s = block_reduce_sum(s, sh);
    if (threadIdx.x == 0) out[j] = s;
  }
}

// ------------------------------------- Gram-Schmidt with delayed second pass --
// Arnoldi step k of GMRES uses classical Gram-Schmidt twice, but the second
// pass of basis vector k runs in step k + 1, fused with the first pass of the
// next vector (the delayed scheme of Bielich, Langou, Thomas, Swirydowicz,
// Yamazaki and Boman, Parallel Computing 2022).  At the start of step k the
// vectors V_0..V_{k-1} are final and V_k holds b v~_k: the provisional vector
// v~_k (one pass, unit norm) times its norm b (1 for V_0).  With
// w = J M^-1 v~_k, one sweep over the basis gives (divided by b or b^2)
// s_j = V_j.v~_k, t_j = V_j.w, sigma = v~_k.v~_k and tau = v~_k.w.  Then
//   v_k = (v~_k - sum_j s_j V_j) / alpha,  alpha = sqrt(sigma - s.s),
// column k-1 of the Hessenberg matrix takes its second-pass correction, and
// by the linearity of J M^-1 the product with the final v_k is
//   J M^-1 v_k = (w - V_{0..k} H_{0..k,0..k-1} s) / alpha,
// whose first-pass coefficients h follow from t, tau and s without another
// sweep.  A second sweep writes v_k and the new provisional vector w' = J M^-1 v_k
// - V_{0..k} h, unscaled, into V_{k+1}: its norm b (bprov) divides the next
// step's sums instead of a scaling pass.  Two sweeps over the basis per
// step instead of three.  The stored preconditioned vectors are those of the
// stored provisional vectors, Z~ = Z R with R the upper triangle of
// (b s, b alpha); the solution update uses R^-1 y.
constexpr int kDcTile = 16;  // basis vectors per dot workgroup (two sums each)

template <class TV, int K, bool W>
__device__ __forceinline__ void dc_dot_rows(const TV* __restrict__ Vt, int64_t stride, const TV* __restrict__ vk,
                                            const TV* __restrict__ w, int64_t n, bool self,
                                            double (&sa)[kDcTile], double (&ta)[kDcTile], double (&st)[2]) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    TV v[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = Vt[j * stride + i];
    const double x = (double)vk[i];
    const double y = W ? (double)w[i] : 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      sa[j] += (double)v[j] * x;
      if (W) ta[j] += (double)v[j] * y;
    }
    if (self) {
      st[0] += x * x;
      if (W) st[1] += x * y;
    }
  }
}

// Partial sums of step k (k from kdev when given): part[q * gridDim.x + b]
// with q = j: V_j.V_k, q = k + j: V_j.w (j < k; blockIdx.y picks kDcTile of
// them), q = 2k: V_k.V_k, q = 2k + 1: V_k.w (workgroups with blockIdx.y = 0).
// w == nullptr: the V_j.V_k and V_k.V_k sums only.
template <class TV>
__global__ __launch_bounds__(256) void k_dc_dots(const TV* __restrict__ V, int64_t stride, int k,
                                                 const int* __restrict__ kdev, const TV* __restrict__ w, int64_t n,
                                                 double* __restrict__ part, const int* skip) {
  if (skipped(skip)) return;
  if (kdev) k = *kdev;
  const int j0 = blockIdx.y * kDcTile;
  if (blockIdx.y > 0 && j0 >= k) return;  // whole workgroup: no basis vector in this tile
  __shared__ double shs[4 * kDcTile], sht[4 * kDcTile], shv[4 * 2];
  const int kk = max(0, min(kDcTile, k - j0));
  const bool self = blockIdx.y == 0;
  const TV* Vt = V + (int64_t)j0 * stride;
  const TV* vk = V + (int64_t)k * stride;
  double sa[kDcTile], ta[kDcTile], st[2] = {0.0, 0.0};
#pragma unroll
  for (int j = 0; j < kDcTile; ++j) sa[j] = ta[j] = 0.0;
  if (w) {
    if (kk == 0)
      dc_dot_rows<TV, 0, true>(Vt, stride, vk, w, n, self, sa, ta, st);
    else
      with_count<kDcTile>(kk, [&](auto KC) {
        dc_dot_rows<TV, decltype(KC)::value, true>(Vt, stride, vk, w, n, self, sa, ta, st);
      });
  } else {
    if (kk == 0)
      dc_dot_rows<TV, 0, false>(Vt, stride, vk, w, n, self, sa, ta, st);
    else
      with_count<kDcTile>(kk, [&](auto KC) {
        dc_dot_rows<TV, decltype(KC)::value, false>(Vt, stride, vk, w, n, self, sa, ta, st);
      });
  }
  const int nb = gridDim.x;
  block_reduce_sums<kDcTile>(sa, kk, shs, part + (int64_t)j0 * nb + blockIdx.x, nb);
  block_reduce_sums<kDcTile>(ta, w ? kk : 0, sht, part + (int64_t)(k + j0) * nb + blockIdx.x, nb);
  if (self) block_reduce_sums<2>(st, w ? 2 : 1, shv, part + (int64_t)(2 * k) * nb + blockIdx.x, nb);
}

// One row of the update sweep: v_k = (V_k / b - sum_j s_j V_j) / alpha into
// V_k and w' = w / (b alpha) - sum_{j<k} g_j V_j - g_k v_k into V_{k+1} (the
// stored vectors are b times the unit provisional vector and J M^-1 of it),
// then w'.w' (of the stored w').
template <class TV, int K>
__device__ __forceinline__ double dc_update_row(TV* __restrict__ V, int64_t stride, int k, const TV* __restrict__ w,
                                                int64_t i, const double* cs, const double* cg, double ia,
                                                double ib) {
  double a = (double)V[(int64_t)k * stride + i] * ib;
  double b = (double)w[i] * (ib * ia);
  if constexpr (K >= 0) {
    TV v[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) v[j] = V[j * stride + i];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      a -= cs[j] * (double)v[j];
      b -= cg[j] * (double)v[j];
    }
  } else {
#pragma unroll 8
    for (int j = 0; j < k; ++j) {
      const double v = (double)V[j * stride + i];
      a -= cs[j] * v;
      b -= cg[j] * v;
    }
  }
  a *= ia;
  b -= cg[k] * a;
  const TV bs = (TV)b;
  V[(int64_t)k * stride + i] = (TV)a;
  V[(int64_t)(k + 1) * stride + i] = bs;
  return (double)bs * (double)bs;
}

template <class TV, int K>
__device__ __forceinline__ double dc_update_rows(TV* __restrict__ V, int64_t stride, int k,
                                                 const TV* __restrict__ w, int64_t n, const double* cs,
                                                 const double* cg, double ia, double ib) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += dc_update_row<TV, K>(V, stride, k, w, i, cs, cg, ia, ib);
  return acc;
}

struct GmresCtl;
template <class TV>
__global__ __launch_bounds__(256) void k_dc_update(TV* __restrict__ V, int64_t stride, int k,
                                                   const TV* __restrict__ w, int64_t n,
                                                   const GmresCtl* __restrict__ C, double* __restrict__ part,
                                                   const int* skip);

__global__ void k_finish_max(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sh[4];
  double s = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s = nan_max(s, part[b]);
  s = block_reduce_max(s, sh);
  if (threadIdx.x == 0) out[0] = s;
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
  int its;       // Arnoldi columns completed
  int err;       // 1: a norm was not finite
  int kcols;     // completed Arnoldi columns of the current cycle
  int ncols;     // columns used by the last solution update
  int max_it, mres;
  int kprov;   // the column whose second Gram-Schmidt pass is pending, -1: none
  int noprov;  // 1 when kprov < 0 (the skip flag of the cycle's last pass)
  int kfin;    // kprov + 1, the basis vector that pass reorthogonalises
  int nfin;    // 2 kfin + 2, the count of its sums
  double rtol, bn, beta;
  double inv_scale;  // 1/beta for V_0
  double inv_alpha;  // 1/alpha of the step's reorthogonalised vector
  double bprov;      // norm of the stored provisional vector (1 for V_0)
  double inv_b;      // 1/bprov for the update sweep
  double dsum[2 * kMaxBasis + 2];       // the step's sums (see k_dc_dots)
  double cs_[kMaxBasis], cg_[kMaxBasis + 1];  // update coefficients s and g
  double Hr[(kMaxBasis + 1) * kMaxBasis];  // Hessenberg columns as built: (i, j) at Hr[i * kMaxBasis + j]
  double H[kMaxBasis * kMaxBasis];         // the rotated columns: (i, j) at H[i * kMaxBasis + j]
  double R[kMaxBasis * kMaxBasis];         // provisional-to-final basis change, same layout
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
  C->kprov = -1;
  C->noprov = 1;
  C->kfin = 0;
  C->nfin = 0;
  C->bprov = 1.0;
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

// Column j of the Hessenberg matrix is final: rotate it by the previous
// Givens rotations, make rotation j, advance the residual estimate g and test
// for the end of the run.  Thread 0 only; col is scratch for kMaxBasis + 1.
__device__ void close_column(GmresCtl* __restrict__ C, int j, double* col) {
  const int ld = kMaxBasis;
  for (int i = 0; i <= j + 1; ++i) col[i] = C->Hr[i * ld + j];
  const double hn = col[j + 1];
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = C->cs[i] * a + C->sn[i] * b;
    col[i + 1] = -C->sn[i] * a + C->cs[i] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double den = hypot(a, b);
  C->cs[j] = den > 0 ? a / den : 1.0;
  C->sn[j] = den > 0 ? b / den : 0.0;
  col[j] = den;
  for (int i = 0; i <= j; ++i) C->H[i * ld + j] = col[i];
  C->g[j + 1] = -C->sn[j] * C->g[j];
  C->g[j] = C->cs[j] * C->g[j];
  C->its += 1;
  C->kcols = j + 1;
  C->kprov = -1;
  C->noprov = 1;
  if (!isfinite(den)) C->err = 1;
  if (C->err || fabs(C->g[j + 1]) <= C->rtol * C->bn || den == 0.0 || hn == 0.0 || C->its >= C->max_it) {
    C->finished = 1;
    C->idle = 1;
  }
}

// The second pass of the provisional vector k from its sums (s_j = S[j],
// sigma = S[2k]): alpha, the correction of column k - 1 and its closing, and
// column k of R.  Thread 0 only; returns alpha.
__device__ double dc_reorth(GmresCtl* __restrict__ C, int k, double* col) {
  const int ld = kMaxBasis;
  const double* S = C->dsum;  // sums of the stored vector, bprov times the unit one
  const double b = C->bprov, ib = 1.0 / b;
  double ss = 0.0;
  for (int j = 0; j < k; ++j) ss += (S[j] * ib) * (S[j] * ib);
  const double a2 = S[2 * k] * ib * ib - ss;
  if (!isfinite(a2)) C->err = 1;
  const double alpha = a2 > 0.0 ? sqrt(a2) : 0.0;
  for (int j = 0; j < k; ++j) C->R[j * ld + k] = S[j];
  C->R[k * ld + k] = b * alpha;
  if (k == 0) {
    C->g[0] *= alpha;  // r = beta v~_0 = beta alpha v_0
    if (C->err || alpha == 0.0) {
      C->finished = 1;
      C->idle = 1;
    }
  } else {
    const double hk = C->Hr[k * ld + k - 1];
    for (int j = 0; j < k; ++j) C->Hr[j * ld + k - 1] += hk * (S[j] * ib);
    C->Hr[k * ld + k - 1] = hk * alpha;
    close_column(C, k - 1, col);  // alpha = 0: the Krylov space is invariant, the run ends
  }
  return alpha;
}

// Step k after its dot sweep: the second pass of v~_k, then the first-pass
// coefficients of J M^-1 v_k (column k of Hr) and the update coefficients.
__global__ __launch_bounds__(256) void k_dc_coef(GmresCtl* __restrict__ C, int k) {
  if (C->idle) return;
  __shared__ double col[kMaxBasis + 1];
  __shared__ double sh_alpha, sh_st;
  __shared__ int stop;
  const int ld = kMaxBasis;
  const double* S = C->dsum;
  const double ib = 1.0 / C->bprov;  // the sums below are of the unit provisional vector
  if (threadIdx.x == 0) {
    const double alpha = dc_reorth(C, k, col);
    double st = 0.0;
    for (int j = 0; j < k; ++j) st += (S[j] * ib) * (S[k + j] * ib);
    sh_alpha = alpha;
    sh_st = st;
    stop = C->idle;
  }
  __syncthreads();
  if (stop) return;
  const double ia = 1.0 / sh_alpha;
  for (int i = threadIdx.x; i <= k; i += blockDim.x) {
    double c = 0.0;  // (H_{0..k,0..k-1} s)_i; H is upper Hessenberg
    for (int j = i > 0 ? i - 1 : 0; j < k; ++j) c += C->Hr[i * ld + j] * (S[j] * ib);
    const double t = i < k ? S[k + i] * ib : (S[2 * k + 1] * ib * ib - sh_st) * ia;  // v_i . w / bprov
    const double h = (t - c) * ia;
    C->Hr[i * ld + k] = h;
    C->cg_[i] = c * ia + h;
    if (i < k) C->cs_[i] = S[i] * ib;
  }
  if (threadIdx.x == 0) {
    C->inv_alpha = ia;
    C->inv_b = ib;
  }
}

// After the update sweep of step k: the provisional norm of w' (column k's
// subdiagonal until the next step corrects it) from the partial sums of
// w'.w'.  A zero norm ends the run with column k final.
__global__ __launch_bounds__(256) void k_dc_norm(GmresCtl* __restrict__ C, int k, const double* __restrict__ part,
                                                 int nb) {
  if (C->idle) return;
  __shared__ double col[kMaxBasis + 1];
  const double ww = sum_partials(part, nb);  // synchronises the workgroup
  if (threadIdx.x != 0) return;
  const int ld = kMaxBasis;
  const double hn = sqrt(ww);
  if (!isfinite(hn)) {
    C->err = 1;
    C->finished = 1;
    C->idle = 1;
    return;
  }
  C->Hr[(k + 1) * ld + k] = hn;
  C->inv_scale = hn > 0 ? 1.0 / hn : 0.0;
  if (hn == 0.0) {
    close_column(C, k, col);
    return;
  }
  // V_{k+1} holds w' unscaled, even after the cycle's last step: the next
  // step's sums, or the cycle's final pass (k_dc_final), divide by bprov
  C->bprov = hn;
  C->kprov = k;
  C->noprov = 0;
  C->kfin = k + 1;
  C->nfin = 2 * (k + 1) + 2;
  // The stop test of column k with its provisional entries (the second pass
  // changes them by rounding-level amounts): when it passes, or the next
  // column would reach the iteration cap, no further step is taken and the
  // cycle's final pass closes column k with its exact test.
  for (int i = 0; i <= k; ++i) col[i] = C->Hr[i * ld + k];
  col[k + 1] = hn;
  for (int i = 0; i < k; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = C->cs[i] * a + C->sn[i] * b;
    col[i + 1] = -C->sn[i] * a + C->cs[i] * b;
  }
  const double den = hypot(col[k], col[k + 1]);
  const double gk1 = den > 0 ? fabs(col[k + 1] / den * C->g[k]) : 0.0;
  if (gk1 <= C->rtol * C->bn || C->its + 1 >= C->max_it) C->idle = 1;
}

// End of a cycle whose last column is provisional: its second pass from the
// sums of k_dc_dots (w == nullptr) and its closing.
__global__ __launch_bounds__(256) void k_dc_final(GmresCtl* __restrict__ C) {
  if (C->noprov) return;
  __shared__ double col[kMaxBasis + 1];
  if (threadIdx.x != 0) return;
  dc_reorth(C, C->kfin, col);
}

// The solution coefficients of the cycle: back substitution H y = g over the
// completed columns, then R y' = y (the stored vectors are Z~ = Z R), column
// by column (one workgroup: y_i on thread 0, then every thread updates the
// rows above).
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
    }
    __syncthreads();
    for (int j = threadIdx.x; j < i; j += blockDim.x) gg[j] -= C->H[j * ld + i] * yi;
    if (threadIdx.x == 0) gg[i] = yi;
    __syncthreads();
  }
  for (int i = k - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const double d = C->R[i * ld + i];
      yi = d != 0 ? gg[i] / d : 0.0;
      C->y[i] = yi;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < i; j += blockDim.x) gg[j] -= C->R[j * ld + i] * yi;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    C->ncols = k;
    C->kcols = 0;
  }
}

// The update sweep of step k: V_k <- v_k, V_{k+1} <- w' (unscaled) and the
// partial sums of w'.w' (part[b]).  Up to kDotTile basis vectors a row's
// loads are issued together; beyond, a loop reads them in order.
template <class TV>
__global__ __launch_bounds__(256) void k_dc_update(TV* __restrict__ V, int64_t stride, int k,
                                                   const TV* __restrict__ w, int64_t n,
                                                   const GmresCtl* __restrict__ C, double* __restrict__ part,
                                                   const int* skip) {
  if (skipped(skip)) return;
  __shared__ double sh[4];
  __shared__ double cs[kMaxBasis], cg[kMaxBasis + 1];
  for (int j = threadIdx.x; j <= k; j += blockDim.x) {
    if (j < k) cs[j] = C->cs_[j];
    cg[j] = C->cg_[j];
  }
  __syncthreads();
  const double ia = C->inv_alpha, ib = C->inv_b;
  double acc = 0.0;
  if (k == 0)
    acc = dc_update_rows<TV, 0>(V, stride, k, w, n, cs, cg, ia, ib);
  else if (k <= kDotTile)
    with_count<kDotTile>(k, [&](auto KC) {
      acc = dc_update_rows<TV, decltype(KC)::value>(V, stride, k, w, n, cs, cg, ia, ib);
    });
  else
    acc = dc_update_rows<TV, -1>(V, stride, k, w, n, cs, cg, ia, ib);
  const double t = block_reduce_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
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
  C->kprov = -1;
  C->noprov = 1;
  C->bprov = 1.0;
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
