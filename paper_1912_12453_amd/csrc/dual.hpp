// Forward-mode dual numbers for device code: x = v + d eps with eps^2 = 0.
// Instantiating the templated residual code of the element loop with
// Dual<T> and seeding d with a direction gives the exact directional
// derivative of the residual, every cross term included, without deriving
// any of them by hand (used for the rows of the coupled Jacobian).
// Comparisons look at the value only, so branches (the pull-back of phi,
// the sign tests) follow the linearisation point.
#pragma once
#include <hip/hip_runtime.h>

namespace chns {
namespace dev {

template <class T>
struct Dual {
  T v, d;
  __host__ __device__ Dual() : v(0), d(0) {}
  __host__ __device__ Dual(T a) : v(a), d(0) {}
  __host__ __device__ Dual(T a, T b) : v(a), d(b) {}

  friend __device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
  friend __device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
  friend __device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
  friend __device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
  friend __device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const T q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
  }
  friend __device__ __forceinline__ Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
  friend __device__ __forceinline__ Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
  friend __device__ __forceinline__ Dual& operator*=(Dual& a, Dual b) { return a = a * b; }
  friend __device__ __forceinline__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
  friend __device__ __forceinline__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
  friend __device__ __forceinline__ bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
  friend __device__ __forceinline__ bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
  // sqrt(x)' = x' / (2 sqrt(x))
  friend __device__ __forceinline__ Dual sqrt(Dual a) {
    const T r = sqrt(a.v);
    return Dual(r, a.d / (T(2) * r));
  }
};

// lane exchanges move both parts
template <int CTRL, class T>
__device__ __forceinline__ Dual<T> xchg(Dual<T> x) {
  return Dual<T>(xchg<CTRL>(x.v), xchg<CTRL>(x.d));
}

}  // namespace dev
}  // namespace chns
