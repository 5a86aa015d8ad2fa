// Frozen-branch scalar: a pair (base, perturbed) carried through the same
// templated device code as float/double.  Arithmetic acts on both members;
// every comparison reads the base member only, so each branch of the scheme
// (minmod choice, wave-speed extremes and clamps, HLLD region and degeneracy
// tests) is decided by the unperturbed run while the perturbed member follows
// that fixed sequence of branches.  A finite difference of the perturbed
// member is then a difference of one smooth branch of the discrete map, the
// map whose exact derivative the adjoint computes.
#pragma once
#include "amr_internal.hpp"
#include "mhd_device.hpp"

namespace amr {

template <class S> struct Frozen {
  S b, p;
  Frozen() = default;
  __host__ __device__ Frozen(double x) : b(S(x)), p(S(x)) {}
  __host__ __device__ Frozen(S bb, S pp, int) : b(bb), p(pp) {}

  friend __host__ __device__ Frozen operator+(Frozen x, Frozen y) { return Frozen(x.b + y.b, x.p + y.p, 0); }
  friend __host__ __device__ Frozen operator-(Frozen x, Frozen y) { return Frozen(x.b - y.b, x.p - y.p, 0); }
  friend __host__ __device__ Frozen operator*(Frozen x, Frozen y) { return Frozen(x.b * y.b, x.p * y.p, 0); }
  friend __host__ __device__ Frozen operator/(Frozen x, Frozen y) { return Frozen(x.b / y.b, x.p / y.p, 0); }
  friend __host__ __device__ Frozen operator-(Frozen x) { return Frozen(-x.b, -x.p, 0); }
  friend __host__ __device__ bool operator<(Frozen x, Frozen y) { return x.b < y.b; }
  friend __host__ __device__ bool operator>(Frozen x, Frozen y) { return x.b > y.b; }
  friend __host__ __device__ bool operator<=(Frozen x, Frozen y) { return x.b <= y.b; }
  friend __host__ __device__ bool operator>=(Frozen x, Frozen y) { return x.b >= y.b; }
  __host__ __device__ Frozen& operator+=(Frozen y) { return *this = *this + y; }
  __host__ __device__ Frozen& operator-=(Frozen y) { return *this = *this - y; }
  __host__ __device__ Frozen& operator*=(Frozen y) { return *this = *this * y; }
};

template <> __host__ __device__ __forceinline__ Frozen<double> dsqrt<Frozen<double>>(Frozen<double> x) {
  return Frozen<double>(__builtin_sqrt(x.b), __builtin_sqrt(x.p), 0);
}
template <> __host__ __device__ __forceinline__ Frozen<float> dsqrt<Frozen<float>>(Frozen<float> x) {
  return Frozen<float>(__builtin_sqrtf(x.b), __builtin_sqrtf(x.p), 0);
}

// 64-bit byte offsets for the pair types in the flux kernel's addressing.
// The 32-bit offsets of the arithmetic types are exact for 16-byte elements
// too (amr_selfcheck_addressing walks every work list with that element
// size), yet the pair-type flux kernel compiled with them produced results
// that read unwritten workspace on the GPU; the cause lies outside the
// offset arithmetic and was not found, so the pair types keep 64-bit
// offsets (finite-difference verification only; they take no part in the
// timed path).
template <class S> struct ByteOffset<Frozen<S>> { using type = uint64_t; };

using FrozenD = Frozen<double>;
using FrozenF = Frozen<float>;

}  // namespace amr
