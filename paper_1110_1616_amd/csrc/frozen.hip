// Packing of (base, perturbed) state pairs for the frozen-branch advance.
#include "amr_internal.hpp"
#include "frozen.hpp"
#include "frozen_internal.hpp"

namespace amr {

namespace {

template <class S>
__global__ __launch_bounds__(256) void k_pack(DevState<S> B, DevState<S> P, DevState<Frozen<S>> out, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int q = 0; q < 8; ++q) out.f[q][t] = Frozen<S>(B.f[q][t], P.f[q][t], 0);
}

template <class S>
__global__ __launch_bounds__(256) void k_unpack(DevState<Frozen<S>> in, DevState<S> P, int64_t e0, int64_t e1) {
  for (int64_t t = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < e1; t += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int q = 0; q < 8; ++q) P.f[q][t] = in.f[q][t].p;
}

inline int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

template <class S>
void launch_pack(DevState<S> B, DevState<S> P, DevState<Frozen<S>> out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_pack<S>), dim3(blocks_for(n)), dim3(256), 0, s, B, P, out, n);
}

template <class S>
void launch_unpack(DevState<Frozen<S>> in, DevState<S> P, int64_t e0, int64_t e1, hipStream_t s) {
  if (e1 > e0) hipLaunchKernelGGL((k_unpack<S>), dim3(blocks_for(e1 - e0)), dim3(256), 0, s, in, P, e0, e1);
}

template void launch_pack<double>(DevState<double>, DevState<double>, DevState<FrozenD>, int64_t, hipStream_t);
template void launch_pack<float>(DevState<float>, DevState<float>, DevState<FrozenF>, int64_t, hipStream_t);
template void launch_unpack<double>(DevState<FrozenD>, DevState<double>, int64_t, int64_t, hipStream_t);
template void launch_unpack<float>(DevState<FrozenF>, DevState<float>, int64_t, int64_t, hipStream_t);

}  // namespace amr
