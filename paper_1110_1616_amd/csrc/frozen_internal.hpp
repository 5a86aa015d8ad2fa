// Launchers of the frozen-branch advance (libamrmhd.so internal).
#pragma once
#include "amr_internal.hpp"
#include "frozen.hpp"

namespace amr {

// out <- (B, P) element pairs over the first n elements of every pool.
template <class S>
void launch_pack(DevState<S> B, DevState<S> P, DevState<Frozen<S>> out, int64_t n, hipStream_t s);
// P[e0, e1) <- the perturbed members of `in`.
template <class S>
void launch_unpack(DevState<Frozen<S>> in, DevState<S> P, int64_t e0, int64_t e1, hipStream_t s);

}  // namespace amr
