// Internal types and launchers of the discrete adjoint (libamrmhd.so).
#pragma once
#include "amr_internal.hpp"

namespace amr {

// One source element of the band copy and the band elements copied from it
// (dsts[begin, end)).  cls: 0 cells, 1 + d faces along d.
struct InvCopy {
  int32_t src;
  int32_t cls;
  int32_t begin;
  int32_t end;
};

// Adjoint scratch arrays, each `stride` elements, indexed by pool element
// minus e0 (the first element of the grids being differentiated).
struct AdjBuffers {
  void* ps;   // predicted face states: 3 x 2 x 7 arrays
  void* af;   // face adjoints: 3 x 15 arrays
  void* ac;   // cell predictor adjoints: 38 arrays
  void* au;   // cell primitive-recovery adjoints: 9 arrays
  void* tmp;  // assembled input adjoint: 8 arrays
  int64_t stride;
  int64_t e0;
};
constexpr int kAdjArrays = 42 + 45 + 38 + 9 + 8;

// Eight double pointers passed by value (interior-layout host-facing arrays).
struct Ptr8 {
  const double* p[8];
};
struct MutPtr8 {
  double* p[8];
};

// One reverse step: Lout (own elements of the listed grids) <- the adjoint of
// the step's input given Lp, the adjoint of its output.  U is the step's
// input state with its band filled.  items: (grid, first local element) of
// 256-element chunks of each grid's padded box.
template <class T>
void launch_adjoint_step(int ndim, const GridDesc* grids, const int2* items, int nitems, const InvCopy* inv, int ninv,
                         const int32_t* dsts, DevState<T> U, DevState<T> Lp, DevState<T> Lout, AdjBuffers buf,
                         double dt0, Phys ph, hipStream_t s);
// Adjoint of amr_store_interior: own elements of L <- g (interior layout).
template <class T>
void launch_store_adj(int ndim, const GridDesc& G, Ptr8 g, DevState<T> L, hipStream_t s);
// Adjoint of amr_load_primitive with respect to rho and v.
template <class T>
void launch_load_prim_adj(int ndim, const GridDesc& G, Ptr8 prim, DevState<T> L, MutPtr8 out, hipStream_t s);

// dst[0, n) <- host[0, n), passed by value in kernel arguments (no host
// memory is read after the call returns).
void launch_put_values(double* dst, const double* host, int n, hipStream_t s);

}  // namespace amr
