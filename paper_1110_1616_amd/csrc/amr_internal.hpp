// Internal types shared by the HIP kernels and the host runtime of
// libamrmhd.so.  Not part of the public ABI (include/amr.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amr {

// Device descriptor of one grid (patch).  The padded box holds every field:
// P[d] = n[d] + 2g + 1 on active axes, 1 on inactive ones; element (i,j,k)
// with i in [-g, n+g] sits at off + ((k+gz) P[1] + (j+g)) P[0] + (i+g).
struct GridDesc {
  int32_t n[3];
  int32_t lo[3];
  int32_t g;
  int32_t level;
  int32_t P[3];
  int32_t pad;
  int64_t off;
};

// Flux-kernel work item: one column tile of one grid, owned planes
// [z0, z1), advanced from valid band gv.  The block's 256 threads form
// tw x (256 / tw) cells (x0-1+tx, y0-1+ty); the first column and row overlap
// the neighbouring tiles, so (x0, y0) is the first owned cell and the tile
// owns (tw-1) x (256/tw - 1) cells of each plane.
struct FluxItem {
  int32_t grid;
  int32_t gv;
  int32_t x0, y0;
  int32_t z0, z1;
  int32_t tw;
  int32_t pad;
};

// Update-kernel work item: a tw x (256 / tw) column tile of the update index
// box starting at (x0, y0), planes [z0, z1).
struct UpdItem {
  int32_t grid;
  int32_t gv;
  int32_t x0, y0;
  int32_t z0, z1;
  int32_t tw;
  int32_t pad;
};

constexpr int kMinTile = 4;   // tile widths the kernels accept
constexpr int kMaxTile = 64;

// Physics constants passed by value.
struct Phys {
  double gamma;
  double dx0[3];
  int32_t ndim;
  int32_t ratio;
};

template <class T> struct DevState {
  T* f[8];
};

// Face fluxes of one substep: F[d][q], rotated components
// (rho, m_n, m_t1, m_t2, E, B_t1, B_t2) of direction d, stored at the
// element of the face's high-side cell (face index f along d <-> cell f).
template <class T> struct DevFlux {
  T* f[3][7];
  // the same 21 arrays as one base and the byte stride from one to the next
  // (f[d][q] = base + (7 d + q) stride)
  char* base;
  uint64_t stride;
  // upwinded EMF only (else null): cell-centred reference EMF per component,
  // and the edge EMFs computed from it once per edge
  T* e[3];
  T* edge[3];
};

// Element load / store at a 32-bit byte offset b from a base pointer that is
// uniform over the work item: the scalar-base address form, one 32-bit lane
// register per access instead of a 64-bit address.
// The offset type: 32-bit for the arithmetic types (a hierarchy's set-up
// bounds each field array below 4 GiB; amr_selfcheck_addressing() checks the
// offsets on the host); the frozen-branch pair types specialise it to 64-bit.
template <class T> struct ByteOffset { using type = uint32_t; };

template <class T, class B> __device__ __forceinline__ T ldb(const T* p, B b) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + b);
}
// (the element `imm` bytes further on, folded into the instruction)
template <class T, class B> __device__ __forceinline__ T ldb(const T* p, B b, int imm) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + b + imm);
}
template <class T, class B> __device__ __forceinline__ void stb(T* p, B b, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + b) = v;
}

// Error flag block in device memory: word 0 = flags, word 1..2 = first bad
// element (int64), words 4.. = reduction scratch.
struct ErrBlock {
  uint32_t flags;
  uint32_t pad;
  int64_t first_bad;
};


// Counters of the persistent launches' shared work queue (device memory,
// zero between launches: each persistent launch resets them as it ends).
struct WorkQueue {
  unsigned head[8];  // one counter per XCD chunk (only [0] without chunks)
  unsigned done;
  unsigned pad[7];
};

// Host-side launchers (defined in the .hip translation units).
// Level l of a grid reads its state from S1 if bit l of `parity` is set,
// else from S0; the update writes the other one.
// pblocks > 0 (with a queue): a persistent launch of pblocks blocks that pop
// the items; else one block per claim.  xcd: items in 8 contiguous chunks,
// one per XCD.  claim: items a block takes at a time (1, 2, 4 or 8).
template <class T>
void launch_flux(int ndim, const GridDesc* grids, const FluxItem* items, int nitems, DevState<T> S0, DevState<T> S1,
                 uint32_t parity, DevFlux<T> F, const double* dt0, Phys ph, ErrBlock* err, WorkQueue* q, int pblocks,
                 bool xcd, int claim, bool upwind_emf, hipStream_t s);
template <class T>
void launch_update(int ndim, const GridDesc* grids, const UpdItem* items, int nitems, DevState<T> S0, DevState<T> S1,
                   uint32_t parity, DevFlux<T> F, const double* dt0, Phys ph, WorkQueue* q, int pblocks,
                   bool xcd, int claim, bool upwind_emf, hipStream_t s);
// Upwinded edge EMFs of every edge the update reads (items: the update tiles
// of the same grids, one column and row wider).
template <class T>
void launch_emf(int ndim, const GridDesc* grids, const UpdItem* items, int nitems, DevFlux<T> F, hipStream_t s);
template <class T> void kernel_occupancy(int ndim, int* flux_blocks_per_cu, int* update_blocks_per_cu);
// Fused flux + update launch over fused work items (tiles overlapping by two
// columns and rows; see fused.hip).  fmask (may be null): per element, bit d
// set where the face flux normal to d must also be stored in F (the
// coarse/fine registers read it).
template <class T>
void launch_fused(int ndim, const GridDesc* grids, const FluxItem* items, int nitems, DevState<T> S0, DevState<T> S1,
                  uint32_t parity, DevFlux<T> F, const uint8_t* fmask, const double* dt0, Phys ph, ErrBlock* err,
                  WorkQueue* q, int pblocks, bool xcd, int claim, hipStream_t s);
template <class T> int fused_occupancy(int ndim);

}  // namespace amr
