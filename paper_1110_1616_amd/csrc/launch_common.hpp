// Launch helpers shared by the batched advance kernels (flux, update and the
// fused flux-update kernel): the flux tile's LDS ring layout and the work
// queue of persistent launches.
#pragma once
#include "amr_internal.hpp"

namespace amr {

// A flux tile is tw x th threads (tw in [kMinTile, kMaxTile], th = 256 / tw)
// over cells (x0-1+tx, y0-1+ty); the LDS plane adds one ring cell on each
// side: (tw+2) x (th+2) entries, at most kMaxPlane.
constexpr int kMaxPlane = 396;  // max over tw in [4, 64] of (tw + 2)(256 / tw + 2)

// Ring entry r in [0, 2 (tw + th)) of the plane -> (ex, ey): the one-cell
// border of the tile's (tw + 2) x (th + 2) LDS plane without its four
// corners, which no cell reads (the slopes use the x and y neighbours only).
// A 16 x 16 tile's 64 ring cells are then one wave's lanes.
__device__ __forceinline__ void ring_entry(int r, int tw, int th, int& ex, int& ey) {
  if (r < tw) { ex = r + 1; ey = 0; }
  else if (r < 2 * tw) { ex = r - tw + 1; ey = th + 1; }
  else if (r < 2 * tw + th) { ex = 0; ey = r - 2 * tw + 1; }
  else { ex = tw + 1; ey = r - 2 * tw - th + 1; }
}

// Next work item of this block.  Grid-stride launches take blockIdx.x,
// blockIdx.x + gridDim.x, ...; persistent launches (a fixed number of blocks)
// pop the shared queue, one atomic per item, in list order (finest level
// first), so blocks that draw cheap items come back for more.  With `xcd`
// the list is cut into 8 contiguous chunks, one per XCD (workgroups are
// dispatched to the 8 XCDs round-robin, so block b runs on XCD b mod 8):
// neighbouring tiles, which share halo data, then run under one L2.  A
// one-block-per-item launch maps block b to item (b mod 8) C + b / 8; a
// persistent block pops its own chunk first, then the others.  Returns -1
// when the list is exhausted.
template <bool PERSIST>
__device__ __forceinline__ int next_item(int& cursor, int nitems, WorkQueue* q, int* s_it, int* s_c, bool xcd) {
  const int C = (nitems + 7) >> 3;
  if (!PERSIST) {
    if (xcd) {
      if (cursor < 0) return -1;
      const int b = cursor;
      cursor = -1;
      const int it = (b & 7) * C + (b >> 3);
      return it < nitems ? it : -1;
    }
    const int it = cursor;
    cursor += gridDim.x;
    return it < nitems ? it : -1;
  }
  if (threadIdx.x == 0) {
    int res = -1;
    if (!xcd) {
      const unsigned i = atomicAdd(&q->head[0], 1u);
      if ((int)i < nitems) res = (int)i;
    } else {
      while (res < 0 && *s_c < 8) {
        const int c = (int)((blockIdx.x + *s_c) & 7);
        const int lo = c * C, len = min(C, nitems - lo);
        if (len > 0) {
          const unsigned i = atomicAdd(&q->head[c], 1u);
          if ((int)i < len) res = lo + (int)i;
        }
        if (res < 0) ++*s_c;  // this chunk is drained: move to the next
      }
    }
    *s_it = res;
  }
  __syncthreads();
  const int it = *s_it;
  __syncthreads();
  return it;
}

// Persistent launches leave the queue ready for the next one: the last block
// to finish resets the counters (every other block has made its final pop
// before it counts itself done).
template <bool PERSIST>
__device__ __forceinline__ void retire(WorkQueue* q) {
  if (!PERSIST) return;
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned d = atomicAdd(&q->done, 1u);
    if (d == gridDim.x - 1) {
      for (int c = 0; c < 8; ++c) atomicExch(&q->head[c], 0u);
      atomicExch(&q->done, 0u);
    }
  }
}

}  // namespace amr
