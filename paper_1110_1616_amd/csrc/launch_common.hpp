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

// Work items are handed to blocks in claims of `claim` consecutive list
// entries (claim in {1, 2, 4, 8}): a block runs its claim's items back to
// back and only then takes another.  Grids of one tile per plane and one
// z-chunk are one item each, so for them the claim is the number of grids a
// workgroup takes at a time; for larger grids it is a run of neighbouring
// tiles of one grid.  A block's current claim is [next, end).
struct ItemRange {
  int next, end;
};

// Claim of a one-block-per-range launch (non-persistent): block b takes
// entries [b claim, (b + 1) claim); with `xcd` the list is cut into 8
// contiguous chunks of C entries, one per XCD (workgroups are dispatched to
// the 8 XCDs round-robin, so block b runs on XCD b mod 8), and block b takes
// the (b / 8)-th claim of chunk b mod 8, so neighbouring tiles, which share
// halo data, run under one L2.  Persistent launches start with an empty
// claim.
template <bool PERSIST>
__device__ __forceinline__ ItemRange first_claim(int nitems, int claim, bool xcd) {
  if (PERSIST) return ItemRange{0, 0};
  const int b = (int)blockIdx.x;
  if (xcd) {
    const int C = (nitems + 7) >> 3;
    const int c = b & 7, lo = c * C + (b >> 3) * claim;
    return ItemRange{lo, min(min(lo + claim, c * C + C), nitems)};
  }
  const int lo = b * claim;
  return ItemRange{lo, min(lo + claim, nitems)};
}

// Next work item of this block, or -1 when there is none.  Non-persistent
// blocks run their one claim.  Persistent launches (a fixed number of
// blocks) pop claims from the shared queue, one atomic per claim, in list
// order (finest level first), so blocks that draw cheap items come back for
// more; with `xcd` a persistent block pops its own chunk first, then the
// others.  Taking an item from the current claim involves no barrier (the
// kernels end each item with one before LDS is reused); popping a claim
// does, so every thread of the block must call this with the same range.
template <bool PERSIST>
__device__ __forceinline__ int next_item(ItemRange& r, int nitems, int claim, WorkQueue* q, int* s_claim, int* s_c,
                                         bool xcd) {
  if (r.next < r.end) return r.next++;
  if (!PERSIST) return -1;
  if (threadIdx.x == 0) {
    int lo = -1, hi = -1;
    if (!xcd) {
      const int i = (int)atomicAdd(&q->head[0], (unsigned)claim);
      if (i < nitems) {
        lo = i;
        hi = min(i + claim, nitems);
      }
    } else {
      const int C = (nitems + 7) >> 3;
      while (lo < 0 && *s_c < 8) {
        const int c = (int)((blockIdx.x + *s_c) & 7);
        const int base = c * C, len = min(C, nitems - base);
        if (len > 0) {
          const int i = (int)atomicAdd(&q->head[c], (unsigned)claim);
          if (i < len) {
            lo = base + i;
            hi = base + min(i + claim, len);
          }
        }
        if (lo < 0) ++*s_c;  // this chunk is drained: move to the next
      }
    }
    s_claim[0] = lo;
    s_claim[1] = hi;
  }
  __syncthreads();
  const int lo = s_claim[0], hi = s_claim[1];
  __syncthreads();
  if (lo < 0) return -1;
  r.next = lo + 1;
  r.end = hi;
  return lo;
}

// Blocks of a non-persistent launch of nitems entries in claims of `claim`.
inline int claim_blocks(int nitems, int claim, bool xcd) {
  if (xcd) {
    const int C = (nitems + 7) / 8;
    return 8 * ((C + claim - 1) / claim);
  }
  return (nitems + claim - 1) / claim;
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
