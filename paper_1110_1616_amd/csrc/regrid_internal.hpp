// Internal types of regridding and the (O)verlap transfer (libamrmhd.so).
#pragma once
#include <array>
#include <functional>
#include <vector>

#include "amr_internal.hpp"
#include "fill_internal.hpp"

namespace amr {

// Flag-kernel work item: interior cells [first, last) (x fastest) of one
// grid, written at out + first.
struct FlagItem {
  int32_t grid;
  int32_t first, last;
  int32_t pad;
  int64_t out;
};

// One uncovered coarse cell of a new grid whose interior fine faces are
// completed by projection: element of its lowest fine cell.
struct ProjEntry {
  int32_t grid;
  int32_t e0;
};

template <class T>
void launch_flag(int ndim, const GridDesc* grids, const FlagItem* items, int nitems, DevState<T> U, double theta,
                 uint8_t* out, hipStream_t s);
// Copy between two pools (previous iteration -> new iteration).
template <class T>
void launch_copy2(int ndim, const CopyEntry* ent, int n, int4 cls, DevState<T> Us, DevState<T> Ud, hipStream_t s);
template <class T>
void launch_project(int ndim, const ProjEntry* ent, int n, const GridDesc* grids, DevState<T> U, Phys ph,
                    hipStream_t s);

// Integer box [lo, hi) of one level.
struct IBox {
  int lo[3], hi[3];
};

// Berger-Rigoutsos clustering of a set of level cells (each pts entry a
// cell; duplicates are not allowed) inside [0, N): boxes covering every
// point, accepted when points >= eff * volume, every extent <= maxbox and
// admissible(box), or when a single cell.  Deterministic (cut preference
// and tie rules in the source).
std::vector<IBox> cluster_boxes(int ndim, const int (&N)[3], const std::vector<std::array<int, 3>>& pts, double eff,
                                int maxbox, const std::function<bool(const IBox&)>& admissible);

}  // namespace amr
