// Internal synchronisation (reflux / EMF fix / restriction) tables.
#pragma once
#include <vector>

#include "../../include/amr.h"
#include "amr_internal.hpp"

namespace amr {

struct SyncTables {
  void release() {}
};

// Build the tables of fine level `fl`; returns workspace bytes used for its
// registers (placed at byte offset `reg_off`).
inline int64_t build_sync_tables(int ndim, int R, const std::vector<GridDesc>& desc, const std::vector<amr_grid>& grids,
                                 const std::vector<std::vector<int>>& level_grids, const amr_params& p, int fl,
                                 SyncTables& out, int64_t reg_off, size_t esize) {
  (void)ndim; (void)R; (void)desc; (void)grids; (void)level_grids; (void)p; (void)fl; (void)out; (void)reg_off;
  (void)esize;
  return 0;
}

}  // namespace amr
