// Descriptors of the adjoint kernels (kernels_backward.hpp), shared with the
// batch structure.
#pragma once

#include <cstdint>

namespace sosf {

// One channel's adjoint geometry, as the row functions of the adjoint
// kernels see it.
struct AdjView {
  int64_t n, np, tile, warm, ntiles, sstride;
  int64_t shift;            // forward tiles cover [-shift, n); saved arrays start shift elements in
  int64_t nck;              // recompute mode: group checkpoints, one per group of [-shift, np)
  int64_t stash;            // recompute mode: S > 0 keeps u_S per group in LDS (0: none)
  int32_t K, stride;
};

// Batched channels: per channel its sub-plan's tables, its adjoint rows, its
// signal offset and the offsets of its saved outputs (or group checkpoints)
// and sums in the workspace.  Work items are four tiles of one channel, as
// in the forward batch.
struct AdjChan {
  const double *tab;        // the channel's adjoint sub-plan table
  const double *bwd;        // the channel's adjoint rows
  int64_t off, n, np, tile, warm, ntiles, first_item;
  int64_t saved_off;        // doubles into the workspace
  int64_t partial_off;      // doubles into the workspace (ntiles x 5K)
  int64_t sstride;
  int64_t nck;              // recompute mode: group checkpoints (see AdjView)
  int64_t stash;            // recompute mode: stashed section input (see AdjView)
  int32_t K, stride;
  int32_t shift;            // forward tiles cover [-shift, n) (see AdjView)
  int32_t gsos_row;         // first row of the channel in gsos
};

}  // namespace sosf
