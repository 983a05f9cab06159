// Descriptors of the adjoint kernels (kernels_backward.hpp), shared with the
// batch structure.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace sosf {

// Recompute mode: where a group's section inputs u_k come from.  For
// K >= 8 the forward pass keeps, besides the group's checkpoint, the input
// u_H of section H = K / 2 in the workspace (8 bytes per sample, which
// makes that pass HBM-bound; below K = 8 the passes it saves cost less than
// that), which splits the sections into two phases: k >= H recomputed from
// u_H, k < H from the group's input u_0.  Within a phase [b, t] the first input computed is u_t (from u_b),
// and on the way two of its inputs are kept for the later k of the phase:
// one in the row's LDS stash (where the plan has one) and one in
// registers.  adj_slots gives phase p's (0: below H, 1: from H) base b, top
// t and the two kept indices (0: none; a kept index lies strictly between
// b and t).  Host and kernel both take the schedule from here.
struct AdjSlots {
  int base, top, lds, regs;
};

__host__ __device__ inline int adj_mid(int K) { return K >= 8 ? K / 2 : 0; }

__host__ __device__ inline AdjSlots adj_slots(int K, bool lds_stash, int phase) {
  const int H = adj_mid(K);
  AdjSlots s;
  s.base = phase ? H : 0;
  s.top = (phase || H == 0) ? K - 1 : H - 1;
  const int len = s.top - s.base + 1;
  const int l = lds_stash ? s.base + len / 2 : 0;
  const int r = s.base + (lds_stash ? len / 4 : len / 2);
  s.lds = (l > s.base && l < s.top) ? l : 0;
  s.regs = (r > s.base && r < s.top && r != s.lds) ? r : 0;
  return s;
}

// Forward section passes per group of the recompute mode: u_{K-1} and
// w_{K-1} from the top phase's base, then for every other k the passes
// from the nearest kept input at or below it (u_H and u_0 cost none).
__host__ __device__ inline int adj_passes(int K, bool lds_stash) {
  const int H = adj_mid(K);
  int passes = 0;
  for (int k = K - 1; k >= 0; --k) {
    const AdjSlots s = adj_slots(K, lds_stash, H > 0 && k >= H ? 1 : 0);
    int from = s.base;
    if (k != s.top) {
      if (s.lds && s.lds <= k && s.lds > from) from = s.lds;
      if (s.regs && s.regs <= k && s.regs > from) from = s.regs;
    }
    passes += k - from;
  }
  return passes + 1;   // w_{K-1}
}

// One channel's adjoint geometry, as the row functions of the adjoint
// kernels see it.
struct AdjView {
  int64_t n, np, tile, warm, ntiles, sstride;
  int64_t shift;            // forward tiles cover [-shift, n); saved arrays start shift elements in
  int64_t nck;              // recompute mode: group checkpoints, one per group of [-shift, np)
  int64_t stash;            // recompute mode: > 0 when the row has an LDS stash (one FP64 group)
  int64_t mid_off;          // recompute mode: doubles from the checkpoints to the kept inputs u_H
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
  int64_t stash;            // recompute mode: LDS stash (see AdjView)
  int64_t mid_off;          // recompute mode: kept inputs u_H (see AdjView)
  int32_t K, stride;
  int32_t shift;            // forward tiles cover [-shift, n) (see AdjView)
  int32_t gsos_row;         // first row of the channel in gsos
};

}  // namespace sosf
