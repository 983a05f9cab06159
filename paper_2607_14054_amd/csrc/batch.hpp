// Internal batch structure shared by the batched forward (sosfilt_batch.hip)
// and the batched adjoint (sosfilt_backward.hip).
#pragma once

#include <cstdint>
#include <vector>

#include "kernels.hpp"
#include "adjoint_types.hpp"
#include "plan.hpp"
#include "dispatch.hpp"

struct sos_batch_s {
  int C = 0, N = 0, L = 16, io_dtype = SOS_F32, compute_dtype = SOS_F64;
  int kmax = 0, mix = SOS_PH;
  int32_t tile_groups = 0;
  bool b0one = true, host_only = false;
  bool block = false;                     // block-filtering channels (SOS_BLOCK plans)
  int block_pt = 0;                       // their product type
  int block_slices = 1;                   // and slices per operand
  int device = -1;
  int64_t total = 0, items = 0;
  std::vector<int64_t> n, off, tile;
  std::vector<int32_t> order;             // channels in launch order
  std::vector<sosf::BatchChan> chans;     // in launch order
  std::vector<int32_t> item_chan;         // item -> index into chans
  sosf::BatchChan *d_chans = nullptr;
  int32_t *d_item_chan = nullptr;
  // adjoint schedule (device batches whose plans carry the adjoint)
  bool adj = false, adj_b0one = true, adj_rc = false;   // adj_rc: recompute mode
  bool adj_stash = false;                 // recompute mode: the stash fits (per channel with K >= 4)
  int64_t adj_items = 0, adj_rows = 0;    // wave items; rows of gsos (sum of K)
  size_t adj_ws = 0;                      // workspace bytes
  std::vector<int64_t> adj_gsos_row;      // per channel (caller order): first gsos row
  std::vector<sosf::AdjChan> adj_chans;   // in launch order
  std::vector<int32_t> adj_item_chan;     // item -> index into adj_chans
  std::vector<int32_t> adj_red;           // gsos row -> index into adj_chans
  sosf::AdjChan *d_adj = nullptr;
  int32_t *d_adj_item = nullptr;
  int32_t *d_adj_red = nullptr;
  // every device descriptor lives in one allocation (and its pinned host
  // staging copy, for sos_batch_replan), at offsets fixed when the batch is
  // created: a launch captured in a HIP graph stays valid after a replan.
  // The allocation starts with a header of two int64: the forward launch's
  // live item count and the schedule's generation.
  unsigned char *d_blob = nullptr, *h_blob = nullptr;
  size_t blob_cap = 0;
  hipEvent_t copied = nullptr;            // the last staging upload has been read
  // fixed at creation: the room of every descriptor region, the forward
  // launch's grid (items_cap items), its LDS (kmax_cap sections) and its
  // kernel instance (b0 factoring, solver class)
  int32_t C_cap = 0, kmax_cap = 0;
  int64_t items_cap = 0, adj_items_cap = 0, rows_cap = 0;
  bool inst_b0one = true;
  int inst_mix = SOS_PH;
  int64_t gen = 0;                        // schedule generation (header[1])
  const int64_t *d_hdr = nullptr;         // the device header
};

// the descriptor pointers lie inside the device buffer (sosfilt_batch.hip)
bool batch_descriptors_valid(const sos_batch_s &b);

namespace sosf {
// the adjoint schedule, host side (sosfilt_backward.hip)
sos_status schedule_batch_adjoint(sos_batch_s &b, const sos_plan_t *plans, int32_t tile_groups);
// batched block filtering (sosfilt_block.hip)
Residency block_batched_residency(int io_dtype, int pt, int S, int kmax);
sos_status launch_block_batched(const sos_batch_s &b, const void *x, void *y, hipStream_t s);
}
