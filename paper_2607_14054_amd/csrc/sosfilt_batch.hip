// C ABI of the batched ragged-channel filter (include/sosfilt.h): the
// schedule of (channel, tile) work items, built once on the host, and the
// launch of the batched tile kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "dispatch.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "batch.hpp"
#include "kernels_block.hpp"

using namespace sosf;

namespace {

// One channel's share of the schedule, in groups: its span, its run-in
// and its sections.
struct ChanWork {
  int64_t groups, warm_groups;
  int32_t K;
};

// Groups per tile (the cap every channel's tile stays under), from a
// makespan model.  Each candidate cap gives every channel's work items
// (items of 64 / L equal row tiles, or four for block filtering, each
// preceded by its run-in, clamped at
// the channel start) and their cost in group-sections, K (tile + run-in).
// In SIMD time, with a = total / simds and b = (longest item) *
// waves_per_simd, the launch takes between max(a, b) and a + b (the
// list-scheduling bound for one-wavefront items, waves_per_simd of them
// sharing a SIMD); the model takes the midpoint.  Long tiles waste little on
// run-ins; short tiles give more items and a shorter tail.  A channel with
// a long run-in (poles near the unit circle) needs the short tiles for
// parallelism even at the cost of run-in many times its tile.  Ties go to
// the longer tile.
int64_t batch_tile_groups(const std::vector<ChanWork> &w, int64_t simds, int64_t waves_per_simd,
                          int64_t waves_per_item, int64_t tiles_per_item) {
  const int64_t R = tiles_per_item;
  int64_t best_tg = 8;
  double best = -1.0;
  for (int e = 12; e >= 0; --e) {
    const int64_t tg = int64_t(1) << e;
    double total = 0.0, longest = 0.0;
    for (const ChanWork &c : w) {
      if (c.groups == 0) continue;
      const int64_t quads = (c.groups + R * tg - 1) / (R * tg);
      const int64_t tgc = (c.groups + R * quads - 1) / (R * quads);
      const int64_t wc = std::min<int64_t>(c.warm_groups, (c.groups - 1) / tgc * tgc);
      const double item = (double)c.K * (double)(tgc + wc);
      total += (double)(quads * waves_per_item) * item;
      longest = std::max(longest, item);
    }
    const double a = total / (double)std::max<int64_t>(simds, 1), b = longest * (double)waves_per_simd;
    const double cost = 0.5 * (std::max(a, b) + a + b);
    if (best < 0.0 || cost < best * 0.999) {
      best = cost;
      best_tg = tg;
    }
  }
  return best_tg;
}

// The launch depends only on what the batch fixed at creation (grid, LDS,
// instance); the live item count is read from the device header.
template <int N, typename TI, typename T, bool B0ONE, int SOLVER, int L>
struct LaunchBatched {
  static sos_status run(const sos_batch_s &b, const void *x, void *y, hipStream_t s) {
    const int64_t blocks = (b.items_cap + kWavesPerBlock - 1) / kWavesPerBlock;
    const unsigned lds = (unsigned)lds_bytes<N, TI, T, L>(b.kmax_cap);
    hipLaunchKernelGGL((sos_rows_batched_kernel<N, TI, T, B0ONE, SOLVER, L>), dim3((unsigned)blocks),
                       dim3(kWavesPerBlock * 64), lds, s, static_cast<const TI *>(x),
                       static_cast<TI *>(y), b.d_chans, b.d_item_chan, b.d_hdr, (int32_t)b.kmax_cap);
    return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
  }
};

template <int N, typename TI, typename T, bool B0ONE, int SOLVER, int L>
struct ResidencyBatched {
  static sos_status run(int kmax, Residency *r) {
    *r = residency_of(reinterpret_cast<const void *>(&sos_rows_batched_kernel<N, TI, T, B0ONE, SOLVER, L>),
                      (size_t)lds_bytes<N, TI, T, L>(kmax), kWavesPerBlock * 64);
    return SOS_OK;
  }
};

void free_device(sos_batch_s *b) {
  if (!b->d_blob && !b->h_blob && !b->copied) return;
  int cur = -1;
  hipGetDevice(&cur);
  if (b->device >= 0 && cur != b->device) hipSetDevice(b->device);
  if (b->copied) hipEventSynchronize(b->copied);
  if (b->d_blob) hipFree(b->d_blob);
  if (b->h_blob) hipHostFree(b->h_blob);
  if (b->copied) hipEventDestroy(b->copied);
  if (b->device >= 0 && cur >= 0 && cur != b->device) hipSetDevice(cur);
  b->d_blob = b->h_blob = nullptr;
  b->copied = nullptr;
}

sos_status validate(const sos_plan_t *plans, int32_t C, const int64_t *n, bool host_only) {
  if (!plans || !n || C < 1) return SOS_E_ARG;
  for (int c = 0; c < C; ++c) {
    const sos_plan_s *p = plans[c];
    if (!p || n[c] < 0) return SOS_E_ARG;
    if (!host_only && !p->d_table) return SOS_E_ARG;   // a host-only plan cannot filter
    if (p->solver_opt == SOS_PH_DEFERRED || p->solver_opt == SOS_SCALAR) return SOS_E_UNSUPPORTED;
    if (p->N > 64 || p->N < 8) return SOS_E_UNSUPPORTED;   // wide and narrow groups run single signals only
    // block filtering batches only with block filtering (its own kernel)
    if ((p->solver_opt == SOS_BLOCK) != (plans[0]->solver_opt == SOS_BLOCK)) return SOS_E_UNSUPPORTED;
    if (!host_only && p->solver_opt == SOS_BLOCK && (!p->d_block || !p->d_aop)) return SOS_E_ARG;
    if (p->N != plans[0]->N || p->L != plans[0]->L || p->io_dtype != plans[0]->io_dtype ||
        p->compute_dtype != plans[0]->compute_dtype || p->block_slices != plans[0]->block_slices)
      return SOS_E_UNSUPPORTED;
  }
  return SOS_OK;
}

// The host schedule of a channel set: offsets, per-channel tiles and work
// items (costliest first), and for device batches the adjoint's schedule.
sos_status schedule(sos_batch_s &b, const sos_plan_t *plans, int32_t C, const int64_t *n,
                    const int64_t *offsets, int32_t tile_groups) {
  b.C = C;
  b.N = plans[0]->N;
  b.L = plans[0]->L;
  b.io_dtype = plans[0]->io_dtype;
  b.compute_dtype = plans[0]->compute_dtype;
  b.n.assign(n, n + C);
  b.off.assign(C, 0);
  b.total = 0;
  b.items = 0;
  b.kmax = 0;
  b.b0one = true;
  b.item_chan.clear();
  // offsets: given (channels must not overlap), or dense packing
  if (offsets) {
    std::vector<int32_t> by_off(C);
    std::iota(by_off.begin(), by_off.end(), 0);
    std::stable_sort(by_off.begin(), by_off.end(),
                     [&](int32_t a, int32_t c) { return offsets[a] < offsets[c]; });
    int64_t end = 0;
    for (int i = 0; i < C; ++i) {
      const int32_t c = by_off[i];
      if (offsets[c] < 0 || (n[c] > 0 && offsets[c] < end)) return SOS_E_ARG;
      if (n[c] > 0) end = offsets[c] + n[c];
    }
    for (int c = 0; c < C; ++c) b.off[c] = offsets[c];
  } else {
    int64_t acc = 0;
    for (int c = 0; c < C; ++c) {
      b.off[c] = acc;
      acc += n[c];
    }
  }
  const size_t esz = b.io_dtype == SOS_F64 ? 8 : 4;
  // block filtering: its own kernel, tiles in groups of 16 blocks
  b.block = plans[0]->solver_opt == SOS_BLOCK;
  b.block_pt = plans[0]->block_pt;
  b.block_slices = plans[0]->block_slices;
  const int64_t G = b.block ? (int64_t)kBlockGroup : (int64_t)b.N * b.L;
  // tiles per work item: the rows of one wavefront, or (block filtering)
  // the four wavefronts of a workgroup
  const int64_t R = b.block ? 4 : 64 / b.L;
  for (int c = 0; c < C; ++c) b.total = std::max(b.total, b.off[c] + n[c]);
  // each channel's solver class: SOS_CR or SOS_PH when all its sections use
  // that solver, SOS_AUTO otherwise; the batch takes a specialised kernel
  // when every channel has the same class, else the kernel that branches
  // once per wavefront on the channel's class
  std::vector<int32_t> cls(C);
  for (int c = 0; c < C; ++c) {
    const sos_plan_s *p = plans[c];
    b.kmax = std::max(b.kmax, p->K);
    b.b0one = b.b0one && p->b0_factored;
    cls[c] = p->solver[0];
    for (int k = 1; k < p->K; ++k)
      if (p->solver[k] != cls[c]) cls[c] = SOS_AUTO;
  }
  b.mix = cls[0];
  for (int c = 1; c < C; ++c)
    if (cls[c] != b.mix) b.mix = SOS_AUTO;
  Residency res;
  if (!b.host_only && b.block)
    res = block_batched_residency(b.io_dtype, b.block_pt, b.block_slices, b.kmax);
  else if (!b.host_only)
    dispatch_rows_l<ResidencyBatched>(b.N, b.L, b.io_dtype, b.compute_dtype, b.b0one, b.mix, b.kmax, &res);
  // a channel whose first sample is off a 16-byte boundary is filtered over
  // [-shift, n): the shift samples before it read as zeros (zero state stays
  // zero) and are not stored, and every group then starts on a boundary.
  // Block filtering moves 4 samples per lane (16 or 32 bytes).
  const int64_t V = b.block ? 4 : 16 / (int64_t)esz;
  std::vector<int32_t> shift(C, 0);
  std::vector<ChanWork> work(C);
  for (int c = 0; c < C; ++c) {
    shift[c] = (int32_t)(b.off[c] % V);
    work[c] = ChanWork{n[c] == 0 ? 0 : (n[c] + shift[c] + G - 1) / G, plans[c]->warm / G, plans[c]->K};
  }
  // an item is four row tiles in one wavefront, or (block filtering) four
  // tiles in the four wavefronts of a workgroup
  const int64_t tg = tile_groups > 0 ? tile_groups
                                     : batch_tile_groups(work, res.simds, res.waves_per_simd, b.block ? 4 : 1, R);
  // per-channel tiles: items of R row tiles under the cap, as even as
  // the length allows
  b.tile.assign(C, 0);
  std::vector<int64_t> quads(C, 0);
  std::vector<double> cost(C, 0.0);
  for (int c = 0; c < C; ++c) {
    const sos_plan_s *p = plans[c];
    const int64_t groups = work[c].groups;
    if (groups == 0) {
      b.tile[c] = G;
      continue;
    }
    quads[c] = (groups + R * tg - 1) / (R * tg);
    const int64_t tgc = (groups + R * quads[c] - 1) / (R * quads[c]);
    b.tile[c] = tgc * G;
    const int64_t warm = std::min<int64_t>(p->warm, (groups - 1) / tgc * tgc * G);
    cost[c] = (double)p->K * (double)(warm + b.tile[c]);
  }
  // launch order: costliest items first (the dispatcher then fills the
  // tail of the launch with the cheap ones)
  b.order.resize(C);
  std::iota(b.order.begin(), b.order.end(), 0);
  std::stable_sort(b.order.begin(), b.order.end(), [&](int32_t a, int32_t c) { return cost[a] > cost[c]; });
  b.chans.assign(C, BatchChan{});
  for (int i = 0; i < C; ++i) {
    const int32_t c = b.order[i];
    const sos_plan_s *p = plans[c];
    BatchChan &ch = b.chans[i];
    ch.tab = b.block ? p->d_block : p->d_table;
    ch.aop = b.block ? p->d_aop : nullptr;
    ch.solver = static_cast<const int32_t *>(p->d_solver);
    ch.off = b.off[c];
    ch.n = n[c];
    ch.tile = b.tile[c];
    ch.warm = p->warm;
    ch.first_item = b.items;
    ch.K = p->K;
    ch.stride = p->stride;
    ch.gain = p->gain;
    ch.shift = shift[c];
    ch.mix = cls[c];
    for (int64_t q = 0; q < quads[c]; ++q) b.item_chan.push_back(i);
    b.items += quads[c];
  }
  b.adj = false;
  if (!b.host_only) return schedule_batch_adjoint(b, plans, tile_groups);
  return SOS_OK;
}

// The device descriptors of a schedule, packed into one blob: the header
// (live item count, generation), forward channels, forward items, adjoint
// channels, adjoint items, gsos rows.  The regions are sized by the batch's
// room, fixed at creation.
struct BlobLayout {
  size_t hdr, chans, items, adj, adj_items, red, bytes;
};

size_t up16(size_t v) { return (v + 15) & ~(size_t)15; }

BlobLayout blob_layout(size_t C, size_t items, size_t adj_items, size_t rows) {
  BlobLayout l;
  l.hdr = 0;
  l.chans = 16;
  l.items = up16(l.chans + C * sizeof(BatchChan));
  l.adj = up16(l.items + items * sizeof(int32_t));
  l.adj_items = up16(l.adj + C * sizeof(AdjChan));
  l.red = up16(l.adj_items + adj_items * sizeof(int32_t));
  l.bytes = up16(l.red + rows * sizeof(int32_t));
  return l;
}

// The layout of the batch's room.
BlobLayout blob_layout(const sos_batch_s &b) {
  return blob_layout((size_t)b.C_cap, (size_t)b.items_cap, (size_t)b.adj_items_cap, (size_t)b.rows_cap);
}

void pack(const sos_batch_s &b, const BlobLayout &l, unsigned char *dst) {
  const int64_t hdr[2] = {b.items, b.gen};
  std::memcpy(dst + l.hdr, hdr, sizeof(hdr));
  std::memcpy(dst + l.chans, b.chans.data(), b.chans.size() * sizeof(BatchChan));
  std::memcpy(dst + l.items, b.item_chan.data(), b.item_chan.size() * sizeof(int32_t));
  if (b.adj) {
    std::memcpy(dst + l.adj, b.adj_chans.data(), b.adj_chans.size() * sizeof(AdjChan));
    std::memcpy(dst + l.adj_items, b.adj_item_chan.data(), b.adj_item_chan.size() * sizeof(int32_t));
    std::memcpy(dst + l.red, b.adj_red.data(), b.adj_red.size() * sizeof(int32_t));
  }
}

void point(sos_batch_s &b, const BlobLayout &l) {
  if (!b.d_blob) {
    b.d_hdr = nullptr;
    b.d_chans = nullptr;
    b.d_item_chan = nullptr;
    b.d_adj = nullptr;
    b.d_adj_item = nullptr;
    b.d_adj_red = nullptr;
    return;
  }
  b.d_hdr = reinterpret_cast<const int64_t *>(b.d_blob + l.hdr);
  b.d_chans = reinterpret_cast<BatchChan *>(b.d_blob + l.chans);
  b.d_item_chan = reinterpret_cast<int32_t *>(b.d_blob + l.items);
  b.d_adj = reinterpret_cast<AdjChan *>(b.d_blob + l.adj);
  b.d_adj_item = reinterpret_cast<int32_t *>(b.d_blob + l.adj_items);
  b.d_adj_red = reinterpret_cast<int32_t *>(b.d_blob + l.red);
}

// Room for channel sets of up to C channels and `samples` samples in all:
// tiles of at least one group give at most samples / (4 G) + 2 C work items
// (a channel's span has at most n / G + 2 groups, in items of R tiles),
// and likewise for the adjoint's items.
void reserve_room(sos_batch_s &b, int64_t C, int64_t samples, int kmax) {
  const int64_t G = b.block ? (int64_t)kBlockGroup : (int64_t)b.N * b.L;
  const int64_t R = b.block ? 4 : 64 / b.L;
  const int64_t Gb = (int64_t)kBwdN * kL;
  b.C_cap = (int32_t)std::max<int64_t>(C, b.C);
  b.items_cap = std::max<int64_t>(samples / (R * G) + 2 * C + 1, b.items);
  b.adj_items_cap = std::max<int64_t>((samples + 3 * C) / (4 * Gb) + 2 * C + 1, b.adj ? (int64_t)b.adj_item_chan.size() : 0);
  b.kmax_cap = std::max(kmax, b.kmax);
  b.rows_cap = std::max<int64_t>(C * (int64_t)b.kmax_cap, b.adj ? (int64_t)b.adj_red.size() : 0);
}

// The schedule t fits the room of batch b, and b's forward kernel instance
// serves every channel of t.
sos_status fits(const sos_batch_s &b, const sos_batch_s &t) {
  // an instance with b0 factored out cannot run a channel that keeps b0;
  // one specialised on a solver class runs only that class
  if (b.inst_b0one && !t.b0one) return SOS_E_UNSUPPORTED;
  if (b.inst_mix != SOS_AUTO && t.mix != b.inst_mix) return SOS_E_UNSUPPORTED;
  if (t.C > b.C_cap || t.items > b.items_cap || t.kmax > b.kmax_cap) return SOS_E_NOMEM;
  if (t.adj != b.adj) return SOS_E_UNSUPPORTED;
  if (t.adj && ((int64_t)t.adj_item_chan.size() > b.adj_items_cap || (int64_t)t.adj_red.size() > b.rows_cap))
    return SOS_E_NOMEM;
  return SOS_OK;
}

}  // namespace

// The descriptor pointers of a device batch lie inside its buffer (a launch
// with any other value would read outside it).
bool batch_descriptors_valid(const sos_batch_s &b) {
  if (!b.d_blob) return false;
  auto inside = [&](const void *p) {
    const unsigned char *q = static_cast<const unsigned char *>(p);
    return q >= b.d_blob && q < b.d_blob + b.blob_cap;
  };
  return inside(b.d_hdr) && inside(b.d_chans) && inside(b.d_item_chan) && inside(b.d_adj) && inside(b.d_adj_item) &&
         inside(b.d_adj_red);
}

extern "C" {

sos_status sos_batch_plan(const sos_plan_t *plans, int32_t C, const int64_t *n,
                          const int64_t *offsets, const sos_batch_opts *opts, sos_batch_t *out) {
  if (!out) return SOS_E_ARG;
  sos_batch_opts o{0, 0, 0, 0, 0};
  if (opts) o = *opts;
  if (o.tile_groups < 0 || o.max_channels < 0 || o.max_samples < 0) return SOS_E_ARG;
  const bool host_only = (o.flags & SOS_FLAG_HOST_ONLY) != 0;
  sos_status st = validate(plans, C, n, host_only);
  if (st != SOS_OK) return st;
  sos_batch_s *b = new (std::nothrow) sos_batch_s;
  if (!b) return SOS_E_NOMEM;
  b->host_only = host_only;
  b->tile_groups = o.tile_groups;
  st = schedule(*b, plans, C, n, offsets, o.tile_groups);
  if (st != SOS_OK) {
    delete b;
    return st;
  }
  // the room and the forward launch, fixed from here on
  const bool reserve = o.max_channels > 0 || o.max_samples > 0 || o.max_sections > 0;
  if (o.max_sections < 0 || o.max_sections > SOS_MAX_SECTIONS) {
    delete b;
    return SOS_E_ARG;
  }
  if (reserve) {
    reserve_room(*b, std::max<int64_t>(o.max_channels, C), std::max<int64_t>(o.max_samples, b->total),
                 o.max_sections);
    // the kernel instance that serves every channel a replan may bring
    b->inst_b0one = false;
    b->inst_mix = SOS_AUTO;
  } else {
    b->C_cap = C;
    b->items_cap = b->items;
    b->adj_items_cap = b->adj ? (int64_t)b->adj_item_chan.size() : 0;
    b->kmax_cap = b->kmax;
    b->rows_cap = b->adj ? (int64_t)b->adj_red.size() : 0;
    b->inst_b0one = b->b0one;
    b->inst_mix = b->mix;
  }
  if (!host_only) {
    const BlobLayout l = blob_layout(*b);
    b->blob_cap = l.bytes;
    if (hipGetDevice(&b->device) != hipSuccess) {
      delete b;
      return SOS_E_DEVICE;
    }
    if (hipMalloc(&b->d_blob, b->blob_cap) != hipSuccess) {
      b->d_blob = nullptr;
      delete b;
      return SOS_E_NOMEM;
    }
    if (hipHostMalloc(&b->h_blob, b->blob_cap, hipHostMallocDefault) != hipSuccess) {
      b->h_blob = nullptr;
      free_device(b);
      delete b;
      return SOS_E_NOMEM;
    }
    if (hipEventCreateWithFlags(&b->copied, hipEventDisableTiming) != hipSuccess) {
      b->copied = nullptr;
      free_device(b);
      delete b;
      return SOS_E_DEVICE;
    }
    pack(*b, l, b->h_blob);
    if (hipMemcpy(b->d_blob, b->h_blob, l.bytes, hipMemcpyHostToDevice) != hipSuccess) {
      free_device(b);
      delete b;
      return SOS_E_DEVICE;
    }
    point(*b, l);
  }
  *out = b;
  return SOS_OK;
}

sos_status sos_batch_replan(sos_batch_t b, const sos_plan_t *plans, int32_t C, const int64_t *n,
                            const int64_t *offsets, sos_stream_t stream) {
  if (!b) return SOS_E_ARG;
  sos_status st = validate(plans, C, n, b->host_only);
  if (st != SOS_OK) return st;
  if (plans[0]->N != b->N || plans[0]->L != b->L || plans[0]->io_dtype != b->io_dtype ||
      plans[0]->compute_dtype != b->compute_dtype ||
      (plans[0]->solver_opt == SOS_BLOCK) != b->block || plans[0]->block_slices != b->block_slices)
    return SOS_E_UNSUPPORTED;
  // schedule into a copy, so that an invalid request leaves the batch as it was
  sos_batch_s t;
  t.host_only = b->host_only;
  t.tile_groups = b->tile_groups;
  st = schedule(t, plans, C, n, offsets, b->tile_groups);
  if (st != SOS_OK) return st;
  // a device batch keeps its room and its launch; a host-only batch is only
  // a schedule, and takes the new set's
  if (!b->host_only) {
    st = fits(*b, t);
    if (st != SOS_OK) return st;
  }
  // t keeps the device resources of b, its room and its launch (the
  // descriptor pointers of t are then derived from b's buffer below; a
  // host-only batch has none)
  t.device = b->device;
  t.d_blob = b->d_blob;
  t.h_blob = b->h_blob;
  t.blob_cap = b->blob_cap;
  t.copied = b->copied;
  if (b->host_only) {
    t.C_cap = t.C;
    t.kmax_cap = t.kmax;
    t.items_cap = t.items;
    t.adj_items_cap = 0;
    t.rows_cap = 0;
    t.inst_b0one = t.b0one;
    t.inst_mix = t.mix;
  } else {
    t.C_cap = b->C_cap;
    t.kmax_cap = b->kmax_cap;
    t.items_cap = b->items_cap;
    t.adj_items_cap = b->adj_items_cap;
    t.rows_cap = b->rows_cap;
    t.inst_b0one = b->inst_b0one;
    t.inst_mix = b->inst_mix;
  }
  t.gen = b->gen + 1;
  if (!b->host_only) {
    const BlobLayout l = blob_layout(t);
    if (l.bytes > b->blob_cap) return SOS_E_NOMEM;
    // the staging copy is free once the previous upload has been read
    if (hipEventSynchronize(b->copied) != hipSuccess) return SOS_E_DEVICE;
    pack(t, l, b->h_blob);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(b->d_blob, b->h_blob, l.bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(b->copied, s) != hipSuccess)
      return SOS_E_DEVICE;
    point(t, l);
  }
  *b = std::move(t);
  return SOS_OK;
}

sos_status sos_batch_destroy(sos_batch_t b) {
  if (!b) return SOS_OK;
  free_device(b);
  delete b;
  return SOS_OK;
}

sos_status sos_batch_query(sos_batch_t b, int64_t *total, int64_t *items, int64_t *offsets,
                           int64_t *tile, int32_t *order) {
  if (!b) return SOS_E_ARG;
  if (total) *total = b->total;
  if (items) *items = b->items;
  for (int c = 0; c < b->C; ++c) {
    if (offsets) offsets[c] = b->off[c];
    if (tile) tile[c] = b->tile[c];
    if (order) order[c] = b->order[c];
  }
  return SOS_OK;
}

sos_status sos_filt_batched(sos_batch_t b, const void *x, void *y, void *workspace,
                            sos_stream_t stream) {
  (void)workspace;
  if (!b) return SOS_E_ARG;
  if (b->host_only || !batch_descriptors_valid(*b)) return SOS_E_ARG;
  if (b->items_cap == 0) return SOS_OK;
  if (!x || !y) return SOS_E_ARG;
  const size_t esz = b->io_dtype == SOS_F64 ? 8 : 4;
  const uintptr_t xb = (uintptr_t)x, yb = (uintptr_t)y, bytes = (uintptr_t)b->total * esz;
  if (xb < yb + bytes && yb < xb + bytes) return SOS_E_ARG;   // overlap
  if ((xb | yb) & 15) return SOS_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (b->block) return launch_block_batched(*b, x, y, s);
  return dispatch_rows_l<LaunchBatched>(b->N, b->L, b->io_dtype, b->compute_dtype, b->inst_b0one, b->inst_mix, *b,
                                        x, y, s);
}

sos_status sos_batch_tune(const double *const *sos, const int32_t *K, int32_t C, const int64_t *n,
                          const int64_t *offsets, const sos_opts *base, const int32_t *Ns, int32_t nN,
                          const int32_t *Ls, int32_t nL, const int32_t *tiles, int32_t nt, const void *x, void *y,
                          int32_t reps, sos_stream_t stream, sos_tune_result *results, sos_tune_result *best) {
  if (!sos || !K || !n || !Ns || !Ls || !tiles || nN < 1 || nL < 1 || nt < 1 || reps < 1 || !best || C < 1)
    return SOS_E_ARG;
  sos_opts o{SOS_F32, SOS_F64, SOS_AUTO, 0, 0, 0, 0};
  if (base) o = *base;
  if (o.flags & SOS_FLAG_HOST_ONLY) return SOS_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return SOS_E_DEVICE;
  }
  best->N = 0;
  best->L = 0;
  best->tile_groups = 0;
  best->seconds = 0.0;
  sos_status st = SOS_OK;
  for (int iNL = 0; iNL < nN * nL && st == SOS_OK; ++iNL) {
    const int iN = iNL / nL, iL = iNL % nL;
    sos_opts on = o;
    on.N = Ns[iN];
    on.L = Ls[iL];
    std::vector<sos_plan_t> plans(C, nullptr);
    for (int c = 0; c < C && st == SOS_OK; ++c) st = sos_plan(sos[c], K[c], &on, &plans[c]);
    for (int it = 0; it < nt && st == SOS_OK; ++it) {
      sos_batch_opts bo{tiles[it], 0};
      sos_batch_t b = nullptr;
      st = sos_batch_plan(plans.data(), C, n, offsets, &bo, &b);
      if (st != SOS_OK) break;
      float ms = 0.f;
      // warm-up: load the code and bring the clocks back up after the host
      // built this configuration's plans (launch until 30 ms have passed)
      const auto t0 = std::chrono::steady_clock::now();
      do {
        st = sos_filt_batched(b, x, y, nullptr, stream);
        if (st == SOS_OK && hipStreamSynchronize(s) != hipSuccess) st = SOS_E_DEVICE;
      } while (st == SOS_OK && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(30));
      if (st == SOS_OK && hipEventRecord(e0, s) != hipSuccess) st = SOS_E_DEVICE;
      for (int r = 0; r < reps && st == SOS_OK; ++r) st = sos_filt_batched(b, x, y, nullptr, stream);
      if (st == SOS_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = SOS_E_DEVICE;
      sos_batch_destroy(b);
      if (st != SOS_OK) break;
      const double sec = (double)ms * 1e-3 / reps;
      if (results) results[iNL * nt + it] = sos_tune_result{Ns[iN], Ls[iL], tiles[it], 0, sec};
      if (best->N == 0 || sec < best->seconds) *best = sos_tune_result{Ns[iN], Ls[iL], tiles[it], 0, sec};
    }
    for (int c = 0; c < C; ++c) sos_plan_destroy(plans[c]);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return st;
}

}  // extern "C"
