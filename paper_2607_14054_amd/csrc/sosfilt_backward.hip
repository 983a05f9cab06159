// C ABI of the cascade's adjoint (include/sosfilt.h): the sub-plan the
// adjoint runs on, the workspace layout and the three launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "dispatch.hpp"
#include "kernels_backward.hpp"
#include "plan.hpp"
#include "batch.hpp"

using namespace sosf;

namespace sosf {

// The adjoint kernels run PH with FP64 arithmetic at N = kBwdN on their own
// tables (same cascade), and read per section the unfactored rows, the
// forward pass's cumulative b0 scale and the caller's a0.  The coefficient
// gradients are sums over the whole signal, so with FP32 I/O their run-ins
// keep the tighter bound 2^-50 (2^-64 with FP64 I/O, as elsewhere).
sos_status attach_adjoint(sos_plan_s &p, const double *sos) {
  sos_opts o{p.io_dtype, SOS_F64, SOS_PH, kBwdN, kL, 0, 0};
  sos_plan_t sub = nullptr;
  sos_status st = create_plan(sos, p.K, &o, false, &sub, p.io_dtype == SOS_F64 ? 0x1p-64 : 0x1p-50);
  if (st != SOS_OK) return st;
  p.bwd = sub;
  std::vector<double> rows((size_t)p.K * kBwdRow, 0.0);
  double scale = 1.0;
  for (int k = 0; k < p.K; ++k) {
    const double *r = &sub->rows_norm[5 * k];
    double *o8 = &rows[(size_t)kBwdRow * k];
    for (int j = 0; j < 5; ++j) o8[j] = r[j];
    if (sub->b0_factored) scale *= r[0];
    o8[BW_SCALE] = sub->b0_factored ? scale : 1.0;
    o8[BW_A0] = sub->a0[k];
  }
  if (hipMalloc(&p.d_bwd_rows, rows.size() * sizeof(double)) != hipSuccess) {
    p.d_bwd_rows = nullptr;
    return SOS_E_NOMEM;
  }
  if (hipMemcpy(p.d_bwd_rows, rows.data(), rows.size() * sizeof(double), hipMemcpyHostToDevice) !=
      hipSuccess)
    return SOS_E_DEVICE;
  return SOS_OK;
}

// The recompute mode's LDS stash (one FP64 group per row, adj_slots): with
// FP32 I/O (whose stage leaves room for it) and K >= 4, where it fits two
// workgroups per CU.
bool adjoint_stash(bool rc, int io_dtype, int kmax) {
  return rc && io_dtype == SOS_F32 && kmax >= 4 && AdjLds<kBwdN, float, true>::bytes(kmax, true) <= 80 * 1024;
}

// Recompute (group checkpoints) or saved outputs, by measured costs of one
// sos_filt_backward call per sample (MI355X, 2^24 samples, ps, fitted over
// K = 1 .. 48 with relative weights; within 11% (FP32 I/O) and 18% (FP64
// I/O) of every measured point):
//   saved outputs (about 16K bytes per sample): 4.23 + 3.38 K (FP32 I/O),
//     7.92 + 3.36 K (FP64 I/O);
//   recompute, P the forward section passes per group (adj_passes):
//     2.34 + 1.75 K + 0.331 P (FP32 I/O), 5.38 + 1.57 K + 0.381 P (FP64
//     I/O), times 1.34 (FP32) or 1.28 (FP64) where the adjoint pass's LDS
//     leaves one wavefront per SIMD instead of two (K > 43 with FP32 I/O,
//     K > 31 with FP64 I/O).
// Recompute is the cheaper up to K = 40 (FP32 I/O) and K = 31 (FP64 I/O).
double adjoint_cost_saved(int K, int io_dtype) {
  return io_dtype == SOS_F64 ? 7.92 + 3.36 * K : 4.23 + 3.38 * K;
}
double adjoint_cost_recompute(int K, int io_dtype, bool stash) {
  const bool lds = stash && K >= 4;
  const double P = adj_passes(K, lds);
  const bool f64 = io_dtype == SOS_F64;
  const size_t bytes = f64 ? AdjLds<kBwdN, double, true>::bytes(K, lds) : AdjLds<kBwdN, float, true>::bytes(K, lds);
  const double c = f64 ? 5.38 + 1.57 * K + 0.381 * P : 2.34 + 1.75 * K + 0.331 * P;
  return bytes <= 80 * 1024 ? c : c * (f64 ? 1.28 : 1.34);
}

bool adjoint_recompute(const sos_plan_s &p) {
  if (p.flags & SOS_FLAG_ADJ_RECOMPUTE) return true;
  if (p.flags & SOS_FLAG_ADJ_SAVE) return false;
  return adjoint_cost_recompute(p.K, p.io_dtype, adjoint_stash(true, p.io_dtype, p.K)) <
         adjoint_cost_saved(p.K, p.io_dtype);
}

}  // namespace sosf

namespace {

// The steps of a backward call: the forward-time pass that fills the
// workspace (and, for a training step's forward, stores y), and the
// reversed-time adjoint with the reduction of the coefficient sums.
enum : int { STEP_FORWARD = 1, STEP_ADJOINT = 2 };

template <typename TI, bool B0ONE, bool RC>
void launch_single(int steps, const BwdArgs &f, const BwdArgs &a, int K, const void *x, void *y, const void *gy,
                   void *gx, double *saved, const double *tab, const double *rows, double *partials, hipStream_t s) {
  constexpr int N = kBwdN;
  const int64_t per_block = (int64_t)kWavesPerBlock * kRows;
  if (steps & STEP_FORWARD) {
    const unsigned lds_f = (unsigned)lds_bytes<N, double, double>(K);
    const unsigned blocks_f = (unsigned)((f.ntiles + per_block - 1) / per_block);
    if (y)
      hipLaunchKernelGGL((sos_rows_save_kernel<N, TI, B0ONE, RC, true>), dim3(blocks_f), dim3(kWavesPerBlock * 64),
                         lds_f, s, static_cast<const TI *>(x), saved, static_cast<TI *>(y), tab, rows, f);
    else
      hipLaunchKernelGGL((sos_rows_save_kernel<N, TI, B0ONE, RC, false>), dim3(blocks_f), dim3(kWavesPerBlock * 64),
                         lds_f, s, static_cast<const TI *>(x), saved, static_cast<TI *>(nullptr), tab, rows, f);
  }
  if (steps & STEP_ADJOINT) {
    const unsigned lds_a = (unsigned)AdjLds<N, TI, RC>::bytes(K, a.stash > 0);
    const unsigned blocks_a = (unsigned)((a.ntiles + per_block - 1) / per_block);
    hipLaunchKernelGGL((sos_rows_adjoint_kernel<N, TI, B0ONE, RC>), dim3(blocks_a), dim3(kWavesPerBlock * 64),
                       lds_a, s, static_cast<const TI *>(gy), static_cast<TI *>(gx), static_cast<const TI *>(x),
                       saved, tab, rows, partials, a);
  }
}

// The adjoint kernel's own residency (it keeps fewer wavefronts per SIMD
// than the forward kernel of the sub-plan), for its launch shape.
Residency adjoint_residency(int io_dtype, bool rc, int K, bool stash) {
  const void *k;
  size_t lds;
  if (io_dtype == SOS_F32) {
    k = rc ? reinterpret_cast<const void *>(&sos_rows_adjoint_kernel<kBwdN, float, true, true>)
           : reinterpret_cast<const void *>(&sos_rows_adjoint_kernel<kBwdN, float, true, false>);
    lds = rc ? AdjLds<kBwdN, float, true>::bytes(K, stash) : AdjLds<kBwdN, float, false>::bytes(K, false);
  } else {
    k = rc ? reinterpret_cast<const void *>(&sos_rows_adjoint_kernel<kBwdN, double, true, true>)
           : reinterpret_cast<const void *>(&sos_rows_adjoint_kernel<kBwdN, double, true, false>);
    lds = rc ? AdjLds<kBwdN, double, true>::bytes(K, stash) : AdjLds<kBwdN, double, false>::bytes(K, false);
  }
  return residency_of(k, lds, kWavesPerBlock * 64);
}

struct BwdLayout {
  bool rc;                  // recompute mode
  int64_t stash;            // recompute mode: 1 with the LDS stash, else 0
  int64_t mid_off;          // recompute mode: doubles from the checkpoints to the kept inputs u_H
  int64_t np, tile, ntiles, sstride;
  int64_t shift, nck;       // forward tiles over [-shift, n); checkpoints (recompute mode)
  int64_t ftile, fntiles;   // the forward pass's tiles
  size_t saved_bytes, partial_bytes;
};

BwdLayout layout(const sos_plan_s &p, int64_t n) {
  const size_t esz = p.io_dtype == SOS_F64 ? 8 : 4;
  const int64_t V = 16 / (int64_t)esz, G = (int64_t)kBwdN * kL;
  BwdLayout l;
  l.rc = adjoint_recompute(p);
  l.stash = adjoint_stash(l.rc, p.io_dtype, p.K) ? 1 : 0;
  l.np = (n + V - 1) / V * V;
  if (p.bwd->tile_groups > 0) {
    l.tile = sos_plan_tile(p.bwd, std::max<int64_t>(l.np, 1));
  } else {
    const Residency r = adjoint_residency(p.io_dtype, l.rc, p.K, l.stash > 0);
    l.tile = model_tile_groups((std::max<int64_t>(l.np, 1) + G - 1) / G, p.bwd->warm / G, r) * G;
  }
  l.ntiles = (l.np + l.tile - 1) / l.tile;
  l.sstride = (n + 63) / 64 * 64;
  if (l.rc) {
    // forward groups start where the reversed-time groups of [0, np) do
    l.shift = (G - l.np % G) % G;
    l.nck = (l.np + l.shift) / G;
    // the checkpoints, then (K >= 8) each group's u_H
    l.mid_off = (l.nck * state_elems(p.K) + 31) / 32 * 32;
    l.saved_bytes = (size_t)(l.mid_off + (adj_mid(p.K) > 0 ? l.nck * G : 0)) * sizeof(double);
  } else {
    l.shift = 0;
    l.nck = 0;
    l.mid_off = 0;
    l.saved_bytes = (size_t)p.K * (size_t)l.sstride * sizeof(double);
  }
  l.ftile = sos_plan_tile(p.bwd, std::max<int64_t>(n + l.shift, 1));
  l.fntiles = (n + l.shift + l.ftile - 1) / l.ftile;
  l.partial_bytes = (size_t)std::max<int64_t>(l.ntiles, 1) * 5 * p.K * sizeof(double);
  return l;
}

template <typename TI>
sos_status launch_adjoint(int steps, const sos_plan_s &p, const void *x, void *y, const void *gy, void *gx,
                          double *gsos, int64_t n, void *ws, hipStream_t s) {
  const sos_plan_s &b = *p.bwd;
  const BwdLayout l = layout(p, n);
  double *saved = static_cast<double *>(ws);
  double *partials = reinterpret_cast<double *>(static_cast<unsigned char *>(ws) +
                                                (l.saved_bytes + 255) / 256 * 256);
  BwdArgs a;
  a.n = n;
  a.np = l.np;
  a.K = p.K;
  a.stride = b.stride;
  a.warm = b.warm;
  a.sstride = l.sstride;
  a.shift = l.shift;
  a.nck = l.nck;
  a.stash = l.stash;
  a.mid_off = l.mid_off;
  const double *tab = static_cast<const double *>(b.d_table);
  const double *rows = static_cast<const double *>(p.d_bwd_rows);
  if (n > 0) {
    // forward-time tiles (saving outputs or checkpoints), then the
    // reversed-time adjoint
    BwdArgs f = a;
    f.tile = l.ftile;
    f.ntiles = l.fntiles;
    a.tile = l.tile;
    a.ntiles = l.ntiles;
    if (l.rc) {
      if (b.b0_factored)
        launch_single<TI, true, true>(steps, f, a, p.K, x, y, gy, gx, saved, tab, rows, partials, s);
      else
        launch_single<TI, false, true>(steps, f, a, p.K, x, y, gy, gx, saved, tab, rows, partials, s);
    } else {
      if (b.b0_factored)
        launch_single<TI, true, false>(steps, f, a, p.K, x, y, gy, gx, saved, tab, rows, partials, s);
      else
        launch_single<TI, false, false>(steps, f, a, p.K, x, y, gy, gx, saved, tab, rows, partials, s);
    }
    if (hipGetLastError() != hipSuccess) return SOS_E_DEVICE;
  }
  if (steps & STEP_ADJOINT)
    hipLaunchKernelGGL(sos_adjoint_reduce_kernel, dim3((unsigned)p.K), dim3(kReduceThreads), 0, s, partials,
                       n > 0 ? l.ntiles : (int64_t)0, (int32_t)p.K, rows, gsos);
  return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
}

template <typename TI>
const void *adjoint_batched_kernel_ptr(bool rc) {
  // both b0 variants use the same resources
  return rc ? reinterpret_cast<const void *>(&sos_rows_adjoint_batched_kernel<kBwdN, TI, true, true>)
            : reinterpret_cast<const void *>(&sos_rows_adjoint_batched_kernel<kBwdN, TI, true, false>);
}

size_t adj_lds_save(int kmax) { return (size_t)lds_bytes<kBwdN, double, double>(kmax); }
size_t adj_lds_adjoint(int io_dtype, int kmax, bool rc, bool stash) {
  if (io_dtype == SOS_F32)
    return rc ? AdjLds<kBwdN, float, true>::bytes(kmax, stash) : AdjLds<kBwdN, float, false>::bytes(kmax, false);
  return rc ? AdjLds<kBwdN, double, true>::bytes(kmax, stash) : AdjLds<kBwdN, double, false>::bytes(kmax, false);
}

template <typename TI, bool B0ONE, bool RC>
void launch_batched(int steps, const sos_batch_s &b, const void *x, void *y, const void *gy, void *gx, double *w,
                    hipStream_t s) {
  constexpr int N = kBwdN;
  const unsigned blocks = (unsigned)((b.adj_items + kWavesPerBlock - 1) / kWavesPerBlock);
  if (steps & STEP_FORWARD) {
    const unsigned lds_f = (unsigned)adj_lds_save(b.kmax);
    if (y)
      hipLaunchKernelGGL((sos_rows_save_batched_kernel<N, TI, B0ONE, RC, true>), dim3(blocks),
                         dim3(kWavesPerBlock * 64), lds_f, s, static_cast<const TI *>(x), w, static_cast<TI *>(y),
                         b.d_adj, b.d_adj_item, b.adj_items, (int32_t)b.kmax, b.d_hdr, b.gen);
    else
      hipLaunchKernelGGL((sos_rows_save_batched_kernel<N, TI, B0ONE, RC, false>), dim3(blocks),
                         dim3(kWavesPerBlock * 64), lds_f, s, static_cast<const TI *>(x), w,
                         static_cast<TI *>(nullptr), b.d_adj, b.d_adj_item, b.adj_items, (int32_t)b.kmax,
                         b.d_hdr, b.gen);
  }
  if (steps & STEP_ADJOINT) {
    const unsigned lds_a = (unsigned)adj_lds_adjoint(b.io_dtype, b.kmax, RC, b.adj_stash);
    hipLaunchKernelGGL((sos_rows_adjoint_batched_kernel<N, TI, B0ONE, RC>), dim3(blocks),
                       dim3(kWavesPerBlock * 64), lds_a, s, static_cast<const TI *>(gy), static_cast<TI *>(gx),
                       static_cast<const TI *>(x), w, b.d_adj, b.d_adj_item, b.adj_items, (int32_t)b.kmax,
                       b.d_hdr, b.gen);
  }
}

template <typename TI>
sos_status launch_adjoint_batched(int steps, const sos_batch_s &b, const void *x, void *y, const void *gy, void *gx,
                                  double *gsos, void *ws, hipStream_t s) {
  double *w = static_cast<double *>(ws);
  if (b.adj_items > 0) {
    if (b.adj_rc) {
      if (b.adj_b0one)
        launch_batched<TI, true, true>(steps, b, x, y, gy, gx, w, s);
      else
        launch_batched<TI, false, true>(steps, b, x, y, gy, gx, w, s);
    } else {
      if (b.adj_b0one)
        launch_batched<TI, true, false>(steps, b, x, y, gy, gx, w, s);
      else
        launch_batched<TI, false, false>(steps, b, x, y, gy, gx, w, s);
    }
    if (hipGetLastError() != hipSuccess) return SOS_E_DEVICE;
  }
  if (steps & STEP_ADJOINT)
    hipLaunchKernelGGL(sos_adjoint_reduce_batched_kernel, dim3((unsigned)b.adj_rows), dim3(256), 0, s, w, b.d_adj,
                       b.d_adj_red, gsos, b.d_hdr, b.gen);
  return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
}

}  // namespace

namespace sosf {

// The batched adjoint's schedule (host side): per channel its adjoint
// sub-plan, tiles in groups of the sub-plan (reversed time, n rounded up to
// the vector width), and its regions of the workspace (saved outputs or
// group checkpoints, per-tile sums) and of gsos.  Channels go in the forward batch's launch
// order.
sos_status schedule_batch_adjoint(sos_batch_s &b, const sos_plan_t *plans, int32_t tile_groups) {
  b.adj = false;
  for (int c = 0; c < b.C; ++c)
    if (!plans[c]->bwd || !plans[c]->d_bwd_rows) return SOS_OK;   // no adjoint for this batch
  const int64_t G = (int64_t)kBwdN * kL;
  const int64_t V = b.io_dtype == SOS_F64 ? 2 : 4;
  // Channel c starts shift = off mod V samples past a 16-byte boundary.  The
  // forward-time tiles cover [-shift, n); reversed time reads
  // r[t] = s[np - 1 - t] with off + np a multiple of V.  Both put every
  // group of x, gy, gx and of the saved arrays (origin shifted by shift) on
  // a 16-byte boundary.  span: the samples the tiles must cover.
  // In recompute mode the shift is -np mod G instead, which is also off
  // mod V, so that the forward groups start where the reversed-time ones do
  // (the checkpoints).  One mode per batch: saved outputs if a plan asks for
  // them, else recompute if a plan asks for it, else the cheaper over the
  // batch's samples.
  bool any_save = false, any_rc = false;
  double cost_rc = 0.0, cost_saved = 0.0;
  for (int c = 0; c < b.C; ++c) {
    any_save = any_save || (plans[c]->flags & SOS_FLAG_ADJ_SAVE);
    any_rc = any_rc || (plans[c]->flags & SOS_FLAG_ADJ_RECOMPUTE);
    cost_rc += (double)b.n[c] * adjoint_cost_recompute(plans[c]->K, b.io_dtype, adjoint_stash(true, b.io_dtype, b.kmax));
    cost_saved += (double)b.n[c] * adjoint_cost_saved(plans[c]->K, b.io_dtype);
  }
  b.adj_rc = !any_save && (any_rc || cost_rc < cost_saved);
  b.adj_stash = adjoint_stash(b.adj_rc, b.io_dtype, b.kmax);
  std::vector<int64_t> np(b.C), shift(b.C), span(b.C);
  int64_t total_groups = 0;
  b.adj_b0one = true;
  for (int c = 0; c < b.C; ++c) {
    const int64_t n = b.n[c];
    np[c] = n ? (b.off[c] + n + V - 1) / V * V - b.off[c] : 0;
    shift[c] = b.adj_rc ? (G - np[c] % G) % G : b.off[c] % V;
    span[c] = n ? std::max(n + shift[c], np[c]) : 0;
    total_groups += (span[c] + G - 1) / G;
    b.adj_b0one = b.adj_b0one && plans[c]->bwd->b0_factored;
  }
  const Residency r = residency_of(b.io_dtype == SOS_F64 ? adjoint_batched_kernel_ptr<double>(b.adj_rc)
                                                         : adjoint_batched_kernel_ptr<float>(b.adj_rc),
                                   adj_lds_adjoint(b.io_dtype, b.kmax, b.adj_rc, b.adj_stash), kWavesPerBlock * 64);
  const int64_t resident_rows = (int64_t)4 * r.simds * r.waves_per_simd;
  b.adj_gsos_row.assign(b.C, 0);
  int64_t rows = 0;
  for (int c = 0; c < b.C; ++c) {
    b.adj_gsos_row[c] = rows;
    rows += plans[c]->K;
  }
  b.adj_rows = rows;
  std::vector<AdjChan> chans(b.C);
  std::vector<int32_t> item_chan, red(rows, 0);
  int64_t ws = 0, items = 0;
  for (int i = 0; i < b.C; ++i) {
    const int32_t c = b.order[i];
    const sos_plan_s *sub = plans[c]->bwd;
    AdjChan &a = chans[i];
    const int64_t groups = (span[c] + G - 1) / G;
    // Tiles as long as 16 run-ins where the batch fills the GPU with them;
    // otherwise as short as fills it, down to 2 run-ins.  The adjoint pass
    // waits on memory and on its reductions more than the forward does, so
    // a second wavefront per SIMD pays for more run-in than it does there
    // (4 run-ins).
    int64_t tg = tile_groups > 0 ? tile_groups : std::max<int64_t>(16 * (sub->warm / G), 8);
    if (tile_groups <= 0) {
      const int64_t tg_par = std::max<int64_t>(total_groups / std::max<int64_t>(resident_rows, 1), 1);
      if (tg_par < tg) tg = std::max<int64_t>(tg_par, std::max<int64_t>(2 * (sub->warm / G), 2));
    }
    const int64_t quads = groups ? (groups + 4 * tg - 1) / (4 * tg) : 0;
    const int64_t tgc = quads ? (groups + 4 * quads - 1) / (4 * quads) : 1;
    a.tab = static_cast<const double *>(sub->d_table);
    a.bwd = static_cast<const double *>(plans[c]->d_bwd_rows);
    a.off = b.off[c];
    a.n = b.n[c];
    a.np = np[c];
    a.tile = tgc * G;
    a.warm = sub->warm;
    a.ntiles = groups ? (span[c] + a.tile - 1) / a.tile : 0;
    a.first_item = items;
    a.sstride = (b.n[c] + shift[c] + 63) / 64 * 64;
    a.nck = b.adj_rc && b.n[c] ? (np[c] + shift[c]) / G : 0;
    a.stash = b.adj_stash && plans[c]->K >= 4 ? 1 : 0;
    a.saved_off = ws;
    // recompute mode: the checkpoints, then (K >= 8) each group's u_H
    a.mid_off = b.adj_rc ? (a.nck * state_elems(plans[c]->K) + 31) / 32 * 32 : 0;
    ws += b.adj_rc ? a.mid_off + (adj_mid(plans[c]->K) > 0 ? a.nck * G : 0) : (int64_t)plans[c]->K * a.sstride;
    a.partial_off = ws;
    ws += (a.ntiles * 5 * plans[c]->K + 31) / 32 * 32;
    a.K = plans[c]->K;
    a.stride = sub->stride;
    a.shift = (int32_t)shift[c];
    a.gsos_row = (int32_t)b.adj_gsos_row[c];
    for (int64_t q = 0; q < quads; ++q) item_chan.push_back(i);
    items += quads;
    for (int k = 0; k < plans[c]->K; ++k) red[b.adj_gsos_row[c] + k] = i;
  }
  b.adj_items = items;
  b.adj_ws = (size_t)std::max<int64_t>(ws, 32) * sizeof(double);
  b.adj_chans = std::move(chans);
  b.adj_item_chan = std::move(item_chan);
  b.adj_red = std::move(red);
  b.adj = true;
  return SOS_OK;
}

}  // namespace sosf

namespace {

bool disjoint(uintptr_t a, uintptr_t b, uintptr_t bytes) { return !(a < b + bytes && b < a + bytes); }

// Arguments of a backward call with `bytes` of signal: the forward step
// reads x and writes y (if any); the adjoint step reads x and gy and writes
// gx.  Signals and workspace 16-byte aligned; what a step writes overlaps
// nothing it reads (tiles read beyond their own range); gsos 8-byte aligned.
sos_status check_backward(int steps, uintptr_t bytes, const void *x, const void *y, const void *gy,
                          const void *gx, const double *gsos, const void *workspace) {
  if (!workspace) return SOS_E_ARG;
  if ((steps & STEP_ADJOINT) && (!gsos || ((uintptr_t)gsos & 7))) return SOS_E_ARG;
  if (bytes == 0) return SOS_OK;
  const uintptr_t xb = (uintptr_t)x, yb = (uintptr_t)y, gyb = (uintptr_t)gy, gxb = (uintptr_t)gx;
  if (!x || ((xb | (uintptr_t)workspace) & 15)) return SOS_E_ARG;
  if (steps & STEP_FORWARD) {
    if (y && ((yb & 15) || !disjoint(xb, yb, bytes))) return SOS_E_ARG;
  }
  if (steps & STEP_ADJOINT) {
    if (!gy || !gx || ((gyb | gxb) & 15)) return SOS_E_ARG;
    if (!disjoint(gxb, xb, bytes) || !disjoint(gxb, gyb, bytes)) return SOS_E_ARG;
  }
  return SOS_OK;
}

sos_status backward_single(int steps, sos_plan_t p, const void *x, void *y, const void *gy, void *gx, double *gsos,
                           int64_t n, void *workspace, sos_stream_t stream) {
  if (!p || n < 0) return SOS_E_ARG;
  if (!p->bwd || !p->d_bwd_rows) return SOS_E_ARG;   // host-only plan
  if ((steps & STEP_FORWARD) && !(steps & STEP_ADJOINT) && n > 0 && !y) return SOS_E_ARG;
  const size_t esz = p->io_dtype == SOS_F64 ? 8 : 4;
  const sos_status st = check_backward(steps, (uintptr_t)n * esz, x, y, gy, gx, gsos, workspace);
  if (st != SOS_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (p->io_dtype == SOS_F32) return launch_adjoint<float>(steps, *p, x, y, gy, gx, gsos, n, workspace, s);
  return launch_adjoint<double>(steps, *p, x, y, gy, gx, gsos, n, workspace, s);
}

sos_status backward_batched(int steps, sos_batch_t b, const void *x, void *y, const void *gy, void *gx, double *gsos,
                            void *workspace, sos_stream_t stream) {
  if (!b || !b->adj) return SOS_E_ARG;
  if (!batch_descriptors_valid(*b)) return SOS_E_ARG;
  if ((steps & STEP_FORWARD) && !(steps & STEP_ADJOINT) && b->adj_items > 0 && !y) return SOS_E_ARG;
  const size_t esz = b->io_dtype == SOS_F64 ? 8 : 4;
  const sos_status st =
      check_backward(steps, b->adj_items > 0 ? (uintptr_t)b->total * esz : 0, x, y, gy, gx, gsos, workspace);
  if (st != SOS_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (b->io_dtype == SOS_F32) return launch_adjoint_batched<float>(steps, *b, x, y, gy, gx, gsos, workspace, s);
  return launch_adjoint_batched<double>(steps, *b, x, y, gy, gx, gsos, workspace, s);
}

}  // namespace

extern "C" {

size_t sos_batch_backward_workspace_size(sos_batch_t b) { return (b && b->adj) ? b->adj_ws : 0; }

sos_status sos_batch_query_adjoint(sos_batch_t b, int64_t *gsos_rows, int64_t *first_row) {
  if (!b || !b->adj) return SOS_E_ARG;
  if (gsos_rows) *gsos_rows = b->adj_rows;
  if (first_row)
    for (int c = 0; c < b->C; ++c) first_row[c] = b->adj_gsos_row[c];
  return SOS_OK;
}

sos_status sos_filt_backward_batched(sos_batch_t b, const void *x, const void *gy, void *gx, double *gsos,
                                     void *workspace, sos_stream_t stream) {
  return backward_batched(STEP_FORWARD | STEP_ADJOINT, b, x, nullptr, gy, gx, gsos, workspace, stream);
}

sos_status sos_filt_batched_for_backward(sos_batch_t b, const void *x, void *y, void *workspace,
                                         sos_stream_t stream) {
  return backward_batched(STEP_FORWARD, b, x, y, nullptr, nullptr, nullptr, workspace, stream);
}

sos_status sos_filt_backward_batched_stored(sos_batch_t b, const void *x, const void *gy, void *gx, double *gsos,
                                            void *workspace, sos_stream_t stream) {
  return backward_batched(STEP_ADJOINT, b, x, nullptr, gy, gx, gsos, workspace, stream);
}

size_t sos_backward_workspace_size(sos_plan_t p, int64_t n) {
  if (!p || n < 0 || !p->bwd) return 0;
  const BwdLayout l = layout(*p, n);
  return (l.saved_bytes + 255) / 256 * 256 + l.partial_bytes;
}

sos_status sos_filt_backward(sos_plan_t p, const void *x, const void *gy, void *gx, double *gsos,
                             int64_t n, void *workspace, sos_stream_t stream) {
  return backward_single(STEP_FORWARD | STEP_ADJOINT, p, x, nullptr, gy, gx, gsos, n, workspace, stream);
}

sos_status sos_filt_for_backward(sos_plan_t p, const void *x, void *y, int64_t n, void *workspace,
                                 sos_stream_t stream) {
  return backward_single(STEP_FORWARD, p, x, y, nullptr, nullptr, nullptr, n, workspace, stream);
}

sos_status sos_filt_backward_stored(sos_plan_t p, const void *x, const void *gy, void *gx, double *gsos, int64_t n,
                                    void *workspace, sos_stream_t stream) {
  return backward_single(STEP_ADJOINT, p, x, nullptr, gy, gx, gsos, n, workspace, stream);
}

}  // extern "C"
