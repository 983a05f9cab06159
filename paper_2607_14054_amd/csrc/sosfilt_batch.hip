// C ABI of the batched ragged-channel filter (include/sosfilt.h): the
// schedule of (channel, tile) work items, built once on the host, and the
// launch of the batched tile kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "dispatch.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "batch.hpp"

using namespace sosf;

namespace {

// Groups per tile for a channel: as for one signal, long enough that the
// run-in costs little, short enough that the whole batch keeps every
// resident row of the device busy.
int64_t batch_tile_groups(int64_t warm_groups, int64_t total_groups, int64_t resident_rows,
                          int32_t cap) {
  if (cap > 0) return cap;
  int64_t tg = std::max<int64_t>(16 * warm_groups, 8);
  const int64_t tg_par = std::max<int64_t>(total_groups / std::max<int64_t>(resident_rows, 1), 1);
  if (tg_par < tg) tg = std::max<int64_t>(tg_par, std::max<int64_t>(4 * warm_groups, 4));
  return tg;
}

template <int N, typename TI, typename T, bool B0ONE, int SOLVER>
struct LaunchBatched {
  static sos_status run(const sos_batch_s &b, const void *x, void *y, hipStream_t s) {
    const int64_t blocks = (b.items + kWavesPerBlock - 1) / kWavesPerBlock;
    const unsigned lds = (unsigned)lds_bytes<N, TI, T>(b.kmax);
    hipLaunchKernelGGL((sos_rows_batched_kernel<N, TI, T, B0ONE, SOLVER>), dim3((unsigned)blocks),
                       dim3(kWavesPerBlock * 64), lds, s, static_cast<const TI *>(x),
                       static_cast<TI *>(y), b.d_chans, b.d_item_chan, b.items, (int32_t)b.kmax);
    return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
  }
};

template <int N, typename TI, typename T, bool B0ONE, int SOLVER>
struct ResidencyBatched {
  static sos_status run(int kmax, Residency *r) {
    *r = residency_of(reinterpret_cast<const void *>(&sos_rows_batched_kernel<N, TI, T, B0ONE, SOLVER>),
                      (size_t)lds_bytes<N, TI, T>(kmax), kWavesPerBlock * 64);
    return SOS_OK;
  }
};

void free_device(sos_batch_s *b) {
  void **ptrs[] = {reinterpret_cast<void **>(&b->d_chans), reinterpret_cast<void **>(&b->d_item_chan),
                   reinterpret_cast<void **>(&b->d_adj), reinterpret_cast<void **>(&b->d_adj_item),
                   reinterpret_cast<void **>(&b->d_adj_red)};
  bool any = false;
  for (void **q : ptrs) any = any || *q;
  if (!any) return;
  int cur = -1;
  hipGetDevice(&cur);
  if (b->device >= 0 && cur != b->device) hipSetDevice(b->device);
  for (void **q : ptrs)
    if (*q) {
      hipFree(*q);
      *q = nullptr;
    }
  if (b->device >= 0 && cur >= 0 && cur != b->device) hipSetDevice(cur);
}

}  // namespace

extern "C" {

sos_status sos_batch_plan(const sos_plan_t *plans, int32_t C, const int64_t *n,
                          const int64_t *offsets, const sos_batch_opts *opts, sos_batch_t *out) {
  if (!plans || !n || !out || C < 1) return SOS_E_ARG;
  sos_batch_opts o{0, 0};
  if (opts) o = *opts;
  if (o.tile_groups < 0) return SOS_E_ARG;
  const bool host_only = (o.flags & SOS_FLAG_HOST_ONLY) != 0;
  for (int c = 0; c < C; ++c) {
    const sos_plan_s *p = plans[c];
    if (!p || n[c] < 0) return SOS_E_ARG;
    if (!host_only && !p->d_table) return SOS_E_ARG;   // a host-only plan cannot filter
    if (p->solver_opt == SOS_PH_DEFERRED || p->solver_opt == SOS_SCALAR || p->solver_opt == SOS_BLOCK)
      return SOS_E_UNSUPPORTED;
    if (p->N != plans[0]->N || p->io_dtype != plans[0]->io_dtype ||
        p->compute_dtype != plans[0]->compute_dtype)
      return SOS_E_UNSUPPORTED;
  }
  sos_batch_s *b = new (std::nothrow) sos_batch_s;
  if (!b) return SOS_E_NOMEM;
  b->C = C;
  b->N = plans[0]->N;
  b->io_dtype = plans[0]->io_dtype;
  b->compute_dtype = plans[0]->compute_dtype;
  b->host_only = host_only;
  b->n.assign(n, n + C);
  b->off.resize(C);
  // offsets: given (channels must not overlap), or dense packing
  if (offsets) {
    std::vector<int32_t> by_off(C);
    std::iota(by_off.begin(), by_off.end(), 0);
    std::stable_sort(by_off.begin(), by_off.end(),
                     [&](int32_t a, int32_t c) { return offsets[a] < offsets[c]; });
    int64_t end = 0;
    for (int i = 0; i < C; ++i) {
      const int32_t c = by_off[i];
      if (offsets[c] < 0 || (n[c] > 0 && offsets[c] < end)) {
        delete b;
        return SOS_E_ARG;
      }
      if (n[c] > 0) end = offsets[c] + n[c];
    }
    for (int c = 0; c < C; ++c) b->off[c] = offsets[c];
  } else {
    int64_t acc = 0;
    for (int c = 0; c < C; ++c) {
      b->off[c] = acc;
      acc += n[c];
    }
  }
  const size_t esz = b->io_dtype == SOS_F64 ? 8 : 4;
  const int64_t G = (int64_t)b->N * kL;
  int64_t total_groups = 0;
  for (int c = 0; c < C; ++c) {
    total_groups += (n[c] + G - 1) / G;
    b->total = std::max(b->total, b->off[c] + n[c]);
  }
  b->mix = plans[0]->solver[0];
  for (int c = 0; c < C; ++c) {
    const sos_plan_s *p = plans[c];
    b->kmax = std::max(b->kmax, p->K);
    b->b0one = b->b0one && p->b0_factored;
    for (int k = 0; k < p->K; ++k)
      if (p->solver[k] != b->mix) b->mix = SOS_AUTO;
  }
  Residency res;
  if (!host_only)
    dispatch_rows<ResidencyBatched>(b->N, b->io_dtype, b->compute_dtype, b->b0one, b->mix, b->kmax, &res);
  const int64_t resident_rows = (int64_t)4 * res.simds * res.waves_per_simd;
  // per-channel tiles: quads of four row tiles, as even as the length allows
  b->tile.assign(C, 0);
  std::vector<int64_t> quads(C, 0);
  std::vector<double> cost(C, 0.0);
  for (int c = 0; c < C; ++c) {
    const sos_plan_s *p = plans[c];
    const int64_t groups = (n[c] + G - 1) / G;
    const int64_t tg = batch_tile_groups(p->warm / G, total_groups, resident_rows, o.tile_groups);
    if (groups == 0) {
      b->tile[c] = G;
      continue;
    }
    quads[c] = (groups + 4 * tg - 1) / (4 * tg);
    const int64_t tgc = (groups + 4 * quads[c] - 1) / (4 * quads[c]);
    b->tile[c] = tgc * G;
    const int64_t warm = std::min<int64_t>(p->warm, (groups - 1) / tgc * tgc * G);
    cost[c] = (double)p->K * (double)(warm + b->tile[c]);
  }
  // launch order: costliest items first (the dispatcher then fills the
  // tail of the launch with the cheap ones)
  b->order.resize(C);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int32_t a, int32_t c) { return cost[a] > cost[c]; });
  b->chans.resize(C);
  for (int i = 0; i < C; ++i) {
    const int32_t c = b->order[i];
    const sos_plan_s *p = plans[c];
    BatchChan &ch = b->chans[i];
    ch.tab = p->d_table;
    ch.solver = static_cast<const int32_t *>(p->d_solver);
    ch.off = b->off[c];
    ch.n = n[c];
    ch.tile = b->tile[c];
    ch.warm = p->warm;
    ch.first_item = b->items;
    ch.K = p->K;
    ch.stride = p->stride;
    ch.gain = p->gain;
    ch.aligned = ((b->off[c] * (int64_t)esz) % 16) == 0;
    ch.pad = 0;
    for (int64_t q = 0; q < quads[c]; ++q) b->item_chan.push_back(i);
    b->items += quads[c];
  }
  if (!host_only) {
    const sos_status sa = build_batch_adjoint(*b, plans, o.tile_groups);
    if (sa != SOS_OK) {
      free_device(b);
      delete b;
      return sa;
    }
  }
  if (!host_only && b->items > 0) {
    if (hipGetDevice(&b->device) != hipSuccess) {
      delete b;
      return SOS_E_DEVICE;
    }
    if (hipMalloc(&b->d_chans, (size_t)C * sizeof(BatchChan)) != hipSuccess ||
        hipMalloc(&b->d_item_chan, (size_t)b->items * sizeof(int32_t)) != hipSuccess) {
      free_device(b);
      delete b;
      return SOS_E_NOMEM;
    }
    if (hipMemcpy(b->d_chans, b->chans.data(), (size_t)C * sizeof(BatchChan), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(b->d_item_chan, b->item_chan.data(), (size_t)b->items * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
      free_device(b);
      delete b;
      return SOS_E_DEVICE;
    }
  }
  *out = b;
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
  if (b->host_only) return SOS_E_ARG;
  if (b->items == 0) return SOS_OK;
  if (!x || !y) return SOS_E_ARG;
  const size_t esz = b->io_dtype == SOS_F64 ? 8 : 4;
  const uintptr_t xb = (uintptr_t)x, yb = (uintptr_t)y, bytes = (uintptr_t)b->total * esz;
  if (xb < yb + bytes && yb < xb + bytes) return SOS_E_ARG;   // overlap
  if ((xb | yb) & 15) return SOS_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return dispatch_rows<LaunchBatched>(b->N, b->io_dtype, b->compute_dtype, b->b0one, b->mix, *b, x, y, s);
}

sos_status sos_batch_tune(const double *const *sos, const int32_t *K, int32_t C, const int64_t *n,
                          const int64_t *offsets, const sos_opts *base, const int32_t *Ns, int32_t nN,
                          const int32_t *tiles, int32_t nt, const void *x, void *y, int32_t reps,
                          sos_stream_t stream, sos_tune_result *results, sos_tune_result *best) {
  if (!sos || !K || !n || !Ns || !tiles || nN < 1 || nt < 1 || reps < 1 || !best || C < 1)
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
  best->tile_groups = 0;
  best->seconds = 0.0;
  sos_status st = SOS_OK;
  for (int iN = 0; iN < nN && st == SOS_OK; ++iN) {
    sos_opts on = o;
    on.N = Ns[iN];
    std::vector<sos_plan_t> plans(C, nullptr);
    for (int c = 0; c < C && st == SOS_OK; ++c) st = sos_plan(sos[c], K[c], &on, &plans[c]);
    for (int it = 0; it < nt && st == SOS_OK; ++it) {
      sos_batch_opts bo{tiles[it], 0};
      sos_batch_t b = nullptr;
      st = sos_batch_plan(plans.data(), C, n, offsets, &bo, &b);
      if (st != SOS_OK) break;
      float ms = 0.f;
      st = sos_filt_batched(b, x, y, nullptr, stream);   // warm-up (code load, clocks)
      if (st == SOS_OK && hipEventRecord(e0, s) != hipSuccess) st = SOS_E_DEVICE;
      for (int r = 0; r < reps && st == SOS_OK; ++r) st = sos_filt_batched(b, x, y, nullptr, stream);
      if (st == SOS_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = SOS_E_DEVICE;
      sos_batch_destroy(b);
      if (st != SOS_OK) break;
      const double sec = (double)ms * 1e-3 / reps;
      if (results) results[iN * nt + it] = sos_tune_result{Ns[iN], tiles[it], sec};
      if (best->N == 0 || sec < best->seconds) *best = sos_tune_result{Ns[iN], tiles[it], sec};
    }
    for (int c = 0; c < C; ++c) sos_plan_destroy(plans[c]);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return st;
}

}  // extern "C"
