// C ABI of the cascade's adjoint (include/sosfilt.h): the sub-plan the
// adjoint runs on, the workspace layout and the three launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "dispatch.hpp"
#include "kernels_backward.hpp"
#include "plan.hpp"

using namespace sosf;

namespace sosf {

// The adjoint kernels run PH with FP64 arithmetic at N = kBwdN on their own
// tables (same cascade), and read per section the unfactored rows, the
// forward pass's cumulative b0 scale and the caller's a0.
sos_status attach_adjoint(sos_plan_s &p, const double *sos) {
  sos_opts o{p.io_dtype, SOS_F64, SOS_PH, kBwdN, kL, 0, 0};
  sos_plan_t sub = nullptr;
  sos_status st = create_plan(sos, p.K, &o, false, &sub);
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

}  // namespace sosf

namespace {

struct BwdLayout {
  int64_t np, tile, ntiles, sstride;
  size_t saved_bytes, partial_bytes;
};

BwdLayout layout(const sos_plan_s &p, int64_t n) {
  const sos_plan_s &b = *p.bwd;
  const size_t esz = p.io_dtype == SOS_F64 ? 8 : 4;
  const int64_t V = 16 / (int64_t)esz;
  BwdLayout l;
  l.np = (n + V - 1) / V * V;
  l.tile = sos_plan_tile(p.bwd, std::max<int64_t>(l.np, 1));
  l.ntiles = (l.np + l.tile - 1) / l.tile;
  l.sstride = (n + 63) / 64 * 64;
  l.saved_bytes = (size_t)p.K * (size_t)l.sstride * sizeof(double);
  l.partial_bytes = (size_t)std::max<int64_t>(l.ntiles, 1) * 5 * p.K * sizeof(double);
  (void)b;
  return l;
}

template <typename TI>
sos_status launch_adjoint(const sos_plan_s &p, const void *x, const void *gy, void *gx, double *gsos,
                          int64_t n, void *ws, hipStream_t s) {
  constexpr int N = kBwdN;
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
  const double *tab = static_cast<const double *>(b.d_table);
  const double *rows = static_cast<const double *>(p.d_bwd_rows);
  const int64_t per_block = (int64_t)kWavesPerBlock * kRows;
  if (n > 0) {
    // forward pass saving every section's output (forward-time tiles)
    a.tile = sos_plan_tile(p.bwd, n);
    a.ntiles = (n + a.tile - 1) / a.tile;
    const unsigned lds_f = (unsigned)lds_bytes<N, double, double>(p.K);
    const unsigned blocks_f = (unsigned)((a.ntiles + per_block - 1) / per_block);
    if (b.b0_factored)
      hipLaunchKernelGGL((sos_rows_save_kernel<N, TI, true>), dim3(blocks_f), dim3(kWavesPerBlock * 64),
                         lds_f, s, static_cast<const TI *>(x), saved, tab, rows, a);
    else
      hipLaunchKernelGGL((sos_rows_save_kernel<N, TI, false>), dim3(blocks_f), dim3(kWavesPerBlock * 64),
                         lds_f, s, static_cast<const TI *>(x), saved, tab, rows, a);
    if (hipGetLastError() != hipSuccess) return SOS_E_DEVICE;
    // reversed-time adjoint
    a.tile = l.tile;
    a.ntiles = l.ntiles;
    const unsigned lds_a = (unsigned)(stage_bytes<N, double>() + kWavesPerBlock * kRows * 7 * p.K * 8);
    const unsigned blocks_a = (unsigned)((a.ntiles + per_block - 1) / per_block);
    hipLaunchKernelGGL((sos_rows_adjoint_kernel<N, TI>), dim3(blocks_a), dim3(kWavesPerBlock * 64), lds_a,
                       s, static_cast<const TI *>(gy), static_cast<TI *>(gx), static_cast<const TI *>(x),
                       saved, tab, rows, partials, a);
    if (hipGetLastError() != hipSuccess) return SOS_E_DEVICE;
  }
  hipLaunchKernelGGL(sos_adjoint_reduce_kernel, dim3((unsigned)p.K), dim3(256), 0, s, partials,
                     n > 0 ? l.ntiles : (int64_t)0, (int32_t)p.K, rows, gsos);
  return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
}

}  // namespace

extern "C" {

size_t sos_backward_workspace_size(sos_plan_t p, int64_t n) {
  if (!p || n < 0 || !p->bwd) return 0;
  const BwdLayout l = layout(*p, n);
  return (l.saved_bytes + 255) / 256 * 256 + l.partial_bytes;
}

sos_status sos_filt_backward(sos_plan_t p, const void *x, const void *gy, void *gx, double *gsos,
                             int64_t n, void *workspace, sos_stream_t stream) {
  if (!p || n < 0 || !gsos || !workspace) return SOS_E_ARG;
  if (!p->bwd || !p->d_bwd_rows) return SOS_E_ARG;   // host-only plan
  const size_t esz = p->io_dtype == SOS_F64 ? 8 : 4;
  if (n > 0) {
    if (!x || !gy || !gx) return SOS_E_ARG;
    const uintptr_t xb = (uintptr_t)x, gyb = (uintptr_t)gy, gxb = (uintptr_t)gx;
    const uintptr_t bytes = (uintptr_t)n * esz;
    if ((xb | gyb | gxb | (uintptr_t)workspace) & 15) return SOS_E_ARG;
    // gx may not overlap x or gy (tiles read both beyond their own range)
    if ((gxb < xb + bytes && xb < gxb + bytes) || (gxb < gyb + bytes && gyb < gxb + bytes)) return SOS_E_ARG;
  }
  if ((uintptr_t)gsos & 7) return SOS_E_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (p->io_dtype == SOS_F32) return launch_adjoint<float>(*p, x, gy, gx, gsos, n, workspace, s);
  return launch_adjoint<double>(*p, x, gy, gx, gsos, n, workspace, s);
}

}  // extern "C"
