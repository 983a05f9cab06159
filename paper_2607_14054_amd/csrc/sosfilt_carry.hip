// Exact inter-tile carry for single signals (kernels_carry.hpp): when to use
// it instead of the run-in, the caller workspace it needs, and its launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "dispatch.hpp"
#include "kernels_carry.hpp"
#include "plan.hpp"

using namespace sosf;

namespace {

template <int N, typename TI, typename T, bool B0ONE, int SOLVER>
struct LaunchCarry {
  static sos_status run(int mode, const void *x, void *y, const void *tab, const int32_t *solver,
                        const CarryArgs &a, hipStream_t s) {
    if constexpr (!std::is_same<T, double>::value) {
      return SOS_E_UNSUPPORTED;   // the carry runs with FP64 arithmetic only
    } else {
      const int64_t per_block = (int64_t)kWavesPerBlock * kRows;
      const unsigned blocks = (unsigned)((a.ntiles + per_block - 1) / per_block);
      const unsigned lds = (unsigned)lds_bytes<N, TI, double>(a.K);
      const TI *xi = static_cast<const TI *>(x);
      TI *yi = static_cast<TI *>(y);
      const double *t = static_cast<const double *>(tab);
      if (mode == CARRY_AGG)
        hipLaunchKernelGGL((sos_rows_carry_kernel<N, TI, B0ONE, SOLVER, CARRY_AGG>), dim3(blocks),
                           dim3(kWavesPerBlock * 64), lds, s, xi, yi, t, solver, a);
      else
        hipLaunchKernelGGL((sos_rows_carry_kernel<N, TI, B0ONE, SOLVER, CARRY_FROM>), dim3(blocks),
                           dim3(kWavesPerBlock * 64), lds, s, xi, yi, t, solver, a);
      return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
    }
  }
};

size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

int mix_of(const sos_plan_s &p) {
  int mix = p.solver[0];
  for (int k = 1; k < p.K; ++k)
    if (p.solver[k] != mix) mix = SOS_AUTO;
  return mix;
}

}  // namespace

namespace sosf {

constexpr int64_t kCarryMinSaving = 8192;   // section-samples of run-in per row

bool carry_supported(const sos_plan_s &p) {
  return p.compute_dtype == SOS_F64 && p.L == kL && p.N >= 8 && p.N <= 64 &&
         (p.solver_opt == SOS_AUTO || p.solver_opt == SOS_PH || p.solver_opt == SOS_CR) &&
         2 * p.K <= kCarryDMax;
}

CarryLayout carry_layout(const sos_plan_s &p, int64_t n, int64_t runin_tile) {
  CarryLayout l;
  if (n <= 0 || !p.d_phi || !carry_supported(p) || (p.flags & SOS_FLAG_CARRY_RUNIN)) return l;
  // automatic choice: the scan when the run-in would more than double the
  // work of the tiles the run-in launch uses (two passes plus the scan),
  // and the run-in it saves, K (W - T) section-samples, outweighs the
  // scan's extra launches (measured: about 8192 section-samples of a
  // row's serial work)
  if (!(p.flags & SOS_FLAG_CARRY_SCAN) &&
      (5 * p.warm <= 6 * runin_tile || (int64_t)p.K * (p.warm - runin_tile) < kCarryMinSaving))
    return l;
  const int64_t G = (int64_t)p.N * kL;
  Residency r;
  r.simds = p.simds;
  r.waves_per_simd = p.waves_per_simd;
  l.tile = (p.tile_groups > 0 ? (int64_t)p.tile_groups : model_tile_groups((n + G - 1) / G, 0, r)) * G;
  l.ntiles = (n + l.tile - 1) / l.tile;
  // rounds until Phi^(tile 2^R) is below the run-in bound, or the scan spans
  // every tile
  l.rounds = 0;
  while (l.rounds < 62 && (l.tile << l.rounds) < p.warm && ((int64_t)1 << l.rounds) < l.ntiles) ++l.rounds;
  const size_t D = 2 * (size_t)p.K;
  l.aggs_off = 0;
  l.buf_off = up256((size_t)l.ntiles * D * 8);
  l.pow_off = l.buf_off + up256((size_t)l.ntiles * D * 8);
  l.bytes = l.pow_off + up256((size_t)std::max(l.rounds, 1) * D * D * 8);
  l.use = true;
  return l;
}

sos_status launch_carry(const sos_plan_s &p, const CarryLayout &l, const void *x, void *y, int64_t n, void *ws,
                        hipStream_t s) {
  unsigned char *w = static_cast<unsigned char *>(ws);
  double *aggs = reinterpret_cast<double *>(w + l.aggs_off);
  double *buf = reinterpret_cast<double *>(w + l.buf_off);
  double *P = reinterpret_cast<double *>(w + l.pow_off);
  const int D = 2 * p.K;
  CarryArgs a;
  a.n = n;
  a.tile = l.tile;
  a.ntiles = l.ntiles;
  a.K = p.K;
  a.stride = p.stride;
  a.gain = p.gain;
  a.states = nullptr;
  a.aggs = aggs;
  const int32_t *solver = static_cast<const int32_t *>(p.d_solver);
  const int mix = mix_of(p);
  // 1. every tile from zero section states: c_t
  sos_status st = dispatch_rows<LaunchCarry>(p.N, p.io_dtype, p.compute_dtype, p.b0_factored, mix, CARRY_AGG,
                                             x, y, p.d_table, solver, a, s);
  if (st != SOS_OK) return st;
  // 2. S_t = c_t + Phi^T S_{t-1}, in log-depth rounds
  double *in = aggs, *out = buf;
  if (l.rounds > 0 && l.ntiles * D <= kCarryOneBlock) {
    // every state in one workgroup's LDS: powers and rounds in one launch
    const size_t lds = ((size_t)l.ntiles * D + 2 * (size_t)D * D) * sizeof(double);
    hipLaunchKernelGGL(carry_scan_one_block_kernel, dim3(1), dim3(1024), lds, s,
                       static_cast<const double *>(p.d_phi), D, l.tile, l.rounds, (int)l.ntiles, in, out);
    if (hipGetLastError() != hipSuccess) return SOS_E_DEVICE;
    std::swap(in, out);
  } else if (l.rounds > 0) {
    hipLaunchKernelGGL(carry_powers_kernel, dim3(1), dim3(1024), 0, s, static_cast<const double *>(p.d_phi), D,
                       l.tile, l.rounds, P);
    if (hipGetLastError() != hipSuccess) return SOS_E_DEVICE;
    const int64_t elems = l.ntiles * D;
    const unsigned blocks = (unsigned)((elems + 255) / 256);
    for (int j = 0; j < l.rounds; ++j) {
      hipLaunchKernelGGL(carry_scan_kernel, dim3(blocks), dim3(256), 0, s, in, out, P + (int64_t)j * D * D, D,
                         l.ntiles, (int64_t)1 << j);
      if (hipGetLastError() != hipSuccess) return SOS_E_DEVICE;
      std::swap(in, out);
    }
  }
  // 3. every tile from S_{t-1}, storing its outputs
  a.states = in;
  a.aggs = nullptr;
  return dispatch_rows<LaunchCarry>(p.N, p.io_dtype, p.compute_dtype, p.b0_factored, mix, CARRY_FROM, x, y,
                                    p.d_table, solver, a, s);
}

}  // namespace sosf
