// Wide groups (N = 128 .. 1024): the plan's kernel instance, its residency,
// the tiles and the workspace that holds the lane runs, and the launch.
// At N = 128 a lane's run (128 doubles) still fits in one wavefront's
// registers when the wavefront has its SIMD to itself (256 architectural
// plus 256 accumulation registers), so with FP32 I/O that width runs the
// register tile kernel of kernels.hpp; the other wide plans keep the runs in
// the workspace (kernels_wide.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "dispatch.hpp"
#include "kernels_wide.hpp"
#include "kernels_wide_deferred.hpp"
#include "plan.hpp"

using namespace sosf;

namespace {

constexpr int kRegN = 128;   // the widest run kept in registers

constexpr size_t kLdsPerCu = 160 * 1024;

// FP32 I/O only: the four wavefronts' staging of a 128-block group in FP64
// would take 266 KB of LDS
bool in_registers(const sos_plan_s &p) {
  return p.N == kRegN && p.io_dtype == SOS_F32 && p.solver_opt != SOS_PH_DEFERRED &&
         (size_t)lds_bytes<kRegN, float, double>(p.K) <= kLdsPerCu;
}

bool deferred(const sos_plan_s &p) { return p.solver_opt == SOS_PH_DEFERRED; }

// the deferred kernel's instance: Theta's 4-wide state blocks (as the plan
// built them, 2, 4 or 8) and b0 factoring
template <typename TI>
const void *wide_deferred_kernel_t(const sos_plan_s &p) {
#define SOSF_DK(B, KB) reinterpret_cast<const void *>(&sos_rows_wide_deferred_kernel<TI, B, KB>)
  if (p.K <= 4) return p.b0_factored ? SOSF_DK(true, 2) : SOSF_DK(false, 2);
  if (p.K <= 8) return p.b0_factored ? SOSF_DK(true, 4) : SOSF_DK(false, 4);
  return p.b0_factored ? SOSF_DK(true, 8) : SOSF_DK(false, 8);
#undef SOSF_DK
}

template <typename TI>
const void *wide_kernel_t(bool regs, bool b0one, int mix) {
#define SOSF_PICK(K)                                                            \
  if (mix == SOS_PH) return b0one ? K(true, SOS_PH) : K(false, SOS_PH);         \
  if (mix == SOS_CR) return b0one ? K(true, SOS_CR) : K(false, SOS_CR);         \
  return b0one ? K(true, SOS_AUTO) : K(false, SOS_AUTO);
#define SOSF_REG(B, S) reinterpret_cast<const void *>(&sos_rows_kernel<kRegN, float, double, B, S, kL>)
#define SOSF_WS(B, S) reinterpret_cast<const void *>(&sos_rows_wide_kernel<TI, B, S>)
  if constexpr (std::is_same<TI, float>::value) {
    if (regs) { SOSF_PICK(SOSF_REG) }
  }
  SOSF_PICK(SOSF_WS)
#undef SOSF_WS
#undef SOSF_REG
#undef SOSF_PICK
}

int mix_of(const sos_plan_s &p) {
  int mix = p.solver[0];
  for (int k = 1; k < p.K; ++k)
    if (p.solver[k] != mix) mix = SOS_AUTO;
  return mix;
}

const void *wide_kernel(const sos_plan_s &p) {
  if (deferred(p))
    return p.io_dtype == SOS_F32 ? wide_deferred_kernel_t<float>(p) : wide_deferred_kernel_t<double>(p);
  return p.io_dtype == SOS_F32 ? wide_kernel_t<float>(in_registers(p), p.b0_factored, mix_of(p))
                               : wide_kernel_t<double>(in_registers(p), p.b0_factored, mix_of(p));
}

size_t wide_lds(const sos_plan_s &p) {
  if (deferred(p))
    return p.io_dtype == SOS_F32 ? (size_t)wide_deferred_lds_bytes<float>(p.K)
                                 : (size_t)wide_deferred_lds_bytes<double>(p.K);
  if (in_registers(p)) return (size_t)lds_bytes<kRegN, float, double>(p.K);   // FP32 I/O only
  return p.io_dtype == SOS_F32 ? (size_t)lds_bytes<kWideChunk, float, double>(p.K)
                               : (size_t)lds_bytes<kWideChunk, double, double>(p.K);
}

}  // namespace

namespace sosf {

bool wide_plan(const sos_plan_s &p) { return p.N > 64; }

Residency wide_residency(const sos_plan_s &p) {
  return residency_of(wide_kernel(p), wide_lds(p), kWavesPerBlock * 64);
}

// Tiles of a wide plan: every SIMD gets one wavefront (four row tiles).  The
// workspace holds N x 64 doubles per wavefront of the launch, so the launch
// keeps to one wavefront per SIMD.  PH and CR also keep to as many
// wavefronts as keep the whole workspace within the 256 MB last-level cache
// that MI355X puts in front of HBM: every section pass reads and writes the
// runs, and from the cache they move faster than the idle SIMDs cost.  At
// N = 1024 that is 512 wavefronts of 512 KB (measured on 2^28 samples, PH:
// 29.6 GS/s, against 27.0 with 1024 wavefronts and 512 MB).  The deferred
// PH moves each run once and uses every SIMD (150 GS/s at N = 1024 with
// 1024 wavefronts, 125 with 512).
constexpr int64_t kWideCacheBytes = (int64_t)256 << 20;

int64_t wide_tile(const sos_plan_s &p, int64_t n) {
  const int64_t G = (int64_t)p.N * kL;
  if (p.tile_groups > 0) return (int64_t)p.tile_groups * G;
  Residency r;
  r.simds = deferred(p) ? p.simds
                        : (int)std::max<int64_t>(
                              std::min<int64_t>(p.simds, kWideCacheBytes / ((int64_t)p.N * 64 * 8)), 1);
  r.waves_per_simd = 1;
  return model_tile_groups((n + G - 1) / G, p.warm / G, r) * G;
}

// AUTO on a wide plan whose runs live in the workspace takes the deferred
// PH (K <= 16): one pass over the run for every section against one per
// section, 4-5 times faster at N = 256 .. 1024 (2^28 samples, K = 8:
// 242 / 204 / 150 against 48 / 43 / 30 GS/s) and at N = 128 with FP64 I/O
// (169 against 43 on 2^26).  N = 128 with FP32 I/O keeps PH in registers
// (321 against 198 on 2^26).
bool wide_auto_deferred(int N, int io_dtype, int K) {
  if (N <= 64 || K > 16) return false;
  return !(N == kRegN && io_dtype == SOS_F32 && (size_t)lds_bytes<kRegN, float, double>(K) <= kLdsPerCu);
}

size_t wide_workspace(const sos_plan_s &p, int64_t n) {
  if (n <= 0 || in_registers(p)) return 0;
  const int64_t tile = wide_tile(p, n);
  const int64_t ntiles = (n + tile - 1) / tile;
  const int64_t waves = (ntiles + kRows - 1) / kRows;
  return (size_t)waves * (size_t)p.N * 64 * sizeof(double);
}

sos_status launch_wide(const sos_plan_s &p, const void *x, void *y, int64_t n, void *ws, hipStream_t s) {
  const int64_t per_block = (int64_t)kWavesPerBlock * kRows;
  const void *xa = x, *ta = p.d_table, *sa = p.d_solver;
  void *ya = y;
  if (in_registers(p)) {
    FiltArgs f;
    f.n = n;
    f.K = p.K;
    f.stride = p.stride;
    f.tile = wide_tile(p, n);
    f.warm = p.warm;
    f.ntiles = (n + f.tile - 1) / f.tile;
    f.gain = p.gain;
    const int64_t blocks = (f.ntiles + per_block - 1) / per_block;
    void *args[] = {&xa, &ya, &ta, &sa, &f};   // addresses of the kernel's five arguments
    if (hipLaunchKernel(wide_kernel(p), dim3((unsigned)blocks), dim3(kWavesPerBlock * 64), args, wide_lds(p),
                        s) != hipSuccess)
      return SOS_E_DEVICE;
    return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
  }
  WideArgs a;
  a.n = n;
  a.K = p.K;
  a.stride = p.stride;
  a.N = p.N;
  a.lgN = p.lgN;
  a.tile = wide_tile(p, n);
  a.warm = p.warm;
  a.ntiles = (n + a.tile - 1) / a.tile;
  a.gain = p.gain;
  a.ws = static_cast<double *>(ws);
  const int64_t blocks = (a.ntiles + per_block - 1) / per_block;
  if (deferred(p)) {
    const void *ca = p.d_coupling, *tha = p.d_theta;
    void *dargs[] = {&xa, &ya, &ta, &ca, &tha, &a};   // addresses of the kernel's six arguments
    if (hipLaunchKernel(wide_kernel(p), dim3((unsigned)blocks), dim3(kWavesPerBlock * 64), dargs, wide_lds(p),
                        s) != hipSuccess)
      return SOS_E_DEVICE;
    return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
  }
  void *args[] = {&xa, &ya, &ta, &sa, &a};   // addresses of the kernel's five arguments
  if (hipLaunchKernel(wide_kernel(p), dim3((unsigned)blocks), dim3(kWavesPerBlock * 64), args, wide_lds(p), s) !=
      hipSuccess)
    return SOS_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
}

}  // namespace sosf
