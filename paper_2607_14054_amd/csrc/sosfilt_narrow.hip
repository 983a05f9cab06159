// Narrow groups (N = 4 blocks per lane run, L = 16): single signals, PH and
// CR (Section VI), on the register tile kernel of kernels.hpp.  The width
// the paper's reformulation admits at its low end (cyclic reduction's
// four- and two-block levels need N >= 4); it has its own instances so that
// the batched and carry kernels are not built for it.
#include <hip/hip_runtime.h>

#include "dispatch.hpp"
#include "kernels.hpp"
#include "plan.hpp"

using namespace sosf;

namespace {

constexpr int kNarrowN = 4;

template <typename TI, typename T>
const void *narrow_kernel_t(bool b0one, int mix) {
#define SOSF_K(B, S) reinterpret_cast<const void *>(&sos_rows_kernel<kNarrowN, TI, T, B, S, kL>)
  if (mix == SOS_PH) return b0one ? SOSF_K(true, SOS_PH) : SOSF_K(false, SOS_PH);
  if (mix == SOS_CR) return b0one ? SOSF_K(true, SOS_CR) : SOSF_K(false, SOS_CR);
  return b0one ? SOSF_K(true, SOS_AUTO) : SOSF_K(false, SOS_AUTO);
#undef SOSF_K
}

int mix_of(const sos_plan_s &p) {
  int mix = p.solver[0];
  for (int k = 1; k < p.K; ++k)
    if (p.solver[k] != mix) mix = SOS_AUTO;
  return mix;
}

const void *narrow_kernel(const sos_plan_s &p) {
  if (p.io_dtype == SOS_F64) return narrow_kernel_t<double, double>(p.b0_factored, mix_of(p));
  if (p.compute_dtype == SOS_F64) return narrow_kernel_t<float, double>(p.b0_factored, mix_of(p));
  return narrow_kernel_t<float, float>(p.b0_factored, mix_of(p));
}

size_t narrow_lds(const sos_plan_s &p) {
  if (p.io_dtype == SOS_F64) return (size_t)lds_bytes<kNarrowN, double, double>(p.K);
  if (p.compute_dtype == SOS_F64) return (size_t)lds_bytes<kNarrowN, float, double>(p.K);
  return (size_t)lds_bytes<kNarrowN, float, float>(p.K);
}

}  // namespace

namespace sosf {

bool narrow_plan(const sos_plan_s &p) { return p.N == kNarrowN; }

Residency narrow_residency(const sos_plan_s &p) {
  return residency_of(narrow_kernel(p), narrow_lds(p), kWavesPerBlock * 64);
}

sos_status launch_narrow(const sos_plan_s &p, const void *x, void *y, const FiltArgs &a, hipStream_t s) {
  const int64_t per_block = (int64_t)kWavesPerBlock * kRows;
  const int64_t blocks = (a.ntiles + per_block - 1) / per_block;
  const void *xa = x, *ta = p.d_table, *sa = p.d_solver;
  void *ya = y;
  FiltArgs f = a;
  void *args[] = {&xa, &ya, &ta, &sa, &f};   // addresses of the kernel's five arguments
  if (hipLaunchKernel(narrow_kernel(p), dim3((unsigned)blocks), dim3(kWavesPerBlock * 64), args, narrow_lds(p),
                      s) != hipSuccess)
    return SOS_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
}

}  // namespace sosf
