// Host-side selection of a tile-kernel instance (N, I/O type, compute type,
// b0 factoring, solver mix) and the launch-shape model shared by the
// single-signal and batched launches.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "plan.hpp"

namespace sosf {

// Calls Op<N, TI, T, B0ONE, SOLVER>::run(args...) for the runtime choice.
template <template <int, typename, typename, bool, int> class Op, int N, typename TI, typename T,
          bool B0ONE, typename... A>
sos_status dispatch_mix(int mix, A &&...args) {
  if (mix == SOS_PH) return Op<N, TI, T, B0ONE, SOS_PH>::run(args...);
  if (mix == SOS_CR) return Op<N, TI, T, B0ONE, SOS_CR>::run(args...);
  return Op<N, TI, T, B0ONE, SOS_AUTO>::run(args...);
}

template <template <int, typename, typename, bool, int> class Op, typename TI, typename T,
          typename... A>
sos_status dispatch_n(int N, bool b0one, int mix, A &&...args) {
#define SOSF_CASE(NN)                                                        \
  case NN:                                                                   \
    return b0one ? dispatch_mix<Op, NN, TI, T, true>(mix, args...)           \
                 : dispatch_mix<Op, NN, TI, T, false>(mix, args...);
  switch (N) {
    SOSF_CASE(8)
    SOSF_CASE(16)
    SOSF_CASE(32)
    SOSF_CASE(64)
    default: return SOS_E_UNSUPPORTED;
  }
#undef SOSF_CASE
}

template <template <int, typename, typename, bool, int> class Op, typename... A>
sos_status dispatch_rows(int N, int io, int cd, bool b0one, int mix, A &&...args) {
  if (io == SOS_F32 && cd == SOS_F32) return dispatch_n<Op, float, float>(N, b0one, mix, args...);
  if (io == SOS_F32 && cd == SOS_F64) return dispatch_n<Op, float, double>(N, b0one, mix, args...);
  if (io == SOS_F64 && cd == SOS_F64) return dispatch_n<Op, double, double>(N, b0one, mix, args...);
  return SOS_E_UNSUPPORTED;
}

// The same for kernels that also take the block size L (16, 32 or 64):
// Op<N, TI, T, B0ONE, SOLVER, L>.
template <template <int, typename, typename, bool, int, int> class Op, int L>
struct BindL {
  template <int N, typename TI, typename T, bool B0ONE, int SOLVER>
  struct type : Op<N, TI, T, B0ONE, SOLVER, L> {};
};

template <template <int, typename, typename, bool, int, int> class Op, typename... A>
sos_status dispatch_rows_l(int N, int L, int io, int cd, bool b0one, int mix, A &&...args) {
  switch (L) {
    case 16: return dispatch_rows<BindL<Op, 16>::template type>(N, io, cd, b0one, mix, args...);
    case 32: return dispatch_rows<BindL<Op, 32>::template type>(N, io, cd, b0one, mix, args...);
    case 64: return dispatch_rows<BindL<Op, 64>::template type>(N, io, cd, b0one, mix, args...);
    default: return SOS_E_UNSUPPORTED;
  }
}

// Resident capacity of the device for one kernel: SIMDs and wavefronts per
// SIMD (from the kernel's registers and LDS).
struct Residency {
  int simds = 1024;
  int waves_per_simd = 4;
};

inline Residency residency_of(const void *kernel, size_t lds, int block_threads) {
  Residency r;
  int dev = 0, cus = 0, blocks = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    r.simds = 4 * cus;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, block_threads, lds) == hipSuccess &&
      blocks > 0)
    r.waves_per_simd = std::max(1, blocks * (block_threads / 64) / 4);
  return r;
}

// Groups per tile for a signal of `groups` groups.  64 / L rows (tiles)
// make one wavefront.  Measured on the 2^28-sample cascade, launches are
// fastest when every SIMD receives the same number of wavefronts m, and m
// is the largest power of two the kernel keeps resident per SIMD: fewer
// leaves the recurrences' latency exposed, and counts that do not divide
// evenly (or odd multiples) leave part of the chip idle at the end.  So the
// tile is the shortest that gives at most m wavefronts per SIMD.
inline int64_t model_tile_groups(int64_t groups, int64_t warm_groups, const Residency &r, int rows_per_wave = 4) {
  (void)warm_groups;
  int64_t m = 1;
  while (2 * m <= r.waves_per_simd) m *= 2;
  const int64_t rows = (int64_t)rows_per_wave * r.simds * m;
  return std::max<int64_t>((groups + rows - 1) / rows, 1);
}

// residency of a wide plan's kernel (sosfilt_wide.hip), and whether AUTO
// takes the deferred PH there
Residency wide_residency(const sos_plan_s &p);
bool wide_auto_deferred(int N, int io_dtype, int K);

// a narrow plan's residency and launch (sosfilt_narrow.hip)
struct FiltArgs;
Residency narrow_residency(const sos_plan_s &p);
sos_status launch_narrow(const sos_plan_s &p, const void *x, void *y, const FiltArgs &a, hipStream_t s);

}  // namespace sosf
