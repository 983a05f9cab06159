// C ABI entry points (include/sosfilt.h): plan creation and upload, queries,
// and the launch of the tile kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "kernels.hpp"
#include "dispatch.hpp"
#include "kernels_deferred.hpp"
#include "kernels_scalar.hpp"
#include "kernels_block.hpp"
#include "kernels_wide.hpp"
#include "plan.hpp"

using namespace sosf;

namespace {

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

sos_status upload(sos_plan_s &p) {
  if (hipGetDevice(&p.device) != hipSuccess) return SOS_E_DEVICE;
  const size_t count = (size_t)p.K * p.stride;
  const size_t esz = p.compute_dtype == SOS_F64 ? 8 : 4;
  if (hipMalloc(&p.d_table, count * esz) != hipSuccess) { p.d_table = nullptr; return SOS_E_NOMEM; }
  if (hipMalloc(&p.d_solver, (size_t)p.K * sizeof(int32_t)) != hipSuccess) {
    hipFree(p.d_table);
    p.d_table = nullptr;
    p.d_solver = nullptr;
    return SOS_E_NOMEM;
  }
  hipError_t e1, e2;
  if (esz == 8) {
    e1 = hipMemcpy(p.d_table, p.table.data(), count * 8, hipMemcpyHostToDevice);
  } else {
    std::vector<float> f(count);
    for (size_t i = 0; i < count; ++i) f[i] = (float)p.table[i];
    e1 = hipMemcpy(p.d_table, f.data(), count * 4, hipMemcpyHostToDevice);
  }
  e2 = hipMemcpy(p.d_solver, p.solver.data(), (size_t)p.K * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e1 != hipSuccess || e2 != hipSuccess) return SOS_E_DEVICE;
  if (p.solver_opt == SOS_PH_DEFERRED) {
    const size_t nt = p.theta_mfma.size(), nc = p.coupling.size() ? p.coupling.size() : 1;
    if (hipMalloc(&p.d_theta, nt * 8) != hipSuccess) { p.d_theta = nullptr; return SOS_E_NOMEM; }
    if (hipMalloc(&p.d_coupling, nc * 8) != hipSuccess) { p.d_coupling = nullptr; return SOS_E_NOMEM; }
    if (hipMemcpy(p.d_theta, p.theta_mfma.data(), nt * 8, hipMemcpyHostToDevice) != hipSuccess) return SOS_E_DEVICE;
    if (p.coupling.size() &&
        hipMemcpy(p.d_coupling, p.coupling.data(), p.coupling.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return SOS_E_DEVICE;
  }
  return SOS_OK;
}

struct Ptrs {
  const void *x;
  void *y;
  const void *tab;
  const int32_t *solver;
};

template <int N, typename TI, typename T, bool B0ONE, int SOLVER, int L>
struct LaunchRows {
  static sos_status run(const Ptrs &q, const FiltArgs &a, hipStream_t s) {
    const int64_t per_block = (int64_t)kWavesPerBlock * (64 / L);
    const int64_t blocks = (a.ntiles + per_block - 1) / per_block;
    const unsigned lds = (unsigned)lds_bytes<N, TI, T, L>(a.K);
    hipLaunchKernelGGL((sos_rows_kernel<N, TI, T, B0ONE, SOLVER, L>), dim3((unsigned)blocks),
                       dim3(kWavesPerBlock * 64), lds, s,
                       static_cast<const TI *>(q.x), static_cast<TI *>(q.y),
                       static_cast<const T *>(q.tab), q.solver, a);
    return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
  }
};

template <int N, typename TI, typename T, bool B0ONE, int SOLVER, int L>
struct ResidencyRows {
  static sos_status run(int K, Residency *r) {
    *r = residency_of(reinterpret_cast<const void *>(&sos_rows_kernel<N, TI, T, B0ONE, SOLVER, L>),
                      (size_t)lds_bytes<N, TI, T, L>(K), kWavesPerBlock * 64);
    return SOS_OK;
  }
};

template <int N, typename TI, int KBM>
sos_status launch_deferred_k(const Ptrs &q, const void *coup, const void *theta, const FiltArgs &a,
                             bool b0one, hipStream_t s) {
  const int64_t per_block = (int64_t)kWavesPerBlock * kRows;
  const int64_t blocks = (a.ntiles + per_block - 1) / per_block;
  const TI *x = static_cast<const TI *>(q.x);
  TI *y = static_cast<TI *>(q.y);
  const double *tab = static_cast<const double *>(q.tab);
  const double *cp = static_cast<const double *>(coup), *th = static_cast<const double *>(theta);
  const unsigned lds = (unsigned)deferred_lds_bytes<N, TI>(a.K, KBM);
  if (b0one)
    hipLaunchKernelGGL((sos_rows_deferred_kernel<N, TI, true, KBM>), dim3((unsigned)blocks),
                       dim3(kWavesPerBlock * 64), lds, s, x, y, tab, cp, th, a);
  else
    hipLaunchKernelGGL((sos_rows_deferred_kernel<N, TI, false, KBM>), dim3((unsigned)blocks),
                       dim3(kWavesPerBlock * 64), lds, s, x, y, tab, cp, th, a);
  return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
}

template <int N, typename TI>
sos_status launch_deferred_n(const Ptrs &q, const void *coup, const void *theta, const FiltArgs &a,
                             bool b0one, hipStream_t s) {
  if (a.K <= 4) return launch_deferred_k<N, TI, 2>(q, coup, theta, a, b0one, s);
  if (a.K <= 8) return launch_deferred_k<N, TI, 4>(q, coup, theta, a, b0one, s);
  return launch_deferred_k<N, TI, 8>(q, coup, theta, a, b0one, s);
}

template <typename TI>
sos_status launch_deferred(int N, const Ptrs &q, const void *coup, const void *theta,
                           const FiltArgs &a, bool b0one, hipStream_t s) {
  switch (N) {
    case 16: return launch_deferred_n<16, TI>(q, coup, theta, a, b0one, s);
    case 32: return launch_deferred_n<32, TI>(q, coup, theta, a, b0one, s);
    case 64: return launch_deferred_n<64, TI>(q, coup, theta, a, b0one, s);
    default: return SOS_E_UNSUPPORTED;
  }
}

template <int N, typename TI>
Residency deferred_residency_n(int K, bool b0one) {
  const int kbm = K <= 4 ? 2 : (K <= 8 ? 4 : 8);
  const size_t lds = (size_t)deferred_lds_bytes<N, TI>(K, kbm);
  const void *f;
  if (kbm == 2) f = b0one ? reinterpret_cast<const void *>(&sos_rows_deferred_kernel<N, TI, true, 2>)
                          : reinterpret_cast<const void *>(&sos_rows_deferred_kernel<N, TI, false, 2>);
  else if (kbm == 4) f = b0one ? reinterpret_cast<const void *>(&sos_rows_deferred_kernel<N, TI, true, 4>)
                               : reinterpret_cast<const void *>(&sos_rows_deferred_kernel<N, TI, false, 4>);
  else f = b0one ? reinterpret_cast<const void *>(&sos_rows_deferred_kernel<N, TI, true, 8>)
                 : reinterpret_cast<const void *>(&sos_rows_deferred_kernel<N, TI, false, 8>);
  return residency_of(f, lds, kWavesPerBlock * 64);
}

template <typename TI>
Residency deferred_residency(int N, int K, bool b0one) {
  if (N == 16) return deferred_residency_n<16, TI>(K, b0one);
  if (N == 32) return deferred_residency_n<32, TI>(K, b0one);
  return deferred_residency_n<64, TI>(K, b0one);
}

int solver_mix(const sos_plan_s &p) {
  int mix = p.solver[0];
  for (int k = 1; k < p.K; ++k)
    if (p.solver[k] != mix) mix = SOS_AUTO;
  return mix;
}

// Scalar filtering (comparison point): kernel instance by I/O and compute
// type, b0 factoring and the bound on K.
template <typename TI, typename T, int KMAX>
const void *scalar_kernel_k(bool b0one) {
  return b0one ? reinterpret_cast<const void *>(&sos_scalar_kernel<TI, T, true, KMAX>)
               : reinterpret_cast<const void *>(&sos_scalar_kernel<TI, T, false, KMAX>);
}
template <typename TI, typename T>
const void *scalar_kernel_t(int K, bool b0one) {
  if (K <= 4) return scalar_kernel_k<TI, T, 4>(b0one);
  if (K <= 8) return scalar_kernel_k<TI, T, 8>(b0one);
  return scalar_kernel_k<TI, T, 16>(b0one);
}
const void *scalar_kernel(const sos_plan_s &p) {
  if (p.io_dtype == SOS_F32 && p.compute_dtype == SOS_F32) return scalar_kernel_t<float, float>(p.K, p.b0_factored);
  if (p.io_dtype == SOS_F32) return scalar_kernel_t<float, double>(p.K, p.b0_factored);
  return scalar_kernel_t<double, double>(p.K, p.b0_factored);
}
size_t scalar_lds(const sos_plan_s &p) {
  return (size_t)kWavesPerBlock * (p.io_dtype == SOS_F32 ? ScalarStage<float>::ELEMS * 4
                                                           : ScalarStage<double>::ELEMS * 8);
}
Residency scalar_residency(const sos_plan_s &p) {
  return residency_of(scalar_kernel(p), scalar_lds(p), kWavesPerBlock * 64);
}

// Segment length of the scalar kernel: every SIMD gets m wavefronts of 64
// segments, m as in model_tile_groups.
int64_t scalar_segment(const sos_plan_s &p, int64_t n) {
  int64_t m = 1;
  while (2 * m <= p.waves_per_simd) m *= 2;
  const int64_t lanes = (int64_t)p.simds * m * 64;
  const int64_t seg = (n + lanes - 1) / lanes;
  return std::max<int64_t>((seg + kScalarChunk - 1) / kScalarChunk * kScalarChunk, kScalarChunk);
}

sos_status launch_scalar(const sos_plan_s &p, const void *x, void *y, int64_t n, hipStream_t s) {
  ScalarArgs a;
  a.n = n;
  a.seg = p.tile_groups > 0 ? (int64_t)p.tile_groups * kScalarChunk : scalar_segment(p, n);
  a.warm = p.warm;
  a.nseg = (n + a.seg - 1) / a.seg;
  a.K = p.K;
  a.stride = p.stride;
  a.gain = p.gain;
  const int64_t blocks = (a.nseg + kWavesPerBlock * 64 - 1) / (kWavesPerBlock * 64);
  const void *xa = x, *ta = p.d_table;
  void *ya = y;
  void *args[] = {&xa, &ya, &ta, &a};   // addresses of the kernel's four arguments
  const void *f = scalar_kernel(p);
  if (hipLaunchKernel(f, dim3((unsigned)blocks), dim3(kWavesPerBlock * 64), args, scalar_lds(p), s) !=
      hipSuccess)
    return SOS_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
}

// Tile length for n samples: the plan's fixed choice, or the launch-shape
// model for the kernel the plan runs.
int64_t choose_tile(const sos_plan_s &p, int64_t n) {
  const int64_t G = (int64_t)p.N * p.L;
  if (p.tile_groups > 0) return (int64_t)p.tile_groups * G;
  const int64_t groups = (n + G - 1) / G;
  Residency r;
  r.simds = p.simds;
  r.waves_per_simd = p.waves_per_simd;
  return model_tile_groups(groups, p.warm / G, r, 64 / p.L) * G;
}

}  // namespace

namespace sosf {

// sos_filt's checks of x, y and the plan for n > 0 samples.
sos_status check_filt_args(const sos_plan_s &p, const void *x, const void *y, int64_t n) {
  if (!x || !y) return SOS_E_ARG;
  if (!p.d_table) return SOS_E_ARG;   // a host-only plan cannot filter
  const size_t esz = p.io_dtype == SOS_F64 ? 8 : 4;
  const uintptr_t xb = (uintptr_t)x, yb = (uintptr_t)y;
  if (xb < yb + (uintptr_t)n * esz && yb < xb + (uintptr_t)n * esz) return SOS_E_ARG;   // overlap
  if ((xb | yb) & 15) return SOS_E_ARG;   // 16-byte vector access
  return SOS_OK;
}

}  // namespace sosf

extern "C" {

const char *sos_status_string(sos_status s) {
  switch (s) {
    case SOS_OK: return "ok";
    case SOS_E_ARG: return "invalid argument";
    case SOS_E_COEF: return "invalid coefficients (a0 == 0 or non-finite)";
    case SOS_E_UNSTABLE: return "unstable section (a pole on or outside the unit circle)";
    case SOS_E_UNSUPPORTED: return "unsupported configuration";
    case SOS_E_DEVICE: return "HIP device error";
    case SOS_E_NOMEM: return "out of memory";
    case SOS_E_SCRATCH: return "workspace needed exceeds the static scratch buffer (SOS_STATIC_SCRATCH_BYTES)";
  }
  return "unknown status";
}

sos_status sos_plan(const double *sos, int32_t K, const sos_opts *opts, sos_plan_t *out) {
  constexpr uint32_t known = SOS_FLAG_HOST_ONLY | SOS_FLAG_CARRY_SCAN | SOS_FLAG_CARRY_RUNIN |
                             SOS_FLAG_ADJ_SAVE | SOS_FLAG_ADJ_RECOMPUTE | SOS_FLAG_SLICES_MASK;
  if (opts && (opts->flags & ~known)) return SOS_E_ARG;
  if (opts && (opts->flags & SOS_FLAG_CARRY_SCAN) && (opts->flags & SOS_FLAG_CARRY_RUNIN)) return SOS_E_ARG;
  if (opts && (opts->flags & SOS_FLAG_ADJ_SAVE) && (opts->flags & SOS_FLAG_ADJ_RECOMPUTE)) return SOS_E_ARG;
  return create_plan(sos, K, opts, true, out);
}

}  // extern "C"

// Plan creation; `adjoint` also attaches the adjoint's sub-plan (device
// plans only).
sos_status create_plan(const double *sos, int32_t K, const sos_opts *opts, bool adjoint,
                       sos_plan_t *out, double runin_eps) {
  if (!sos || !out || K < 1 || K > SOS_MAX_SECTIONS) return SOS_E_ARG;
  sos_opts o{SOS_F32, SOS_F64, SOS_AUTO, 0, 0, 0, 0};
  if (opts) o = *opts;
  if (o.N == 0) o.N = 32;
  if (o.L == 0) o.L = 16;
  if (o.io_dtype != SOS_F32 && o.io_dtype != SOS_F64) return SOS_E_ARG;
  if (o.compute_dtype < SOS_F32 || o.compute_dtype > SOS_BF16) return SOS_E_ARG;
  if (o.solver < SOS_AUTO || o.solver > SOS_BLOCK) return SOS_E_ARG;
  const bool low = o.compute_dtype == SOS_F16 || o.compute_dtype == SOS_BF16;
  if (low && o.solver != SOS_BLOCK) return SOS_E_UNSUPPORTED;
  if (o.solver == SOS_BLOCK && o.compute_dtype == SOS_F32) return SOS_E_UNSUPPORTED;
  if (o.tile_groups < 0) return SOS_E_ARG;
  if (!pow2_in(o.N, 4, kWideMaxN) || !pow2_in(o.L, 16, 64)) return SOS_E_UNSUPPORTED;
  // N = 4: single signals, PH and CR on 16-lane rows (sosfilt_narrow.hip)
  if (o.N == 4 && (o.L != kL || !(o.solver == SOS_AUTO || o.solver == SOS_PH || o.solver == SOS_CR)))
    return SOS_E_UNSUPPORTED;
  // N = 128 .. 1024: the lane runs live in the workspace (kernels_wide.hpp),
  // for PH, CR and the deferred-correction PH with FP64 arithmetic and
  // 16-lane rows
  if (o.N > 64 && (o.L != kL || o.compute_dtype != SOS_F64 ||
                   !(o.solver == SOS_AUTO || o.solver == SOS_PH || o.solver == SOS_CR ||
                     o.solver == SOS_PH_DEFERRED)))
    return SOS_E_UNSUPPORTED;
  // the block sizes L = 32, 64 exist for PH and CR (the other solvers work
  // on 16-lane rows or single lanes)
  if (o.L != kL && !(o.solver == SOS_AUTO || o.solver == SOS_PH || o.solver == SOS_CR)) return SOS_E_UNSUPPORTED;
  if (o.io_dtype == SOS_F64 && (o.compute_dtype == SOS_F32 || low)) return SOS_E_UNSUPPORTED;
  const bool deferred_ok = o.compute_dtype == SOS_F64 && o.N >= 16 && K <= 16;
  if (o.solver == SOS_PH_DEFERRED && !deferred_ok) return SOS_E_UNSUPPORTED;
  if (o.solver == SOS_SCALAR && K > kScalarKMax) return SOS_E_UNSUPPORTED;
  if (o.solver == SOS_BLOCK && K > kBlockKMax) return SOS_E_UNSUPPORTED;
  const int slices = (int)((o.flags & SOS_FLAG_SLICES_MASK) >> 8);
  if (slices > kMaxSlices) return SOS_E_ARG;
  if (slices > 1 && !low) return SOS_E_UNSUPPORTED;   // FP64 products are not sliced
  sos_plan_s *p = new (std::nothrow) sos_plan_s;
  if (!p) return SOS_E_NOMEM;
  p->K = K;
  p->N = o.N;
  p->L = o.L;
  p->lgN = __builtin_ctz((unsigned)o.N);
  p->io_dtype = o.io_dtype;
  p->compute_dtype = o.compute_dtype;
  p->solver_opt = (o.solver == SOS_AUTO && o.compute_dtype == SOS_F64 && o.L == kL &&
                   wide_auto_deferred(o.N, o.io_dtype, K))
                      ? SOS_PH_DEFERRED
                      : o.solver;
  p->tile_groups = o.tile_groups;
  p->flags = o.flags;
  p->block_slices = !low ? 1 : (slices ? slices : (o.compute_dtype == SOS_F16 ? 3 : 4));
  p->runin_eps = runin_eps;
  sos_status st = build_plan_tables(*p, sos);
  if (st == SOS_OK && p->solver_opt == SOS_PH_DEFERRED) {
    build_deferred_tables(*p);
    for (int k = 0; k < K; ++k) p->solver[k] = SOS_PH_DEFERRED;
  }
  if (st == SOS_OK && p->solver_opt == SOS_BLOCK) {
    for (int k = 0; k < K; ++k) p->solver[k] = SOS_BLOCK;
    st = build_block_plan(*p);
  }
  if (st == SOS_OK && p->solver_opt == SOS_SCALAR) {
    for (int k = 0; k < K; ++k) p->solver[k] = SOS_SCALAR;
    // the scalar kernel's run-in moves in whole chunks
    p->warm = (p->warm + kScalarChunk - 1) / kScalarChunk * kScalarChunk;
  }
  if (st == SOS_OK && !(o.flags & SOS_FLAG_HOST_ONLY)) {
    st = upload(*p);
    if (st == SOS_OK && carry_supported(*p)) {
      // the transition the exact inter-tile carry raises to the tile length
      const size_t bytes = p->phi.size() * sizeof(double);
      if (hipMalloc(&p->d_phi, bytes) != hipSuccess) {
        p->d_phi = nullptr;
        st = SOS_E_NOMEM;
      } else if (hipMemcpy(p->d_phi, p->phi.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        st = SOS_E_DEVICE;
      }
    }
    Residency r;
    if (st == SOS_OK && p->solver_opt == SOS_PH_DEFERRED && !wide_plan(*p))
      r = p->io_dtype == SOS_F32 ? deferred_residency<float>(p->N, p->K, p->b0_factored)
                                 : deferred_residency<double>(p->N, p->K, p->b0_factored);
    else if (st == SOS_OK && p->solver_opt == SOS_SCALAR)
      r = scalar_residency(*p);
    else if (st == SOS_OK && p->solver_opt == SOS_BLOCK) {
      st = upload_block_plan(*p);
      r.simds = p->simds;
      r.waves_per_simd = p->waves_per_simd;
    } else if (st == SOS_OK && wide_plan(*p)) {
      r = wide_residency(*p);
    } else if (st == SOS_OK && narrow_plan(*p)) {
      r = narrow_residency(*p);
    } else if (st == SOS_OK)
      dispatch_rows_l<ResidencyRows>(p->N, p->L, p->io_dtype, p->compute_dtype, p->b0_factored, solver_mix(*p),
                                     p->K, &r);
    p->simds = r.simds;
    p->waves_per_simd = r.waves_per_simd;
    if (st == SOS_OK && adjoint) st = attach_adjoint(*p, sos);
  }
  if (st != SOS_OK) {
    sos_plan_destroy(p);
    return st;
  }
  *out = p;
  return SOS_OK;
}

extern "C" {

sos_status sos_plan_destroy(sos_plan_t p) {
  if (!p) return SOS_OK;
  if (p->d_table || p->d_solver) {
    int cur = -1;
    hipGetDevice(&cur);
    if (p->device >= 0 && cur != p->device) hipSetDevice(p->device);
    if (p->d_table) hipFree(p->d_table);
    if (p->d_solver) hipFree(p->d_solver);
    if (p->d_theta) hipFree(p->d_theta);
    if (p->d_coupling) hipFree(p->d_coupling);
    if (p->d_bwd_rows) hipFree(p->d_bwd_rows);
    if (p->d_block) hipFree(p->d_block);
    if (p->d_aop) hipFree(p->d_aop);
    if (p->d_phi) hipFree(p->d_phi);
    if (p->device >= 0 && cur >= 0 && cur != p->device) hipSetDevice(cur);
  }
  if (p->bwd) sos_plan_destroy(p->bwd);
  delete p;
  return SOS_OK;
}

sos_status sos_plan_query(sos_plan_t p, sos_plan_info *info, int32_t *solver) {
  if (!p) return SOS_E_ARG;
  if (info) {
    info->K = p->K;
    info->N = p->N;
    info->L = p->L;
    info->io_dtype = p->io_dtype;
    info->compute_dtype = p->compute_dtype;
    info->b0_factored = p->b0_factored ? 1 : 0;
    info->warm_samples = p->warm;
    info->gain = p->gain;
    info->transition_norm_W = p->warm_norm;
    info->simds = p->d_table ? p->simds : 0;
    info->waves_per_simd = p->d_table ? p->waves_per_simd : 0;
    info->block_slices = p->block_slices;
    info->reserved = 0;
  }
  if (solver)
    for (int k = 0; k < p->K; ++k) solver[k] = p->solver[k];
  return SOS_OK;
}

sos_status sos_plan_table(sos_plan_t p, int32_t table, int32_t section, double *out,
                          int32_t count, int32_t *size) {
  if (!p || count < 0 || (count > 0 && !out)) return SOS_E_ARG;
  if (table != SOS_TABLE_TRANSITION && table != SOS_TABLE_THETA && (section < 0 || section >= p->K))
    return SOS_E_ARG;
  const double *t = p->table.data() + (size_t)(section < 0 ? 0 : section) * p->stride;
  std::vector<double> buf;
  switch (table) {
    case SOS_TABLE_ROWS: buf.assign(p->rows.begin() + 5 * section, p->rows.begin() + 5 * section + 5); break;
    case SOS_TABLE_U1: buf.assign(t + OFF_U1, t + OFF_U1 + p->N); break;
    case SOS_TABLE_U2: buf.assign(t + off_u2(p->N), t + off_u2(p->N) + p->N); break;
    case SOS_TABLE_C: buf.assign(p->C.begin() + 4 * section, p->C.begin() + 4 * section + 4); break;
    case SOS_TABLE_PH_POWERS: buf.assign(t + OFF_PH_POW, t + OFF_PH_POW + 4 * __builtin_ctz((unsigned)p->L)); break;
    case SOS_TABLE_CR_LEVELS: buf.assign(t + OFF_CR_LVL, t + OFF_CR_LVL + 4 * p->lgN); break;
    case SOS_TABLE_CR_TERMINAL: buf.assign(p->cr_term.begin() + 2 * section, p->cr_term.begin() + 2 * section + 2); break;
    case SOS_TABLE_CR_POWERS: buf.assign(t + OFF_CR_POW, t + OFF_CR_POW + 4 * __builtin_ctz((unsigned)p->L)); break;
    case SOS_TABLE_TRANSITION: buf = p->phi; break;
    case SOS_TABLE_THETA:
      if (p->theta.empty()) return SOS_E_ARG;
      buf = p->theta;
      break;
    case SOS_TABLE_COUPLING:
      if (p->theta.empty()) return SOS_E_ARG;
      buf.assign(p->coupling.begin() + 2 * section * (section - 1),
                 p->coupling.begin() + 2 * section * (section + 1));
      break;
    default: return SOS_E_ARG;
  }
  if (size) *size = (int32_t)buf.size();
  const size_t c = std::min<size_t>((size_t)count, buf.size());
  if (c) std::memcpy(out, buf.data(), c * sizeof(double));
  return SOS_OK;
}

int64_t sos_plan_tile(sos_plan_t p, int64_t n) {
  if (!p || n < 0) return 0;
  if (p->solver_opt == SOS_SCALAR)
    return p->tile_groups > 0 ? (int64_t)p->tile_groups * kScalarChunk : scalar_segment(*p, n);
  if (p->solver_opt == SOS_BLOCK) return block_tile(*p, n);
  if (wide_plan(*p)) return wide_tile(*p, n);
  return choose_tile(*p, n);
}

size_t sos_workspace_size(sos_plan_t p, int64_t n) {
  if (!p || n <= 0) return 0;
  if (wide_plan(*p)) return p->d_table ? wide_workspace(*p, n) : 0;
  return carry_layout(*p, n, choose_tile(*p, n)).bytes;
}

sos_status sos_filt(sos_plan_t p, const void *x, void *y, int64_t n, void *workspace,
                    sos_stream_t stream) {
  if (!p || n < 0) return SOS_E_ARG;
  if (n == 0) return SOS_OK;
  const sos_status chk = sosf::check_filt_args(*p, x, y, n);
  if (chk != SOS_OK) return chk;
  Ptrs q{x, y, p->d_table, static_cast<const int32_t *>(p->d_solver)};
  FiltArgs a;
  a.n = n;
  a.K = p->K;
  a.stride = p->stride;
  a.tile = choose_tile(*p, n);
  a.warm = p->warm;
  a.ntiles = (n + a.tile - 1) / a.tile;
  a.gain = p->gain;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool b0one = p->b0_factored;
  if (p->solver_opt == SOS_SCALAR) return launch_scalar(*p, x, y, n, s);
  if (p->solver_opt == SOS_BLOCK) return launch_block(*p, x, y, n, s);
  if (wide_plan(*p)) {
    // the lane runs of N = 256 .. 1024 live in the caller's workspace
    if (wide_workspace(*p, n) > 0 && (!workspace || ((uintptr_t)workspace & 15))) return SOS_E_ARG;
    return launch_wide(*p, x, y, n, workspace, s);
  }
  if (p->solver_opt == SOS_PH_DEFERRED) {
    if (p->io_dtype == SOS_F32) return launch_deferred<float>(p->N, q, p->d_coupling, p->d_theta, a, b0one, s);
    return launch_deferred<double>(p->N, q, p->d_coupling, p->d_theta, a, b0one, s);
  }
  // the exact inter-tile carry where the run-in would cost more than the
  // carry's second pass (it needs the caller's workspace)
  const CarryLayout cl = carry_layout(*p, n, a.tile);
  if (cl.use) {
    if (workspace && ((uintptr_t)workspace & 15) == 0) return launch_carry(*p, cl, x, y, n, workspace, s);
    if (p->flags & SOS_FLAG_CARRY_SCAN) return SOS_E_ARG;   // asked for, but no workspace
  }
  if (narrow_plan(*p)) return launch_narrow(*p, x, y, a, s);
  // one solver for every section lets the kernel drop the per-section branch
  return dispatch_rows_l<LaunchRows>(p->N, p->L, p->io_dtype, p->compute_dtype, b0one, solver_mix(*p), q, a, s);
}

}  // extern "C"
