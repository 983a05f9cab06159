// Block filtering plans (solver SOS_BLOCK): the FP64 block tables, the MFMA
// A operands of the Toeplitz products, and the launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dispatch.hpp"
#include "kernels_block.hpp"
#include "plan.hpp"
#include "batch.hpp"

using namespace sosf;

namespace {

// Responses of one section over a block of 16 samples, by running its
// recurrence (eq. general_cascaded_equation with the rows divided by a0):
// h (input impulse), gx[c] (unit x[-2] or x[-1]), gy[c] (unit y[-2] or y[-1]).
void block_responses(const double *r, double h[16], double gx[2][16], double gy[2][16]) {
  const double b0 = r[0], b1 = r[1], b2 = r[2], a1 = r[3], a2 = r[4];
  auto run = [&](const double xin[16], double xm2, double xm1, double ym2, double ym1, double out[16]) {
    double x2 = xm2, x1 = xm1, y2 = ym2, y1 = ym1;
    for (int m = 0; m < 16; ++m) {
      const double v = b0 * xin[m] + b1 * x1 + b2 * x2 - a1 * y1 - a2 * y2;
      x2 = x1;
      x1 = xin[m];
      y2 = y1;
      y1 = v;
      out[m] = v;
    }
  };
  double imp[16] = {1.0}, zero[16] = {0.0};
  run(imp, 0, 0, 0, 0, h);
  run(zero, 1, 0, 0, 0, gx[0]);
  run(zero, 0, 1, 0, 0, gx[1]);
  run(zero, 0, 0, 1, 0, gy[0]);
  run(zero, 0, 0, 0, 1, gy[1]);
}

// White-noise RMS gain of the first k sections (k = 0..K-1), from their
// impulse response run until it has decayed below 1e-30 of its peak.
std::vector<double> prefix_rms_gain(const sos_plan_s &p) {
  std::vector<double> g(p.K, 1.0);
  const int64_t len = std::max<int64_t>(4 * p.warm, 4096);
  std::vector<double> sig(len, 0.0);
  sig[0] = 1.0;
  for (int k = 0; k + 1 < p.K; ++k) {
    const double *r = &p.rows_norm[5 * k];
    double x2 = 0, x1 = 0, y2 = 0, y1 = 0;
    double e = 0;
    for (int64_t i = 0; i < len; ++i) {
      const double v = r[0] * sig[i] + r[1] * x1 + r[2] * x2 - r[3] * y1 - r[4] * y2;
      x2 = x1;
      x1 = sig[i];
      y2 = y1;
      y1 = v;
      sig[i] = v;
      e += v * v;
    }
    g[k + 1] = std::sqrt(e);
  }
  return g;
}

uint16_t bf16_bits(double d) {
  float f = (float)d;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

uint16_t f16_bits(double d) {
  const _Float16 h = (_Float16)(float)d;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

template <int PT>
void fill_rows(const double gx[2][16], const double gy[2][16], double *t) {
  for (int q = 0; q < 4; ++q)
    for (int r = 0; r < 4; ++r) {
      const int m = block_row<PT>(q, r);
      double *o = t + BT_G + q * 16 + 4 * r;
      o[0] = gx[0][m];
      o[1] = gx[1][m];
      o[2] = gy[0][m];
      o[3] = gy[1][m];
    }
}

// Kernel instances by I/O type, product type and slices per operand.
template <template <typename, int, int> class KP, typename TI, int PT>
const void *by_slices(int S) {
  switch (S) {
    case 2: return KP<TI, PT, 2>::get();
    case 3: return KP<TI, PT, 3>::get();
    case 4: return KP<TI, PT, 4>::get();
    default: return KP<TI, PT, 1>::get();
  }
}
template <template <typename, int, int> class KP>
const void *block_instance(int io_dtype, int pt, int S) {
  const bool f32 = io_dtype == SOS_F32;
  switch (pt) {
    case PT_F16: return f32 ? by_slices<KP, float, PT_F16>(S) : by_slices<KP, double, PT_F16>(S);
    case PT_BF16: return f32 ? by_slices<KP, float, PT_BF16>(S) : by_slices<KP, double, PT_BF16>(S);
    default: return f32 ? KP<float, PT_F64, 1>::get() : KP<double, PT_F64, 1>::get();
  }
}
template <typename TI, int PT, int S>
struct SingleKernel {
  static const void *get() { return reinterpret_cast<const void *>(&sos_block_kernel<TI, PT, S>); }
};

const void *block_kernel(const sos_plan_s &p) {
  return block_instance<SingleKernel>(p.io_dtype, p.block_pt, p.block_slices);
}

size_t block_lds(const sos_plan_s &p) {
  const size_t aop = (size_t)block_aop_bytes(p.block_pt, p.block_slices);
  return (size_t)p.K * (96 * sizeof(double) + aop) + (size_t)kWavesPerBlock * (2 + 2 * p.K) * sizeof(double);
}

// Integer slices of u (|u| < 2^(W-1)): u = sum_b t_b 2^(-W b) + a remainder
// below 2^(-W (S-1)) / 2; every step is exact in FP64.
void slice(double u, int S, int W, double *t) {
  for (int b = 0; b < S; ++b) {
    t[b] = std::nearbyint(u);
    u = (u - t[b]) * std::ldexp(1.0, W);
  }
}

}  // namespace

namespace sosf {

sos_status build_block_plan(sos_plan_s &p) {
  p.block_pt = p.compute_dtype == SOS_F16 ? PT_F16 : (p.compute_dtype == SOS_BF16 ? PT_BF16 : PT_F64);
  const int S = p.block_slices;
  const int W = p.block_pt == PT_F16 ? slice_bits<PT_F16>() : slice_bits<PT_BF16>();
  p.block_tab.assign((size_t)p.K * kBlockStride, 0.0);
  const size_t aop_bytes = (size_t)block_aop_bytes(p.block_pt, S);
  p.block_aop.assign((size_t)p.K * aop_bytes, 0);
  const std::vector<double> gain = prefix_rms_gain(p);
  for (int k = 0; k < p.K; ++k) {
    double h[16], gx[2][16], gy[2][16];
    block_responses(&p.rows_norm[5 * k], h, gx, gy);
    double *t = &p.block_tab[(size_t)k * kBlockStride];
    t[BT_GXT + 0] = gx[0][14];
    t[BT_GXT + 1] = gx[1][14];
    t[BT_GXT + 2] = gx[0][15];
    t[BT_GXT + 3] = gx[1][15];
    // M = the last two rows of Gy; its powers for the row scan
    double M[4] = {gy[0][14], gy[1][14], gy[0][15], gy[1][15]};
    for (int i = 0; i < 4; ++i) {
      std::memcpy(t + BT_POW + 4 * i, M, sizeof(M));
      const double n0 = M[0] * M[0] + M[1] * M[2], n1 = M[0] * M[1] + M[1] * M[3];
      const double n2 = M[2] * M[0] + M[3] * M[2], n3 = M[2] * M[1] + M[3] * M[3];
      M[0] = n0;
      M[1] = n1;
      M[2] = n2;
      M[3] = n3;
    }
    // inputs of the low-precision products at about unit RMS for white input
    const double sc = p.block_pt == PT_F64 ? 1.0 : std::ldexp(1.0, -(int)std::lround(std::log2(gain[k])));
    t[BT_SCALE] = sc;
    t[BT_ISCALE] = 1.0 / sc;
    if (p.block_pt == PT_F64) fill_rows<PT_F64>(gx, gy, t);
    else fill_rows<PT_F16>(gx, gy, t);   // the 16x16x16 layout serves FP16 and BF16
    // rows 14 and 15 of H per lane row q and register r (16x16x16 layout)
    for (int q = 0; q < 4; ++q)
      for (int r = 0; r < 4; ++r) {
        const int c = block_row<PT_F16>(q, r);
        t[BT_HT + q * 8 + 2 * r] = c <= 14 ? h[14 - c] : 0.0;
        t[BT_HT + q * 8 + 2 * r + 1] = h[15 - c];
      }
    // S >= 2: H in slices, scaled by the power of two that puts max |h|
    // below 2^(W-1) (the same rule as the kernel's columns)
    double hmax = 0.0;
    for (int i = 0; i < 16; ++i) hmax = std::max(hmax, std::fabs(h[i]));
    int eh = 0;
    std::frexp(hmax, &eh);   // hmax < 2^eh
    const double sh = std::ldexp(1.0, W - 1 - eh);
    t[BT_HINV] = 1.0 / sh;
    // A operands of H (H[m][c] = h[m - c] for c <= m)
    unsigned char *ao = p.block_aop.data() + (size_t)k * aop_bytes;
    for (int l = 0; l < 64; ++l) {
      const int m = l % 16;
      if (p.block_pt != PT_F64 && S >= 2) {
        // slice a of H[m][4 (l / 16) + i] at ((a * 64 + l) * 4 + i) halves
        for (int i = 0; i < 4; ++i) {
          const int c = 4 * (l / 16) + i;
          double ts[kMaxSlices];
          slice(c <= m ? h[m - c] * sh : 0.0, S, W, ts);
          for (int a = 0; a < S; ++a) {
            const uint16_t b = p.block_pt == PT_F16 ? f16_bits(ts[a]) : bf16_bits(ts[a]);
            std::memcpy(ao + ((size_t)(a * 64 + l) * 4 + i) * 2, &b, 2);
          }
        }
      } else if (p.block_pt == PT_F64) {
        for (int s = 0; s < 4; ++s) {
          const int c = 4 * s + l / 16;
          const double v = c <= m ? h[m - c] : 0.0;
          std::memcpy(ao + (size_t)(s * 64 + l) * sizeof(double), &v, sizeof(double));
        }
      } else {
        for (int i = 0; i < 4; ++i) {
          const int c = 4 * (l / 16) + i;
          const double v = c <= m ? h[m - c] : 0.0;
          const uint16_t b = p.block_pt == PT_F16 ? f16_bits(v) : bf16_bits(v);
          std::memcpy(ao + (size_t)(l * 4 + i) * 2, &b, 2);
        }
      }
    }
  }
  p.warm = (p.warm + kBlockGroup - 1) / kBlockGroup * kBlockGroup;
  return SOS_OK;
}

sos_status upload_block_plan(sos_plan_s &p) {
  const size_t tb = p.block_tab.size() * sizeof(double), ab = p.block_aop.size();
  if (hipMalloc(&p.d_block, tb) != hipSuccess) {
    p.d_block = nullptr;
    return SOS_E_NOMEM;
  }
  if (hipMalloc(&p.d_aop, ab) != hipSuccess) {
    p.d_aop = nullptr;
    return SOS_E_NOMEM;
  }
  if (hipMemcpy(p.d_block, p.block_tab.data(), tb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p.d_aop, p.block_aop.data(), ab, hipMemcpyHostToDevice) != hipSuccess)
    return SOS_E_DEVICE;
  Residency r = residency_of(block_kernel(p), block_lds(p), kWavesPerBlock * 64);
  p.simds = r.simds;
  p.waves_per_simd = r.waves_per_simd;
  return SOS_OK;
}

// One tile per wavefront; every SIMD gets m wavefronts, m as in
// model_tile_groups.
int64_t block_tile(const sos_plan_s &p, int64_t n) {
  if (p.tile_groups > 0) return (int64_t)p.tile_groups * kBlockGroup;
  int64_t m = 1;
  while (2 * m <= p.waves_per_simd) m *= 2;
  const int64_t waves = (int64_t)p.simds * m;
  const int64_t t = (n + waves - 1) / waves;
  return std::max<int64_t>((t + kBlockGroup - 1) / kBlockGroup * kBlockGroup, kBlockGroup);
}

sos_status launch_block(const sos_plan_s &p, const void *x, void *y, int64_t n, hipStream_t s) {
  BlockArgs a;
  a.n = n;
  a.tile = block_tile(p, n);
  a.warm = p.warm;
  a.ntiles = (n + a.tile - 1) / a.tile;
  a.K = p.K;
  a.pad = 0;
  const int64_t blocks = (a.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  const void *xa = x, *ta = p.d_block, *aa = p.d_aop;
  void *ya = y;
  void *args[] = {&xa, &ya, &ta, &aa, &a};   // addresses of the kernel's five arguments
  if (hipLaunchKernel(block_kernel(p), dim3((unsigned)blocks), dim3(kWavesPerBlock * 64), args, block_lds(p), s) !=
      hipSuccess)
    return SOS_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
}

// Batches of block-filtering channels (sosfilt_batch.hip schedules them):
// one workgroup per item of four tiles, the channel's tables in LDS.
namespace {
template <typename TI, int PT, int S>
struct BatchedKernel {
  static const void *get() { return reinterpret_cast<const void *>(&sos_block_batched_kernel<TI, PT, S>); }
};
size_t block_batched_lds(int kmax, int pt, int S) {
  const size_t aop = (size_t)block_aop_bytes(pt, S);
  return (size_t)kmax * (96 * sizeof(double) + aop) + (size_t)kWavesPerBlock * (2 + 2 * kmax) * sizeof(double);
}
}  // namespace

Residency block_batched_residency(int io_dtype, int pt, int S, int kmax) {
  return residency_of(block_instance<BatchedKernel>(io_dtype, pt, S), block_batched_lds(kmax, pt, S),
                      kWavesPerBlock * 64);
}

sos_status launch_block_batched(const sos_batch_s &b, const void *x, void *y, hipStream_t s) {
  const void *xa = x, *ca = b.d_chans, *ia = b.d_item_chan, *ha = b.d_hdr;
  void *ya = y;
  int32_t kmax = b.kmax_cap;
  void *args[] = {&xa, &ya, &ca, &ia, &ha, &kmax};   // addresses of the kernel's six arguments
  if (hipLaunchKernel(block_instance<BatchedKernel>(b.io_dtype, b.block_pt, b.block_slices),
                      dim3((unsigned)b.items_cap), dim3(kWavesPerBlock * 64), args,
                      block_batched_lds(b.kmax_cap, b.block_pt, b.block_slices), s) != hipSuccess)
    return SOS_E_DEVICE;
  return hipGetLastError() == hipSuccess ? SOS_OK : SOS_E_DEVICE;
}

}  // namespace sosf
