// Block filtering (eq. block_filtering_equation) with the dense Toeplitz
// product on the matrix cores.
//
// A section maps each block of 16 samples by
//   y_n = H x_n + Gx xbar_{n-1} + Gy ybar_{n-1},
// H the 16 x 16 lower-triangular Toeplitz matrix of the first 16 impulse
// response samples, xbar and ybar the last two input and output samples of
// the previous block, Gx and Gy the block's responses to them (eq.
// block_filtering_matrices, with the minus sign of H_a folded into Gy).
//
// One wavefront filters one tile, 256 samples (16 blocks) at a time.  The
// 16 blocks are the 16 columns of one MFMA product H X, whose precision is
// the plan's product type: FP64 (16x16x4 FP64 MFMA), or FP16 / BF16 (16x16x16
// with FP32 accumulation).  Everything after the product is FP64:
// * the blocks' terminal outputs chain through the 2 x 2 recurrence
//   z_j = c_j + M z_{j-1} (M = the last two rows of Gy), solved along the 16
//   lanes of a DPP row by the same log-depth scan as the PH terminal block;
//   in the low-precision forms the two terminal rows of H x are recomputed
//   in FP64, so that no product rounding enters this recurrence;
// * the boundary correction Gx xbar + Gy ybar of every output (4 FMA per
//   sample, the paper's 4/L block FMAs);
// * the carries between groups and sections.
// The low-precision forms take one of two routes to the product, set by the
// number of slices S per operand:
// * S = 1: each section's input is scaled by a power of two (the inverse RMS
//   gain of the sections before it for white input) and rounded to the
//   product type, H is rounded to it, and the FP32 sum is scaled back in
//   FP64.  Its error is the product type's rounding.
// * S >= 2: error-free slicing of both operands (the splitting of Ozaki,
//   Ogita, Oishi and Rump, 2012, used on matrix units with FP16 inputs by
//   Mukunoki et al., 2020).  Each column of the tile (one block of 16
//   samples) is scaled by the power of two that puts its largest value
//   below 2^(W-1), W = 10 (FP16) or 8 (BF16), and cut into S integer slices
//   of W bits, v = sum_b t_b 2^(-W b) / s_v; H is cut the same way on the
//   host.  The integers are exact in the product type, their products are
//   exact in FP32, and the sums of each order a + b = o stay below 2^24, so
//   every FP32 accumulation of the matrix cores is exact.  The orders
//   a + b < S are summed in FP64.  The only errors left are the slices cut
//   off (2^(-W (S-1)) of the column's scale) and the products of order >= S.
#pragma once

#include "kernels_deferred.hpp"

namespace sosf {

typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

enum : int { PT_F64 = 0, PT_F16 = 1, PT_BF16 = 2 };

constexpr int kMaxSlices = 4;
// Bits per slice: a slice is an integer in [-2^(W-1), 2^(W-1)], exact in the
// product type (FP16 holds integers to 2^11, BF16 to 2^8).
template <int PT>
__host__ __device__ constexpr int slice_bits() { return PT == PT_F16 ? 10 : 8; }

// Per-section FP64 block table (kBlockStride doubles).
enum : int {
  BT_GXT = 0,      // 4: rows 14, 15 of Gx, row-major
  BT_POW = 4,      // 16: M^(2^i), i = 0..3, row-major
  BT_SCALE = 20,   // S = 1: input scale before rounding to the product type
  BT_ISCALE = 21,  // its inverse
  BT_HINV = 22,    // S >= 2: inverse of the power-of-two scale of H's slices
  BT_G = 32,       // 64: per lane row q and register r: Gx[m][0..1], Gy[m][0..1] (m per layout)
  BT_HT = 96,      // 32: per lane row q and register r: h[14 - m], h[15 - m] (0 past the diagonal)
  kBlockStride = 128
};
constexpr int kBlockGroup = 256;   // samples per MFMA (16 blocks of 16)
constexpr int kBlockKMax = 32;     // the tables of all sections sit in LDS

struct BlockArgs {
  int64_t n, tile, warm, ntiles;
  int32_t K;
  int32_t pad;
};

__device__ __forceinline__ short to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (short)(u >> 16);
}

// Row of the 16 x 16 tile held in register r of lane (q, j): the FP64 MFMA
// layout is m = q + 4 r, the FP32-accumulating 16x16x16 layout m = 4 q + r.
template <int PT>
__host__ __device__ constexpr int block_row(int q, int r) {
  return PT == PT_F64 ? q + 4 * r : 4 * q + r;
}

// Four consecutive samples (16-byte aligned) <-> four FP64 values.
__device__ __forceinline__ void load4(double (&V)[4], const float *p) {
  const vf4 v = __builtin_nontemporal_load(reinterpret_cast<const vf4 *>(p));
#pragma unroll
  for (int i = 0; i < 4; ++i) V[i] = (double)v[i];
}
__device__ __forceinline__ void load4(double (&V)[4], const double *p) {
  const vd2 u = __builtin_nontemporal_load(reinterpret_cast<const vd2 *>(p));
  const vd2 v = __builtin_nontemporal_load(reinterpret_cast<const vd2 *>(p) + 1);
  V[0] = u[0];
  V[1] = u[1];
  V[2] = v[0];
  V[3] = v[1];
}
__device__ __forceinline__ void store4(float *p, const double (&V)[4]) {
  vf4 v;
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = (float)V[i];
  __builtin_nontemporal_store(v, reinterpret_cast<vf4 *>(p));
}
__device__ __forceinline__ void store4(double *p, const double (&V)[4]) {
  const vd2 u = {V[0], V[1]}, v = {V[2], V[3]};
  __builtin_nontemporal_store(u, reinterpret_cast<vd2 *>(p));
  __builtin_nontemporal_store(v, reinterpret_cast<vd2 *>(p) + 1);
}

// Maximum over the four lanes of a tile column (lanes j, j + 16, j + 32,
// j + 48): permlane16 / permlane32 swaps exchange the rows pairwise.
__device__ __forceinline__ uint32_t column_max_u32(uint32_t v) {
  auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = a[0] > a[1] ? a[0] : a[1];
  auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return b[0] > b[1] ? b[0] : b[1];
}

// A slice of this lane's four scaled values (integers of at most W bits, so
// every conversion below is exact), in the product type.
template <int PT>
__device__ __forceinline__ v4s slice_bits_of(const double (&t)[4]) {
  float f[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) f[r] = (float)t[r];
  if (PT == PT_F16) {
    // two per instruction; round-toward-zero packing is exact for these
    typedef short v2s __attribute__((ext_vector_type(2)));
    const v2s lo = __builtin_bit_cast(v2s, __builtin_amdgcn_cvt_pkrtz(f[0], f[1]));
    const v2s hi = __builtin_bit_cast(v2s, __builtin_amdgcn_cvt_pkrtz(f[2], f[3]));
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3);
  }
  v4s o;
#pragma unroll
  for (int r = 0; r < 4; ++r) o[r] = (short)(__float_as_uint(f[r]) >> 16);   // its low 16 bits are zero
  return o;
}

// x16 product of one slice pair, or x32 product of two pairs (the K
// dimension of a 16x16x32 product is any sum of two 16-deep products).
template <int PT>
__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f acc) {
  if (PT == PT_F16)
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(v4h, a), __builtin_bit_cast(v4h, b), acc, 0, 0,
                                                 0);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
}
template <int PT>
__device__ __forceinline__ v4f mfma32(v4s a0, v4s a1, v4s b0, v4s b1, v4f acc) {
  const v8s a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
  const v8s b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
  if (PT == PT_F16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b), acc, 0, 0,
                                                  0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), acc, 0,
                                                 0, 0);
}

// The product H V of one section with S >= 2 slices per operand (see the
// top of this file).  Aop: this lane's entry of the section's first slice of
// H in the 16x16x16 A layout (lane (q, i) holds H-slice[i][4q .. 4q+3]);
// slice a lies 64 entries (one per lane) after slice a - 1.  V: this lane's
// four values (rows 4q + r of column j); hinv: the inverse of H's slice
// scale.
template <int PT, int S>
__device__ __forceinline__ void sliced_product(const v4s *__restrict__ Aop, const double (&V)[4], double hinv,
                                               double (&P)[4]) {
  v4s A[S];
#pragma unroll
  for (int a = 0; a < S; ++a) A[a] = Aop[64 * a];
  constexpr int W = slice_bits<PT>();
  // the column's largest magnitude, by the high words (sign cleared)
  uint32_t mx = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t h = (uint32_t)((uint64_t)__double_as_longlong(V[r]) >> 32) & 0x7fffffffu;
    mx = h > mx ? h : mx;
  }
  mx = column_max_u32(mx);
  // biased exponent eb: every |v| of the column is below 2^(eb - 1022), so
  // v 2^(W + 1021 - eb) lies in (-2^(W-1), 2^(W-1))
  const int eb = (int)(mx >> 20);
  const double sv = __longlong_as_double((long long)((uint64_t)(W + 2044 - eb) << 52));
  v4s t[S];
  {
    double u[4], tb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) u[r] = V[r] * sv;
#pragma unroll
    for (int b = 0; b < S; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        tb[r] = __builtin_rint(u[r]);
        if (b + 1 < S) u[r] = (u[r] - tb[r]) * (double)(1 << W);   // both steps exact
      }
      t[b] = slice_bits_of<PT>(tb);
    }
  }
  // orders o = a + b (a: slice of H, b: slice of V), each in its own exact
  // FP32 accumulator; pairs two at a time on 16x16x32, a leftover on x16
  v4f acc[S];
#pragma unroll
  for (int o = 0; o < S; ++o) {
    v4f c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a + 1 <= o; a += 2) c = mfma32<PT>(A[a], A[a + 1], t[o - a], t[o - a - 1], c);
    if ((o & 1) == 0) c = mfma16<PT>(A[o], t[0], c);
    acc[o] = c;
  }
  const double inv = __builtin_ldexp(hinv, eb - 1021 - W);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double sum = (double)acc[S - 1][r];
#pragma unroll
    for (int o = S - 2; o >= 0; --o) sum = fma_(sum, 1.0 / (double)(1 << W), (double)acc[o][r]);
    P[r] = sum * inv;
  }
}

// One wavefront's tile: samples [t0, t0 + tile) of a signal of n samples,
// after a run-in over the warm samples before t0 (samples outside [0, n)
// read as zero and are not stored).  g_s, a_s: the sections' correction
// rows and MFMA A operands in LDS; st: the wavefront's 2 + 2K carries (the
// raw input's last two samples, then each section's last two outputs).
template <typename TI, int PT, int S>
__device__ __forceinline__ void block_rows(const TI *__restrict__ x, TI *__restrict__ y, const double *__restrict__ bt,
                                           const double *g_s, const unsigned char *a_s, double *st, int64_t n,
                                           int64_t t0, int64_t tile, int64_t warm, int K) {
  typedef double T;
  const int lane = lane_id(), q = lane >> 4, j = lane & 15;
  for (int i = 0; i < 2 + 2 * K; ++i) st[i] = T(0);
  const ctab<T> cb = as_ctab(bt);
  const int64_t steps = (warm + tile) / kBlockGroup;
  const int src_prev = 48 + ((j + 15) & 15);   // lane (3, j - 1)
  for (int64_t it = 0; it < steps; ++it) {
    const int64_t g = t0 - warm + it * kBlockGroup;
    const int64_t e0 = g + 16 * j + 4 * q;   // this lane's 4 consecutive samples
    T V[4];
    if (e0 >= 0 && e0 + 4 <= n) {
      load4(V, x + e0);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) V[i] = (e0 + i >= 0 && e0 + i < n) ? T(x[e0 + i]) : T(0);
    }
    // the raw input's two samples before block j: lane (3, j - 1), or the carry
    T xb2 = __shfl(V[2], src_prev), xb1 = __shfl(V[3], src_prev);
    if (j == 0) {
      xb2 = st[0];
      xb1 = st[1];
    }
    const T nraw2 = __shfl(V[2], 63), nraw1 = __shfl(V[3], 63);
    if (PT == PT_F64) row_transpose4(V);   // to the FP64 MFMA layout, m = q + 4 r
    for (int k = 0; k < K; ++k) {
      const ctab<T> c = cb + (int64_t)k * kBlockStride;
      T P[4];
      if (PT == PT_F64) {
        const double *A = reinterpret_cast<const double *>(a_s) + k * 256;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[s * 64 + lane], V[s], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) P[r] = acc[r];
      } else if (S >= 2) {
        sliced_product<PT, S>(reinterpret_cast<const v4s *>(a_s) + (size_t)k * S * 64 + lane, V, c[BT_HINV], P);
      } else {
        const T sc = c[BT_SCALE], isc = c[BT_ISCALE];
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        if (PT == PT_F16) {
          const v4h A = reinterpret_cast<const v4h *>(a_s)[k * 64 + lane];
          v4h B;
#pragma unroll
          // the power-of-two scale in FP32 is exact; scaling there keeps the
          // conversion to FP16 one hardware step from FP32 (from FP64 the
          // compiler would emulate it)
          for (int r = 0; r < 4; ++r) B[r] = (_Float16)((float)V[r] * (float)sc);
          acc = __builtin_amdgcn_mfma_f32_16x16x16f16(A, B, acc, 0, 0, 0);
        } else {
          const v4s A = reinterpret_cast<const v4s *>(a_s)[k * 64 + lane];
          v4s B;
#pragma unroll
          for (int r = 0; r < 4; ++r) B[r] = to_bf16((float)(V[r] * sc));
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) P[r] = T(acc[r]) * isc;
      }
      // terminal outputs (rows 14, 15) of block j, in every lane of column j.
      // The low-precision forms recompute them in FP64 (two rows of H, over
      // the four lanes of the column): the block-to-block recurrence then
      // carries no product rounding.
      T p14, p15;
      if (PT == PT_F64) {
        p14 = __shfl(P[3], 32 + j);
        p15 = __shfl(P[3], 48 + j);
      } else {
        const double *ht = g_s + k * 96 + 64 + q * 8;
        T s14 = T(0), s15 = T(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          s14 = fma_(ht[2 * r], V[r], s14);
          s15 = fma_(ht[2 * r + 1], V[r], s15);
        }
        s14 += __shfl_xor(s14, 16);
        s15 += __shfl_xor(s15, 16);
        s14 += __shfl_xor(s14, 32);
        s15 += __shfl_xor(s15, 32);
        p14 = s14;
        p15 = s15;
        // the outputs of rows 14 and 15 themselves come from the FP64 values
        if (q == 3) {
          P[2] = s14;
          P[3] = s15;
        }
      }
      T c0 = fma_(c[BT_GXT + 1], xb1, fma_(c[BT_GXT + 0], xb2, p14));
      T c1 = fma_(c[BT_GXT + 3], xb1, fma_(c[BT_GXT + 2], xb2, p15));
      const T yp2 = st[2 + 2 * k], yp1 = st[3 + 2 * k];
      if (j == 0) {
        c0 = fma_(c[BT_POW + 1], yp1, fma_(c[BT_POW + 0], yp2, c0));
        c1 = fma_(c[BT_POW + 3], yp1, fma_(c[BT_POW + 2], yp2, c1));
      }
      row_scan_2x2(c0, c1, c + BT_POW);    // z_j: the true last two outputs of block j
      const T yb2 = shift_r(c0, yp2), yb1 = shift_r(c1, yp1);
      const double *G = g_s + k * 96 + q * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        V[r] = fma_(G[4 * r + 3], yb1, fma_(G[4 * r + 2], yb2, fma_(G[4 * r + 1], xb1, fma_(G[4 * r], xb2, P[r]))));
      st[2 + 2 * k] = last_of_row(c0);
      st[3 + 2 * k] = last_of_row(c1);
      // the next section's input before block j is this section's output there
      xb2 = yb2;
      xb1 = yb1;
    }
    st[0] = nraw2;
    st[1] = nraw1;
    if (g >= t0) {
      if (PT == PT_F64) row_transpose4(V);   // back to 4 consecutive samples per lane
      if (e0 >= 0 && e0 + 4 <= n) {
        store4(y + e0, V);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (e0 + i >= 0 && e0 + i < n) y[e0 + i] = (TI)V[i];
      }
    }
  }
}

// A-operand bytes per section: one 16 x 16 tile of H (FP64), or S slices of
// it in the product type.
__host__ __device__ constexpr int block_aop_bytes(int pt, int S) {
  return pt == PT_F64 ? 256 * 8 : 256 * 2 * S;
}

// Stage the correction rows and A operands of K sections into LDS.
template <int PT, int S>
__device__ __forceinline__ void block_stage_tables(const double *__restrict__ bt, const void *__restrict__ aop, int K,
                                                   double *g_s, unsigned char *a_s) {
  constexpr int AOP = block_aop_bytes(PT, S);
  for (int i = threadIdx.x; i < K * 96; i += kWavesPerBlock * 64)
    g_s[i] = bt[(int64_t)(i / 96) * kBlockStride + BT_G + (i % 96)];
  for (int i = threadIdx.x; i < K * AOP / 16; i += kWavesPerBlock * 64)
    reinterpret_cast<vf4 *>(a_s)[i] = reinterpret_cast<const vf4 *>(aop)[i];
}

// Single signal: wavefront w takes tile w.
template <typename TI, int PT, int S>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_block_kernel(
    const TI *__restrict__ x, TI *__restrict__ y, const double *__restrict__ bt,
    const void *__restrict__ aop, BlockArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  // LDS: the block's copies of the per-lane correction rows and of the MFMA
  // A operands (every wavefront reads all of them once per group), then the
  // carries of each wavefront
  constexpr int AOP = block_aop_bytes(PT, S);
  double *g_s = reinterpret_cast<double *>(smem);   // per section: G (64), then HT (32)
  unsigned char *a_s = smem + (size_t)a.K * 96 * sizeof(double);
  block_stage_tables<PT, S>(bt, aop, a.K, g_s, a_s);
  __syncthreads();
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wave >= a.ntiles) return;
  double *st = reinterpret_cast<double *>(a_s + (size_t)a.K * AOP) + w * (2 + 2 * a.K);
  block_rows<TI, PT, S>(x, y, bt, g_s, a_s, st, a.n, wave * a.tile, a.tile, a.warm, a.K);
}

// Batches: one workgroup per work item, four tiles of one channel (one per
// wavefront), so that the workgroup stages that channel's tables only.  The
// channel's tiles cover [-shift, n), which puts every 4-sample vector of x
// and y on a 16-byte boundary.
// hdr[0]: the live item count (the grid is sized for the batch's room).
template <typename TI, int PT, int S>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_block_batched_kernel(
    const TI *__restrict__ x, TI *__restrict__ y, const BatchChan *__restrict__ chans,
    const int32_t *__restrict__ item_chan, const int64_t *__restrict__ hdr, int32_t kmax) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int AOP = block_aop_bytes(PT, S);
  if ((int64_t)blockIdx.x >= hdr[0]) return;   // uniform per workgroup
  const BatchChan &ch = chans[item_chan[blockIdx.x]];
  double *g_s = reinterpret_cast<double *>(smem);
  unsigned char *a_s = smem + (size_t)kmax * 96 * sizeof(double);
  block_stage_tables<PT, S>(static_cast<const double *>(ch.tab), ch.aop, ch.K, g_s, a_s);
  __syncthreads();
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t tile_index = ((int64_t)blockIdx.x - ch.first_item) * kWavesPerBlock + w;
  if (tile_index * ch.tile >= ch.n + ch.shift) return;
  double *st = reinterpret_cast<double *>(a_s + (size_t)kmax * AOP) + w * (2 + 2 * kmax);
  block_rows<TI, PT, S>(x + ch.off, y + ch.off, static_cast<const double *>(ch.tab), g_s, a_s, st, ch.n,
                     tile_index * ch.tile - ch.shift, ch.tile, ch.warm, ch.K);
}

}  // namespace sosf
