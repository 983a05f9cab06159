// Wide groups (N = 128 .. 1024, runs in the workspace) by the
// deferred-correction PH of kernels_deferred.hpp.
//
// The per-section PH of kernels_wide.hpp reads and writes a lane's run once
// per section (16 bytes per sample and section).  Deferring the homogeneous
// corrections to the end of the cascade takes every section over the run in
// one pass instead:
//  1. each lane runs the whole cascade from zero state over its run (only
//     the raw input keeps its true history), 64 blocks at a time in
//     registers, sections one after the other on the chunk with their
//     zero-state histories carried in registers, and writes the last
//     section's zero-state output to the workspace;
//  2. the sections' true terminal values follow from their zero-state ones
//     by the per-lane coupling to the sections before them and the row scan
//     (deferred_terminal), which leaves every lane's entry state RS;
//  3. the output is that zero-state output plus Theta RS (the cascade's
//     response at each block to each entry component), a product with inner
//     dimension 2K on FP64 16x16x4 MFMA, as for N <= 64, with Theta read
//     from the plan's device table.
// The workspace then carries 16 bytes per sample in all, whatever K, less
// the run's last chunk of 64 blocks, which stays in registers from the
// first pass to the second (and nothing in the run-in groups).
#pragma once

#include "kernels_deferred.hpp"
#include "kernels_wide.hpp"

namespace sosf {

// LDS: as the wide kernels (staging, then per-row states of 2 + 2K
// doubles).  Between the zero-state pass and the correction a wavefront's
// staging region holds its entry-state responses RS (2K x 64 doubles,
// component-major; 16 KB at K = 16, within the four rows' staging of either
// I/O type); the correction reads its share of them into registers first.
template <typename TI>
__host__ __device__ constexpr int wide_deferred_lds_bytes(int K) {
  return lds_bytes<kWideChunk, TI, double>(K);
}
static_assert(2 * 16 * 64 * 8 <= kRows * Stage<kWideChunk, float>::ROWBUF * 4, "RS fits a wavefront's staging");

// KBM: the plan's 4-wide state blocks (ceil(2K / 4) <= KBM, Theta padded to
// KBM); the zero-state histories of up to 2 KBM sections stay in registers.
template <typename TI, bool B0ONE, int KBM>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_wide_deferred_kernel(
    const TI *__restrict__ x, TI *__restrict__ y, const double *__restrict__ tab,
    const double *__restrict__ coup, const double *__restrict__ theta, WideArgs a) {
  typedef double T;
  constexpr int KMAX = 2 * KBM;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int K = a.K, D = 2 * K, N = a.N;
  TI *stage = reinterpret_cast<TI *>(smem);
  T *state = reinterpret_cast<T *>(smem + stage_bytes<kWideChunk, TI>());
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wave * kRows >= a.ntiles) return;   // uniform per wave
  const int lane = lane_id(), row = lane >> 4, rl = lane & 15, q = lane >> 4;
  const int64_t t0 = (wave * kRows + row) * a.tile;
  // per-row state: st[0..1] the raw input (x[-2], x[-1]); st[2+2k..] section
  // k's entry state (y_k[-2], y_k[-1])
  T *st = state + (int64_t)(w * kRows + row) * state_elems(K);
  // rs[comp * 64 + lane], over the wavefront's staging (see above)
  T *rs = reinterpret_cast<T *>(stage + w * kRows * Stage<kWideChunk, TI>::ROWBUF);
  TI *buf = stage + (w * kRows + row) * Stage<kWideChunk, TI>::ROWBUF;
  T *S = a.ws + (size_t)wave * N * 64 + lane;
  const ctab<T> ct = as_ctab(tab);
  for (int i = 0; i < state_elems(K); ++i) st[i] = T(0);   // the row's lanes write the same value
  const int64_t G = (int64_t)N * kL;
  const int64_t warm_groups = a.warm / G, steps = warm_groups + a.tile / G;
  for (int64_t it = 0; it < steps; ++it) {
    const int64_t g = t0 - a.warm + it * G;
    const bool full = __builtin_amdgcn_ballot_w64(!(g >= 0 && g + G <= a.n)) == 0;
    // step 1: the zero-state cascade over the lane's run.  Histories
    // (input, output) per section; the raw input's is true: the two samples
    // before the lane's run (lane 0: the previous group's last two)
    T xh1[KMAX], xh2[KMAX], yh1[KMAX], yh2[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) xh1[k] = xh2[k] = yh1[k] = yh2[k] = T(0);
    {
      const int64_t i1 = g + (int64_t)rl * N - 1, i2 = i1 - 1;
      const T v1 = (rl > 0 && i1 >= 0 && i1 < a.n) ? (T)x[i1] : T(0);
      const T v2 = (rl > 0 && i2 >= 0 && i2 < a.n) ? (T)x[i2] : T(0);
      xh1[0] = rl == 0 ? st[1] : v1;
      xh2[0] = rl == 0 ? st[0] : v2;
      const int64_t e = g + (int64_t)kL * N;
      st[0] = (e - 2 >= 0 && e - 2 < a.n) ? (T)x[e - 2] : T(0);
      st[1] = (e - 1 >= 0 && e - 1 < a.n) ? (T)x[e - 1] : T(0);
    }
    const bool live = it >= warm_groups;   // uniform per wave
    const int NC = N / kWideChunk;
    T X[kWideChunk];   // after the pass: the last chunk's zero-state output
    for (int cc = 0; cc < NC; ++cc) {
      wide_load_chunk<TI>(X, x, g, N, cc, a.n, full, buf);
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k >= K) break;   // uniform
        const ctab<T> c = ct + (int64_t)k * a.stride;
        const T b0 = c[OFF_B0], b1 = c[OFF_B1], b2 = c[OFF_B2], a1 = c[OFF_A1], a2 = c[OFF_A2];
        T p1 = xh1[k], p2 = xh2[k], w1 = yh1[k], w2 = yh2[k];
#pragma unroll
        for (int j = 0; j < kWideChunk; ++j) {
          const T xin = X[j];
          T v = B0ONE ? xin : b0 * xin;
          v = fma_(b1, p1, v);
          v = fma_(b2, p2, v);
          v = fma_(-a2, w2, v);
          v = fma_(-a1, w1, v);
          X[j] = v;
          p2 = p1;
          p1 = xin;
          w2 = w1;
          w1 = v;
        }
        xh1[k] = p1;
        xh2[k] = p2;
        yh1[k] = w1;
        yh2[k] = w2;
      }
      // the correction pass reads the zero-state output back, except the
      // last chunk's, which stays in registers; the run-in needs none
      if (live && cc + 1 < NC) {
#pragma unroll
        for (int j = 0; j < kWideChunk; ++j) S[64 * (cc * kWideChunk + j)] = X[j];
      }
    }
    // step 2: true terminal values, section by section; RS and the exit
    // state (the next group's entry) from them
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k >= K) break;
      deferred_terminal(yh2[k], yh1[k], ct + (int64_t)k * a.stride, coup + 2 * k * (k - 1), rs, st, k, D);
    }
    __builtin_amdgcn_wave_barrier();
    if (!live) continue;   // the run-in needs only the exit state
    // step 3: Y = W_K + Theta RS, one 16x16 tile per (row, 16 blocks).  The
    // B operands (RS_r[4b + q][rl]) go to registers before the staging
    // region that holds RS is used for the output again
    T bv[KBM][kRows];
#pragma unroll
    for (int b = 0; b < KBM; ++b) {
      const int comp = 4 * b + q;
      const int cidx = comp < D ? comp : D - 1;
#pragma unroll
      for (int r = 0; r < kRows; ++r) bv[b][r] = comp < D ? rs[cidx * 64 + 16 * r + rl] : T(0);
    }
    __builtin_amdgcn_wave_barrier();
    // the last chunk first, from the registers, then the others from the
    // workspace
    for (int ci0 = 0; ci0 < NC; ++ci0) {
      const int cc = ci0 == 0 ? NC - 1 : ci0 - 1;
      if (ci0 > 0) {
#pragma unroll
        for (int j = 0; j < kWideChunk; ++j) X[j] = S[64 * (cc * kWideChunk + j)];
      }
#pragma unroll
      for (int mb = 0; mb < kWideChunk / 16; ++mb) {
        const int64_t mg = (int64_t)cc * (kWideChunk / 16) + mb;   // 16-block of the run
        v4d acc[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) acc[r] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < KBM; ++b) {
          const T av = theta[(mg * KBM + b) * 64 + lane];   // Theta[16 mg + rl][4b + q]
#pragma unroll
          for (int r = 0; r < kRows; ++r)
            acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[b][r], acc[r], 0, 0, 0);
        }
        // acc[r] register i, row q': correction of row r's block
        // 16 mb + q' + 4 i; transposed so that each row holds its own
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          T V[kRows];
#pragma unroll
          for (int r = 0; r < kRows; ++r) V[r] = acc[r][i];
          row_transpose4(V);
#pragma unroll
          for (int ci = 0; ci < 4; ++ci) X[16 * mb + ci + 4 * i] += V[ci];
        }
      }
      wide_store_chunk<TI>(X, y, g, N, cc, a.n, full, a.gain, buf);
    }
  }
}

}  // namespace sosf
