// PH factorisation with the homogeneous correction deferred to the end of
// the cascade and applied on the matrix cores (FP64 arithmetic).
//
// Per group and row (layout as in kernels.hpp), each lane runs every section
// from zero state over its own N samples: the particular solution of Section
// VI-B step 1, taken through the whole cascade.  Only the raw input keeps its
// true history.  By linearity the true output is that zero-state output plus
// the response to the segment's entry state, the 2K values
// (y_j[-2], y_j[-1]) that every section j carries into the segment.
//
// * Terminal blocks (Section VI-B step 2, generalised to the cascade): the
//   true terminal values S_k[l] = (y_k[(l+1)N-2], y_k[(l+1)N-1]) of section
//   k on lane l satisfy
//     S_k[l] = w_e,k[l] + sum_{j<k} Psi_jk S_j[l-1] + Psi_kk S_k[l-1],
//   with Psi_kk = -C of eq. C.  Sections are taken in order: the coupling to
//   the already solved sections j < k is a per-lane 2x2 update, then the
//   row scan of eq. recursive_doubling_equation solves section k.  The
//   group's entry state (the previous group's exit state) enters lane 0.
// * Homogeneous correction (step 3, eq. PH_forward, for all sections at
//   once): Y = W_K + Theta RS, where RS holds every section's S shifted one
//   lane down (R, with the entry state in lane 0) and Theta (N x 2K) is the
//   cascade's response at each block to each entry component.  That is a
//   product with inner dimension 2K, done with FP64 16x16x4 MFMA.
#pragma once

#include "kernels.hpp"

namespace sosf {

typedef double v4d __attribute__((ext_vector_type(4)));

// Transpose of 16-lane row blocks across four 64-bit registers: on entry
// V[i] holds M[i][r] in row r, on exit V[i] holds M[r][i] in row r.  Two
// stages of permlane32 / permlane16 swaps (gfx950).
__device__ __forceinline__ void row_transpose4(double (&V)[4]) {
  uint32_t lo[4], hi[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint64_t b = (uint64_t)__double_as_longlong(V[i]);
    lo[i] = (uint32_t)b;
    hi[i] = (uint32_t)(b >> 32);
  }
#define SOSF_SWAP(FN, A, B)                                 \
  {                                                         \
    auto s = FN(lo[A], lo[B], false, false);                \
    lo[A] = s[0];                                           \
    lo[B] = s[1];                                           \
    auto t = FN(hi[A], hi[B], false, false);                \
    hi[A] = t[0];                                           \
    hi[B] = t[1];                                           \
  }
  SOSF_SWAP(__builtin_amdgcn_permlane32_swap, 0, 2)
  SOSF_SWAP(__builtin_amdgcn_permlane32_swap, 1, 3)
  SOSF_SWAP(__builtin_amdgcn_permlane16_swap, 0, 1)
  SOSF_SWAP(__builtin_amdgcn_permlane16_swap, 2, 3)
#undef SOSF_SWAP
#pragma unroll
  for (int i = 0; i < 4; ++i)
    V[i] = __longlong_as_double((long long)(((uint64_t)hi[i] << 32) | lo[i]));
}

// Per-wave LDS work region: the staging buffer of load/store, reused during
// the section loop for the entry-state responses RS (2K doubles per lane,
// stored component-major so that the lanes of a wave read consecutive
// addresses).
template <int N, typename TI>
__host__ __device__ constexpr int deferred_region_bytes(int K) {
  return ((kRows * Stage<N, TI>::ROWBUF * (int)sizeof(TI) > 64 * 2 * K * 8
               ? kRows * Stage<N, TI>::ROWBUF * (int)sizeof(TI)
               : 64 * 2 * K * 8) + 15) & ~15;
}
// LDS: per-wave regions, per-row states (2 + 2K doubles), then the block's
// copies of Theta (MFMA order) and of the coupling blocks.
template <int N, typename TI>
__host__ __device__ constexpr int deferred_lds_bytes(int K, int kbm) {
  return kWavesPerBlock * deferred_region_bytes<N, TI>(K) + kWavesPerBlock * kRows * (2 + 2 * K) * 8 +
         (N / 16) * kbm * 64 * 8 + 2 * K * (K - 1) * 8;
}

// One section of the zero-state cascade on the lane's segment (step 1
// through the cascade).  FIRST: the raw input keeps its true history.
// Returns the section's zero-state terminal values in (d0, d1).
template <int N, bool B0ONE, bool FIRST>
__device__ __forceinline__ void deferred_zero_state(double (&X)[N], ctab<double> c,
                                                    double *st, double &d0, double &d1) {
  typedef double T;
  T xm1 = T(0), xm2 = T(0);
  if (FIRST) {
    const T nx2 = last_of_row(X[N - 2]), nx1 = last_of_row(X[N - 1]);
    xm1 = shift_r(X[N - 1], st[1]);
    xm2 = shift_r(X[N - 2], st[0]);
    st[0] = nx2;
    st[1] = nx1;
  }
  fir_pass<N, T, B0ONE>(X, c, xm1, xm2);
  __builtin_amdgcn_sched_barrier(0);
  particular_pass<N, T>(X, c[OFF_A1], c[OFF_A2], T(0), T(0));
  d0 = X[N - 2];
  d1 = X[N - 1];
}

// True terminal values of section k (step 2 through the cascade): coupling
// to the sections j < k already solved (two independent accumulation
// chains), the group's entry state on lane 0, then the row scan.  Writes
// R S_k (entry state in lane 0) to rs and the exit state to st.
__device__ __forceinline__ void deferred_terminal(double d0, double d1, ctab<double> c,
                                                  const double *cp, double *rs, double *st, int k,
                                                  int D) {
  typedef double T;
  const int lane = lane_id();
  const bool l0 = (lane & 15) == 0;
  T f0 = T(0), f1 = T(0);
  const T *myrs = rs + lane;   // component c of this lane at myrs[64 c]
  int j = 0;
  for (; j + 1 < k; j += 2) {
    const T r0 = myrs[64 * (2 * j)], r1 = myrs[64 * (2 * j + 1)];
    const T s0 = myrs[64 * (2 * j + 2)], s1 = myrs[64 * (2 * j + 3)];
    d0 = fma_(cp[4 * j], r0, fma_(cp[4 * j + 1], r1, d0));
    d1 = fma_(cp[4 * j + 2], r0, fma_(cp[4 * j + 3], r1, d1));
    f0 = fma_(cp[4 * j + 4], s0, fma_(cp[4 * j + 5], s1, f0));
    f1 = fma_(cp[4 * j + 6], s0, fma_(cp[4 * j + 7], s1, f1));
  }
  if (j < k) {
    const T r0 = myrs[64 * (2 * j)], r1 = myrs[64 * (2 * j + 1)];
    d0 = fma_(cp[4 * j], r0, fma_(cp[4 * j + 1], r1, d0));
    d1 = fma_(cp[4 * j + 2], r0, fma_(cp[4 * j + 3], r1, d1));
  }
  d0 += f0;
  d1 += f1;
  const T e2 = st[2 + 2 * k], e1 = st[3 + 2 * k];
  const ctab<T> A = c + OFF_PH_POW;   // -C
  const T i0 = fma_(A[0], e2, A[1] * e1), i1 = fma_(A[2], e2, A[3] * e1);
  d0 += l0 ? i0 : T(0);
  d1 += l0 ? i1 : T(0);
  row_scan_2x2(d0, d1, c + OFF_PH_POW);
  rs[64 * (2 * k) + lane] = shift_r(d0, e2);
  rs[64 * (2 * k + 1) + lane] = shift_r(d1, e1);
  st[2 + 2 * k] = last_of_row(d0);
  st[3 + 2 * k] = last_of_row(d1);
}

// KBM: compile-time bound on the 4-wide state blocks (ceil(2K / 4) <= KBM);
// Theta is zero-padded to KBM blocks, so the MFMA loop is fully unrolled.
template <int N, typename TI, bool B0ONE, int KBM>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_deferred_kernel(
    const TI *__restrict__ x, TI *__restrict__ y, const double *__restrict__ tab,
    const double *__restrict__ coup, const double *__restrict__ theta, FiltArgs a) {
  typedef double T;
  static_assert(N % 16 == 0, "the correction works on 16-block tiles");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int K = a.K, D = 2 * K;
  // block-wide copies of the constant tables (before any wave may leave)
  T *theta_s = reinterpret_cast<T *>(smem + kWavesPerBlock * deferred_region_bytes<N, TI>(K) +
                                     kWavesPerBlock * kRows * (2 + D) * 8);
  T *coup_s = theta_s + (N / 16) * KBM * 64;
  for (int i = threadIdx.x; i < (N / 16) * KBM * 64; i += kWavesPerBlock * 64) theta_s[i] = theta[i];
  for (int i = threadIdx.x; i < 2 * K * (K - 1); i += kWavesPerBlock * 64) coup_s[i] = coup[i];
  __syncthreads();
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wave * kRows >= a.ntiles) return;   // uniform per wave
  const int lane = lane_id(), row = lane >> 4, rl = lane & 15;
  const int64_t t0 = (wave * kRows + row) * a.tile;
  unsigned char *region = smem + w * deferred_region_bytes<N, TI>(K);
  TI *buf = reinterpret_cast<TI *>(region) + row * Stage<N, TI>::ROWBUF;
  T *rs = reinterpret_cast<T *>(region);   // rs[comp * 64 + lane]: lanes contiguous in LDS
  // per-row state: st[0..1] raw input (x[-2], x[-1]); st[2+2k..] section k's
  // entry state (y_k[-2], y_k[-1])
  T *st = reinterpret_cast<T *>(smem + kWavesPerBlock * deferred_region_bytes<N, TI>(K)) +
          (w * kRows + row) * (2 + D);
  for (int i = 0; i < 2 + D; ++i) st[i] = T(0);   // the row's lanes write the same value
  const int64_t G = (int64_t)N * kL;
  const int64_t warm_groups = a.warm / G, steps = warm_groups + a.tile / G;
  const T gain = (T)a.gain;
  const int q = lane >> 4;
  T X[N];
  for (int64_t it = 0; it < steps; ++it) {
    const int64_t g = t0 - a.warm + it * G;
    const bool full = __builtin_amdgcn_ballot_w64(!(g >= 0 && g + G <= a.n)) == 0;
    load_group<N, TI, T>(X, x, g, a.n, full, buf);
    // software pipelined: the zero-state pass of section k does not depend
    // on the terminal solve of section k-1, so the two run interleaved
    T d0, d1;
    deferred_zero_state<N, B0ONE, true>(X, as_ctab(tab), st, d0, d1);
    for (int k = 1; k < K; ++k) {
      const T p0 = d0, p1 = d1;
      deferred_zero_state<N, B0ONE, false>(X, as_ctab(tab) + (int64_t)k * a.stride, st, d0, d1);
      deferred_terminal(p0, p1, as_ctab(tab) + (int64_t)(k - 1) * a.stride, coup_s + 2 * (k - 1) * (k - 2),
                        rs, st, k - 1, D);
    }
    deferred_terminal(d0, d1, as_ctab(tab) + (int64_t)(K - 1) * a.stride, coup_s + 2 * (K - 1) * (K - 2), rs,
                      st, K - 1, D);
    __builtin_amdgcn_wave_barrier();
    // homogeneous correction of all sections (step 3): Y = W_K + Theta RS,
    // one 16x16 tile per (row, 16 blocks of m), inner dimension in 4-blocks
#pragma unroll
    for (int mb = 0; mb < N / 16; ++mb) {
      v4d acc[kRows];
#pragma unroll
      for (int r = 0; r < kRows; ++r) acc[r] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int b = 0; b < KBM; ++b) {
        const T av = theta_s[(mb * KBM + b) * 64 + lane];   // Theta[16mb + rl][4b + q]
        const int comp = 4 * b + q;
        const int cc = comp < D ? comp : D - 1;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const T bv = comp < D ? rs[cc * 64 + 16 * r + rl] : T(0);   // RS_r[comp][rl]
          acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[r], 0, 0, 0);
        }
      }
      // acc[r] register i, row q': correction of tile r at m = 16mb + q' + 4i.
      // Transpose so that row r holds its own tile, then add.
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        T V[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) V[r] = acc[r][i];
        row_transpose4(V);
#pragma unroll
        for (int cidx = 0; cidx < 4; ++cidx) X[16 * mb + cidx + 4 * i] += V[cidx];
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (it >= warm_groups) store_group<N, TI, T>(X, y, g, a.n, full, gain, buf);
  }
}

}  // namespace sosf
