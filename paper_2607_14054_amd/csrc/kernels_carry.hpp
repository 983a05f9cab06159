// Exact carry between tiles: the alternative to the run-in for signals whose
// run-in is long against the tile the device needs for parallelism.
//
// The cascade state at a tile boundary, s = (y_k[-2], y_k[-1]) for every
// section k in the kernels' scaled domain (2K values), is an affine function
// of the state at the previous boundary.  With Phi the one-step transition of
// that state under zero raw input, a tile of T samples maps
//   s_out = Phi^T s_in + c,
// where c is the tile's end state from zero section states and its true raw
// input history (the input enters linearly, so the two parts add).  So:
//   1. every tile runs once from zero section states and writes c_t;
//   2. an inclusive scan over tiles gives S_t = c_t + Phi^T S_{t-1}, the
//      state at the end of tile t (log-depth: round j adds
//      Phi^(T 2^j) S_{t-2^j}; rounds stop once Phi^(T 2^j) is below the
//      run-in bound);
//   3. every tile runs again from S_{t-1} and stores its outputs.
// Two passes over the data against one pass plus the run-in: this pays when
// the run-in is longer than the tile.
#pragma once

#include "kernels.hpp"

namespace sosf {

constexpr int kCarryDMax = 32;   // 2K for K <= 16: Phi fits one workgroup

struct CarryArgs {
  int64_t n, tile, ntiles;
  int32_t K, stride;
  double gain;
  const double *states;   // from-state pass: [ntiles][2K], S_t (the state at the end of tile t)
  double *aggs;           // aggregate pass: [ntiles][2K], c_t
};

enum : int { CARRY_AGG = 1, CARRY_FROM = 2 };

// One wavefront filters four tiles, one per row, with no run-in.  The row
// starts from the raw input history (x[t0-2], x[t0-1]) and, in the
// from-state pass, the scanned section states at the end of the previous
// tile; the aggregate pass starts the sections from zero, stores nothing and
// writes the row's final section states.
template <int N, typename TI, bool B0ONE, int SOLVER, int MODE>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_carry_kernel(
    const TI *__restrict__ x, TI *__restrict__ y, const double *__restrict__ tab,
    const int32_t *__restrict__ solver, CarryArgs a) {
  typedef double T;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  TI *stage = reinterpret_cast<TI *>(smem);
  T *state = reinterpret_cast<T *>(smem + stage_bytes<N, TI>());
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wave * kRows >= a.ntiles) return;   // uniform per wave
  const int row = lane_id() >> 4;
  const int64_t tile_index = wave * kRows + row;
  const bool live = tile_index < a.ntiles;   // rows past the last tile run on zeros
  const int64_t t0 = tile_index * a.tile;
  const int D = 2 * a.K;
  T *st = state + (int64_t)(w * kRows + row) * state_elems(a.K);
  TI *buf = stage + (w * kRows + row) * Stage<N, TI>::ROWBUF;
  // the row's lanes write the same values
  st[0] = (live && t0 >= 2) ? (T)x[t0 - 2] : T(0);
  st[1] = (live && t0 >= 1) ? (T)x[t0 - 1] : T(0);
  for (int i = 0; i < D; ++i)
    st[2 + i] = (MODE == CARRY_FROM && live && tile_index > 0) ? a.states[(tile_index - 1) * D + i] : T(0);
  const ctab<T> ct = as_ctab(tab);
  const int64_t G = (int64_t)N * kL, steps = a.tile / G;
  T X[N];
  for (int64_t it = 0; it < steps; ++it) {
    const int64_t g = t0 + it * G;
    const bool full = __builtin_amdgcn_ballot_w64(!(g >= 0 && g + G <= a.n)) == 0;
    load_group<N, TI, T>(X, x, g, a.n, full, buf);
    T xs2 = st[0], xs1 = st[1];
    st[0] = last_of_row(X[N - 2]);
    st[1] = last_of_row(X[N - 1]);
    for (int k = 0; k < a.K; ++k) {
      const ctab<T> c = ct + (int64_t)k * a.stride;
      if (SOLVER == SOS_CR || (SOLVER == SOS_AUTO && solver[k] == SOS_CR))
        cr_section<N, T, B0ONE>(X, c, xs2, xs1, st + 2 + 2 * k);
      else
        ph_section<N, T, B0ONE>(X, c, xs2, xs1, st + 2 + 2 * k);
    }
    if (MODE == CARRY_FROM) store_group<N, TI, T>(X, y, g, a.n, full, (T)a.gain, buf);
  }
  if (MODE == CARRY_AGG && live && row_lane() == 0)
    for (int i = 0; i < D; ++i) a.aggs[tile_index * D + i] = st[2 + i];
}

// P[j] = Phi^(T 2^j), j < rounds, for a D x D transition (D <= 32): one
// workgroup, one thread per matrix entry; Phi^T by binary powering.
__global__ __launch_bounds__(1024) void carry_powers_kernel(const double *__restrict__ phi, int D, int64_t T,
                                                            int rounds, double *__restrict__ P) {
  __shared__ double base[kCarryDMax * kCarryDMax], acc[kCarryDMax * kCarryDMax];
  const int tid = threadIdx.x;
  const bool on = tid < D * D;
  const int i = on ? tid / D : 0, j = on ? tid % D : 0;
  if (on) {
    base[tid] = phi[tid];
    acc[tid] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  // acc = a * b, every thread reading before any writes
  auto mul_into = [&](double *dst, const double *a, const double *b) {
    double v = 0.0;
    if (on)
      for (int l = 0; l < D; ++l) v = __builtin_fma(a[i * D + l], b[l * D + j], v);
    __syncthreads();
    if (on) dst[tid] = v;
    __syncthreads();
  };
  for (int64_t e = T; e > 0; e >>= 1) {
    if (e & 1) mul_into(acc, acc, base);
    if (e > 1) mul_into(base, base, base);
  }
  for (int r = 0; r < rounds; ++r) {
    if (on) P[(int64_t)r * D * D + tid] = acc[tid];
    if (r + 1 < rounds) mul_into(acc, acc, acc);
  }
}

// One round of the inclusive scan over tiles:
// out[t] = in[t] + P in[t - off] for t >= off, else in[t].
__global__ __launch_bounds__(256) void carry_scan_kernel(const double *__restrict__ in, double *__restrict__ out,
                                                         const double *__restrict__ P, int D, int64_t ntiles,
                                                         int64_t off) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntiles * D) return;
  const int64_t t = idx / D;
  const int r = (int)(idx - t * D);
  double v = in[idx];
  if (t >= off) {
    const double *src = in + (t - off) * D;
    const double *pr = P + (int64_t)r * D;
    for (int l = 0; l < D; ++l) v = __builtin_fma(pr[l], src[l], v);
  }
  out[idx] = v;
}

// The powers and every scan round in one workgroup, when all tile states
// fit in LDS (ntiles * D <= kCarryOneBlock): the states and the powers live
// in LDS; each round reads all it needs before any thread writes.  The
// powers are kept transposed, so that the lanes of a round, which hold
// consecutive rows of a state, read consecutive words of a power's column.
// Dynamic LDS: (ntiles * D + 2 D^2) doubles.
constexpr int kCarryOneBlock = 8192;

__global__ __launch_bounds__(1024) void carry_scan_one_block_kernel(const double *__restrict__ phi, int D,
                                                                    int64_t T, int rounds, int ntiles,
                                                                    const double *__restrict__ in,
                                                                    double *__restrict__ out) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  double *S = reinterpret_cast<double *>(smem);
  const int E = ntiles * D;
  double *baseT = S + E, *accT = baseT + D * D;   // transposes of Phi^(2^b) and of the running power
  const int tid = threadIdx.x;
  const bool on = tid < D * D;
  const int i = on ? tid / D : 0, j = on ? tid % D : 0;
  for (int e = tid; e < E; e += 1024) S[e] = in[e];
  if (on) {
    baseT[tid] = phi[j * D + i];
    accT[tid] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  // dst = a b, every thread reading before any writes
  auto mul_into = [&](double *dst, const double *a, const double *b) {
    double v = 0.0;
    if (on)
      for (int l = 0; l < D; ++l) v = __builtin_fma(a[i * D + l], b[l * D + j], v);
    __syncthreads();
    if (on) dst[tid] = v;
    __syncthreads();
  };
  // (acc base)^T = base^T acc^T, (base base)^T = base^T base^T
  for (int64_t e = T; e > 0; e >>= 1) {
    if (e & 1) mul_into(accT, baseT, accT);
    if (e > 1) mul_into(baseT, baseT, baseT);
  }
  constexpr int kPer = kCarryOneBlock / 1024;   // states per thread
  for (int r = 0; r < rounds; ++r) {
    const int off = 1 << r;
    double v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * 1024;
      v[k] = 0.0;
      if (e < E) {
        const int t = e / D, row = e - t * D;
        double a = S[e];
        if (t >= off) {
          const double *src = S + (t - off) * D;
          for (int l = 0; l < D; ++l) a = __builtin_fma(accT[l * D + row], src[l], a);
        }
        v[k] = a;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int e = tid + k * 1024;
      if (e < E) S[e] = v[k];
    }
    __syncthreads();
    if (r + 1 < rounds) mul_into(accT, accT, accT);
  }
  for (int e = tid; e < E; e += 1024) out[e] = S[e];
}

}  // namespace sosf
