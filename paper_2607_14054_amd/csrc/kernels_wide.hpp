// Wide groups with the lane runs in memory: N = 256 .. 1024 blocks per lane
// run (and N = 128 with FP64 I/O), L = 16, FP64 arithmetic.
//
// The method is the one of kernels.hpp (Sections V to VII): lane l of a
// 16-lane row holds the run x[g + l N + m], m = 0..N-1, and each section is
// solved on the group by PH or by cyclic reduction.  What changes is where
// a lane's run lives.  At these N it does not fit a lane's registers (N
// doubles; 8 KB at N = 1024), nor the LDS of a compute unit's resident
// lanes, so it lives in a device workspace: element (m, lane) of wavefront
// w at ws[(w N + m) 64 + lane], so that the 64 lanes of a wavefront touch
// 512 consecutive bytes for each m.  An all-PH cascade makes one pass over
// that buffer per section (wide_ph_group); CR makes one per level.
//
// Input and output move between HBM and the workspace 64 blocks at a time,
// staged through the same per-row LDS buffer as N = 64 (the stride-N
// permutation of one chunk of 64 blocks: each lane's 64 samples are 256
// contiguous bytes, and the 16 lanes' chunks are loaded and stored with
// coalesced 16-byte vectors).
#pragma once

#include "kernels.hpp"

namespace sosf {

constexpr int kWideChunk = 64;     // blocks staged per pass through LDS
constexpr int kWideMaxN = 1024;
constexpr int kWideBatch = 8;      // independent CR updates whose reads are issued together

struct WideArgs {
  int64_t n;
  int32_t K;
  int32_t stride;
  int32_t N, lgN;
  int64_t tile;     // samples per tile, a multiple of the group (16 N)
  int64_t warm;     // run-in samples before each tile, a multiple of the group
  int64_t ntiles;
  double gain;
  double *ws;       // (ntiles / 4, rounded up) x N x 64 doubles
};

// Chunk c (blocks 64 c .. 64 c + 63) of the row's group at g <-> X[0..63].
template <typename TI>
__device__ __forceinline__ void wide_load_chunk(double (&X)[kWideChunk], const TI *__restrict__ x, int64_t g,
                                                int N, int c, int64_t n, bool full, TI *__restrict__ buf) {
  typedef typename Vec16<TI>::type VT;
  constexpr int V = Stage<kWideChunk, TI>::V, RUN = Stage<kWideChunk, TI>::RUN;
  const int rl = row_lane();
  if (full) {
#pragma unroll
    for (int j = 0; j < kWideChunk / V; ++j) {
      const int e = (j * kL + rl) * V;   // element of the row's chunk: run e / 64, block e % 64
      const int run = e / kWideChunk, off = e % kWideChunk;
      const VT v = __builtin_nontemporal_load(
          reinterpret_cast<const VT *>(x + g + (int64_t)run * N + (int64_t)c * kWideChunk + off));
      *reinterpret_cast<VT *>(buf + run * RUN + off) = v;
    }
  } else {
#pragma unroll 1
    for (int j = 0; j < kWideChunk; ++j) {
      const int e = j * kL + rl;
      const int run = e / kWideChunk, off = e % kWideChunk;
      const int64_t i = g + (int64_t)run * N + (int64_t)c * kWideChunk + off;
      buf[run * RUN + off] = (i >= 0 && i < n) ? x[i] : TI(0);
    }
  }
  __builtin_amdgcn_wave_barrier();
  stage_to_regs<kWideChunk, TI, double>(X, buf);
  __builtin_amdgcn_wave_barrier();
}

template <typename TI>
__device__ __forceinline__ void wide_store_chunk(const double (&X)[kWideChunk], TI *__restrict__ y, int64_t g,
                                                 int N, int c, int64_t n, bool full, double gain,
                                                 TI *__restrict__ buf) {
  typedef typename Vec16<TI>::type VT;
  constexpr int V = Stage<kWideChunk, TI>::V, RUN = Stage<kWideChunk, TI>::RUN;
  const int rl = row_lane();
  regs_to_stage<kWideChunk, TI, double>(X, gain, buf);
  __builtin_amdgcn_wave_barrier();
  if (full) {
#pragma unroll
    for (int j = 0; j < kWideChunk / V; ++j) {
      const int e = (j * kL + rl) * V;
      const int run = e / kWideChunk, off = e % kWideChunk;
      const VT v = *reinterpret_cast<const VT *>(buf + run * RUN + off);
      __builtin_nontemporal_store(v, reinterpret_cast<VT *>(y + g + (int64_t)run * N +
                                                            (int64_t)c * kWideChunk + off));
    }
  } else {
#pragma unroll 1
    for (int j = 0; j < kWideChunk; ++j) {
      const int e = j * kL + rl;
      const int run = e / kWideChunk, off = e % kWideChunk;
      const int64_t i = g + (int64_t)run * N + (int64_t)c * kWideChunk + off;
      if (i >= 0 && i < n) y[i] = buf[run * RUN + off];
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// PH on a run held in the workspace (Section VI-B, as ph_section): one
// ascending pass forms the non-recursive stage and the particular solution
// together (the inputs x_{m-1}, x_{m-2} and outputs w_{m-1}, w_{m-2} ride
// in registers), the terminal scan runs along the row, and a second pass
// applies the homogeneous correction.  S: this lane's element m at S[64 m].
template <bool B0ONE>
__device__ __forceinline__ void wide_ph_section(double *__restrict__ S, int N, ctab<double> c, double &xs2,
                                                double &xs1, double *ys) {
  const double b0 = c[OFF_B0], b1 = c[OFF_B1], b2 = c[OFF_B2], a1 = c[OFF_A1], a2 = c[OFF_A2];
  const double ys2 = ys[0], ys1 = ys[1];
  // the extended blocks: the previous lane's last two inputs (lane 0: the
  // previous group's, xs1 and xs2)
  double p1 = shift_r(S[64 * (N - 1)], xs1), p2 = shift_r(S[64 * (N - 2)], xs2);
  const double m0 = lane0_mask<double>();
  double w1 = m0 * ys1, w2 = m0 * ys2;
#pragma unroll 8
  for (int m = 0; m < N; ++m) {
    const double xm = S[64 * m];
    double v = B0ONE ? xm : b0 * xm;
    v = fma_(b1, p1, v);
    v = fma_(b2, p2, v);
    v = fma_(-a2, w2, v);
    v = fma_(-a1, w1, v);
    S[64 * m] = v;
    p2 = p1;
    p1 = xm;
    w2 = w1;
    w1 = v;
  }
  double p = w2, q = w1;   // w_{N-2}, w_{N-1}
  row_scan_2x2(p, q, c + OFF_PH_POW);
  S[64 * (N - 2)] = p;
  S[64 * (N - 1)] = q;
  const double pr = shr<1>(p), qr = shr<1>(q);
  const ctab<double> u1 = c + OFF_U1;
  const ctab<double> u2 = c + OFF_U1 + N;
#pragma unroll 8
  for (int m = 0; m < N - 2; ++m) S[64 * m] = fma_(-u2[m], pr, fma_(-u1[m], qr, S[64 * m]));
  ys[0] = last_of_row(p);
  ys[1] = last_of_row(q);
  xs2 = ys2;
  xs1 = ys1;
}

// Cyclic reduction on a run held in the workspace (Section VI-C, as
// cr_section, the same steps in the same order).
template <bool B0ONE>
__device__ __forceinline__ void wide_cr_section(double *__restrict__ S, int N, int LG, ctab<double> c,
                                                double &xs2, double &xs1, double *ys) {
  const double b0 = c[OFF_B0], b1 = c[OFF_B1], b2 = c[OFF_B2], a1 = c[OFF_A1], a2 = c[OFF_A2];
  const double ys2 = ys[0], ys1 = ys[1];
  // non-recursive stage in place, ascending with the inputs in registers
  double p1 = shift_r(S[64 * (N - 1)], xs1), p2 = shift_r(S[64 * (N - 2)], xs2);
#pragma unroll 8
  for (int m = 0; m < N; ++m) {
    const double xm = S[64 * m];
    double v = B0ONE ? xm : b0 * xm;
    v = fma_(b1, p1, v);
    S[64 * m] = fma_(b2, p2, v);
    p2 = p1;
    p1 = xm;
  }
  // the previous group's outputs enter the first element of blocks 0 and 1
  const double m0 = lane0_mask<double>(), z1 = m0 * ys1, z2 = m0 * ys2;
  S[0] = fma_(-a1, z1, fma_(-a2, z2, S[0]));
  S[64] = fma_(-a2, z1, S[64]);
  // reduction, eq. cr_coeff_update coefficients per level.  The updates of
  // one parity at one level are independent (each reads blocks of the other
  // parity), so they go kWideBatch at a time with every read issued before
  // the first write: the compiler cannot tell that the runtime offsets do
  // not overlap, and would otherwise wait on each read in turn.
  for (int i = 0; i < LG; ++i) {
    const int s = 1 << i, ni = N >> i;
    const double fe = c[OFF_CR_LVL + 4 * i], e = c[OFF_CR_LVL + 4 * i + 1];
    const double wrap = shr<1>(S[64 * (N - 1)]);
    for (int par = 0; par < 2; ++par) {
      const double f = par == 0 ? fe : e;
      for (int j0 = par; j0 < ni; j0 += 2 * kWideBatch) {
        double a[kWideBatch], b[kWideBatch];
#pragma unroll
        for (int t = 0; t < kWideBatch; ++t) {
          const int j = j0 + 2 * t, m = s * (j + 1) - 1;
          if (j < ni) {
            a[t] = S[64 * m];
            b[t] = j == 0 ? wrap : S[64 * (m - s)];
          }
        }
#pragma unroll
        for (int t = 0; t < kWideBatch; ++t) {
          const int j = j0 + 2 * t, m = s * (j + 1) - 1;
          if (j < ni) S[64 * m] = fma_(-f, b[t], a[t]);
        }
      }
    }
  }
  // terminal block, eq. cr_terminal_block, by the row scan
  {
    double p = 0.0, q = S[64 * (N - 1)];
    row_scan_2x2(p, q, c + OFF_CR_POW);
    S[64 * (N - 1)] = q;
  }
  // back substitution, eqs. cr_companion_block .. cr_backsub_final
  const double r1 = shr<1>(S[64 * (N - 1)]);
  for (int i = LG - 1; i >= 0; --i) {
    const int s = 1 << i, ni = N >> i;
    const double cc = c[OFF_CR_LVL + 4 * i + 2], dd = c[OFF_CR_LVL + 4 * i + 3];
    const double w3 = ni == 2 ? shr<1>(r1) : shr<1>(S[64 * (N - 2 * s - 1)]);
    // the even blocks of the level read only odd ones: independent, batched
    for (int j0 = 0; j0 < ni; j0 += 2 * kWideBatch) {
      double a[kWideBatch], y1[kWideBatch], y3[kWideBatch];
#pragma unroll
      for (int t = 0; t < kWideBatch; ++t) {
        const int j = j0 + 2 * t, m = s * (j + 1) - 1;
        if (j < ni) {
          a[t] = S[64 * m];
          y1[t] = (j >= 1) ? S[64 * (m - s)] : r1;
          y3[t] = (j >= 3) ? S[64 * (m - 3 * s)] : (j == 0 ? w3 : r1);
        }
      }
#pragma unroll
      for (int t = 0; t < kWideBatch; ++t) {
        const int j = j0 + 2 * t, m = s * (j + 1) - 1;
        if (j < ni) S[64 * m] = fma_(-cc, y1[t], fma_(-dd, y3[t], a[t]));
      }
    }
  }
  ys[0] = last_of_row(S[64 * (N - 2)]);
  ys[1] = last_of_row(S[64 * (N - 1)]);
  xs2 = ys2;
  xs1 = ys1;
}

// One group of a row through an all-PH cascade with the run in the
// workspace (Section VI-B, the steps of ph_section), in one pass over the
// run per section: the input is read chunk by chunk from HBM into section
// 0's pass, every later pass applies the previous section's homogeneous
// correction (step 3) to its input as it reads it, and the store applies
// the last section's.  Each pass forms the non-recursive stage and the
// particular recurrence (step 1) and ends with the terminal scan (step 2).
// That is one read and one write of the run per section, where separate
// FIR-and-recurrence and correction passes take two of each.
// st: the row's boundary values (raw input pair, then each section's output
// pair); live: store the group.
template <typename TI, bool B0ONE>
__device__ __forceinline__ void wide_ph_group(double *__restrict__ S, const TI *__restrict__ x,
                                              TI *__restrict__ y, int64_t g, int N, int64_t n, int K,
                                              int stride, ctab<double> ct, double gain, double *st,
                                              TI *__restrict__ buf, bool full, bool live) {
  const int rl = row_lane();
  const double m0 = lane0_mask<double>();
  // the raw input's extended blocks: the two samples before the lane's run
  // (for lane 0 the previous group's last two, kept in st)
  double p1, p2;
  {
    const int64_t i1 = g + (int64_t)rl * N - 1, i2 = i1 - 1;
    const double v1 = (rl > 0 && i1 >= 0 && i1 < n) ? (double)x[i1] : 0.0;
    const double v2 = (rl > 0 && i2 >= 0 && i2 < n) ? (double)x[i2] : 0.0;
    p1 = rl == 0 ? st[1] : v1;
    p2 = rl == 0 ? st[0] : v2;
    // this group's last two raw inputs, for the next group's lane 0
    const int64_t e = g + (int64_t)kL * N;
    st[0] = (e - 2 >= 0 && e - 2 < n) ? (double)x[e - 2] : 0.0;
    st[1] = (e - 1 >= 0 && e - 1 < n) ? (double)x[e - 1] : 0.0;
  }
  double pr = 0.0, qr = 0.0, xs2 = 0.0, xs1 = 0.0;
  for (int k = 0; k < K; ++k) {
    const ctab<double> c = ct + (int64_t)k * stride;
    const double b0 = c[OFF_B0], b1 = c[OFF_B1], b2 = c[OFF_B2], a1 = c[OFF_A1], a2 = c[OFF_A2];
    double *ys = st + 2 + 2 * k;
    const double ys2 = ys[0], ys1 = ys[1];
    double w1 = m0 * ys1, w2 = m0 * ys2;
    if (k == 0) {
      // section 0 reads the raw input, staged 64 blocks at a time
      for (int cc = 0; cc < N / kWideChunk; ++cc) {
        double X[kWideChunk];
        wide_load_chunk<TI>(X, x, g, N, cc, n, full, buf);
#pragma unroll
        for (int j = 0; j < kWideChunk; ++j) {
          const double xin = X[j];
          double v = B0ONE ? xin : b0 * xin;
          v = fma_(b1, p1, v);
          v = fma_(b2, p2, v);
          v = fma_(-a2, w2, v);
          v = fma_(-a1, w1, v);
          S[64 * (cc * kWideChunk + j)] = v;
          p2 = p1;
          p1 = xin;
          w2 = w1;
          w1 = v;
        }
      }
    } else {
      // the previous section's output: its particular solution plus the
      // homogeneous correction from (pr, qr), true in the last two blocks.
      // The correction e_m = -(u1_m qr + u2_m pr) is the previous section's
      // homogeneous response to (e_-1, e_-2) = (qr, pr), generated by its
      // own recurrence rather than read from the u tables (scalar loads a
      // lone wavefront per SIMD would wait on)
      const ctab<double> cp = c - stride;   // the previous section's table
      const double pa1 = cp[OFF_A1], pa2 = cp[OFF_A2];
      double e1 = qr, e2 = pr;
#pragma unroll 8
      for (int m = 0; m < N - 2; ++m) {
        const double e = fma_(-pa1, e1, -pa2 * e2);
        e2 = e1;
        e1 = e;
        const double xin = S[64 * m] + e;
        double v = B0ONE ? xin : b0 * xin;
        v = fma_(b1, p1, v);
        v = fma_(b2, p2, v);
        v = fma_(-a2, w2, v);
        v = fma_(-a1, w1, v);
        S[64 * m] = v;
        p2 = p1;
        p1 = xin;
        w2 = w1;
        w1 = v;
      }
#pragma unroll
      for (int m = N - 2; m < N; ++m) {
        const double xin = S[64 * m];
        double v = B0ONE ? xin : b0 * xin;
        v = fma_(b1, p1, v);
        v = fma_(b2, p2, v);
        v = fma_(-a2, w2, v);
        v = fma_(-a1, w1, v);
        S[64 * m] = v;
        p2 = p1;
        p1 = xin;
        w2 = w1;
        w1 = v;
      }
    }
    // step 2: the true last two blocks along the row
    double p = w2, q = w1;
    row_scan_2x2(p, q, c + OFF_PH_POW);
    S[64 * (N - 2)] = p;
    S[64 * (N - 1)] = q;
    pr = shr<1>(p);
    qr = shr<1>(q);
    ys[0] = last_of_row(p);
    ys[1] = last_of_row(q);
    // the next section's extended blocks: this section's true output at the
    // end of the previous lane (lane 0: of the previous group)
    xs2 = ys2;
    xs1 = ys1;
    p1 = shift_r(q, xs1);
    p2 = shift_r(p, xs2);
  }
  if (!live) return;
  // the last section's correction by the same recurrence
  const ctab<double> cl = ct + (int64_t)(K - 1) * stride;
  const double pa1 = cl[OFF_A1], pa2 = cl[OFF_A2];
  double e1 = qr, e2 = pr;
  for (int cc = 0; cc < N / kWideChunk; ++cc) {
    double X[kWideChunk];
#pragma unroll
    for (int j = 0; j < kWideChunk; ++j) {
      const int m = cc * kWideChunk + j;
      if (m < N - 2) {
        const double e = fma_(-pa1, e1, -pa2 * e2);
        e2 = e1;
        e1 = e;
        X[j] = S[64 * m] + e;
      } else {
        X[j] = S[64 * m];
      }
    }
    wide_store_chunk<TI>(X, y, g, N, cc, n, full, gain, buf);
  }
}

// One wavefront filters four tiles, one per row, as sos_rows_kernel (run-in,
// then the tile, groups chained through the sections' boundary values).
template <typename TI, bool B0ONE, int SOLVER>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_wide_kernel(
    const TI *__restrict__ x, TI *__restrict__ y, const double *__restrict__ tab,
    const int32_t *__restrict__ solver, WideArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  TI *stage = reinterpret_cast<TI *>(smem);
  double *state = reinterpret_cast<double *>(smem + stage_bytes<kWideChunk, TI>());
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wave * kRows >= a.ntiles) return;   // uniform per wave
  const int row = lane_id() >> 4;
  const int64_t t0 = (wave * kRows + row) * a.tile;
  const int N = a.N;
  double *st = state + (int64_t)(w * kRows + row) * state_elems(a.K);
  TI *buf = stage + (w * kRows + row) * Stage<kWideChunk, TI>::ROWBUF;
  double *S = a.ws + (size_t)wave * N * 64 + lane_id();
  const ctab<double> ct = as_ctab(tab);
  for (int i = 0; i < state_elems(a.K); ++i) st[i] = 0.0;
  const int64_t G = (int64_t)N * kL;
  const int64_t warm_groups = a.warm / G, steps = warm_groups + a.tile / G;
  double X[kWideChunk];
  for (int64_t it = 0; it < steps; ++it) {
    const int64_t g = t0 - a.warm + it * G;
    const bool full = __builtin_amdgcn_ballot_w64(!(g >= 0 && g + G <= a.n)) == 0;
    if constexpr (SOLVER == SOS_PH) {
      wide_ph_group<TI, B0ONE>(S, x, y, g, N, a.n, a.K, a.stride, ct, a.gain, st, buf, full, it >= warm_groups);
      continue;
    }
    for (int c = 0; c < N / kWideChunk; ++c) {
      wide_load_chunk<TI>(X, x, g, N, c, a.n, full, buf);
#pragma unroll
      for (int m = 0; m < kWideChunk; ++m) S[64 * (c * kWideChunk + m)] = X[m];
    }
    double xs2 = st[0], xs1 = st[1];
    st[0] = last_of_row(S[64 * (N - 2)]);
    st[1] = last_of_row(S[64 * (N - 1)]);
    for (int k = 0; k < a.K; ++k) {
      const ctab<double> c = ct + (int64_t)k * a.stride;
      if (SOLVER == SOS_CR || (SOLVER == SOS_AUTO && solver[k] == SOS_CR))
        wide_cr_section<B0ONE>(S, N, a.lgN, c, xs2, xs1, st + 2 + 2 * k);
      else
        wide_ph_section<B0ONE>(S, N, c, xs2, xs1, st + 2 + 2 * k);
    }
    if (it >= warm_groups) {
      for (int c = 0; c < N / kWideChunk; ++c) {
#pragma unroll
        for (int m = 0; m < kWideChunk; ++m) X[m] = S[64 * (c * kWideChunk + m)];
        wide_store_chunk<TI>(X, y, g, N, c, a.n, full, a.gain, buf);
      }
    }
  }
}

}  // namespace sosf
