// Adjoint of the cascade (reverse-mode gradient) on the tile machinery.
//
// For y = F_K ... F_1 x with section k mapping its input u_k to its output
// w_k = u_{k+1} (A_k w_k = B_k u_k in the matrix form of Section II, A_k and
// B_k lower-triangular banded Toeplitz), and a loss with upstream gradient
// lambda_K = dL/dy:
//   mu_k = A_k^{-T} lambda_k,      lambda_{k-1} = B_k^T mu_k,  dL/dx = lambda_0,
//   dL/db_j = sum_i mu_k[i] u_k[i-j],   dL/da_j = -sum_i mu_k[i] w_k[i-j].
// A^{-T} and B^T are the same filters run backwards in time, so in reversed
// time r[t] = s[n' - 1 - t] every step is a causal filter again: the all-pole
// 1/A_k (the PH solve of Section VI-B with a trivial numerator) and the FIR
// B_k.  The sums become sum_t mu_r[t - j] u_r[t], lags of mu that the FIR
// already reads, so they are fused into it.
//
// Two kernels, in one of two modes:
//  * saved outputs: a forward PH pass writes every section's output w_k
//    (true scale, FP64) to the workspace, and the reversed-time adjoint pass
//    reads them back one section at a time (about 16K bytes per sample
//    written and read back);
//  * recompute: the forward pass writes the cascade state at every group
//    boundary (2K + 2 values per group, aligned with the adjoint's
//    reversed-time groups) and, for K >= 8, one section input u_{K/2}
//    (8 bytes per sample), and the adjoint pass recomputes the other section inputs of
//    each group from the nearest kept one, in registers (adj_slots: 7
//    forward section passes per group at K = 8, where every input from its
//    checkpoint would take K(K-1)/2 + 1 = 29).
#pragma once

#include <type_traits>

#include "kernels.hpp"
#include "adjoint_types.hpp"

namespace sosf {

// Sum over the 16 lanes of a row, in the row's last lane.
template <typename T>
__device__ __forceinline__ T row_total(T v) {
  v += shr<1>(v);
  v += shr<2>(v);
  v += shr<4>(v);
  v += shr<8>(v);
  return v;
}

// Reversed-time group I/O.  A signal s of n samples is read as
// r[t] = s[np - 1 - t], np = n rounded up to the vector width (r[t] = 0 for
// t < np - n); the row's group g of r is the ascending source range
// [np - g - G, np - g), moved with 16-byte vectors reversed in the stage.
// full: every row's range lies inside [0, n).
template <int N, typename TI, typename T>
__device__ __forceinline__ void load_group_rev(T (&X)[N], const TI *__restrict__ x, int64_t g,
                                               int64_t n, int64_t np, bool full,
                                               TI *__restrict__ buf) {
  typedef typename Vec16<TI>::type VT;
  constexpr int V = Stage<N, TI>::V, RUN = Stage<N, TI>::RUN, G = N * kL;
  const int rl = row_lane();
  if (full) {
    const VT *src = reinterpret_cast<const VT *>(x + (np - g - G));
#pragma unroll
    for (int j = 0; j < N / V; ++j) {
      const int e = G - V - (j * kL + rl) * V;   // reversed position of the vector's last element
      const VT v = __builtin_nontemporal_load(src + j * kL + rl);
      VT w;
#pragma unroll
      for (int i = 0; i < V; ++i) w[i] = v[V - 1 - i];
      *reinterpret_cast<VT *>(buf + (e / N) * RUN + (e % N)) = w;
    }
  } else {
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
      const int e = j * kL + rl;
      const int64_t i = np - 1 - g - e;
      buf[(e / N) * RUN + (e % N)] = (i >= 0 && i < n) ? x[i] : TI(0);
    }
  }
  __builtin_amdgcn_wave_barrier();
  stage_to_regs<N, TI, T>(X, buf);
  __builtin_amdgcn_wave_barrier();
}

template <int N, typename TI, typename T>
__device__ __forceinline__ void store_group_rev(const T (&X)[N], TI *__restrict__ y, int64_t g,
                                                int64_t n, int64_t np, bool full,
                                                TI *__restrict__ buf, T gain = T(1)) {
  typedef typename Vec16<TI>::type VT;
  constexpr int V = Stage<N, TI>::V, RUN = Stage<N, TI>::RUN, G = N * kL;
  const int rl = row_lane();
  regs_to_stage<N, TI, T>(X, gain, buf);
  __builtin_amdgcn_wave_barrier();
  if (full) {
    VT *dst = reinterpret_cast<VT *>(y + (np - g - G));
#pragma unroll
    for (int j = 0; j < N / V; ++j) {
      const int e = G - V - (j * kL + rl) * V;
      const VT w = *reinterpret_cast<const VT *>(buf + (e / N) * RUN + (e % N));
      VT v;
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = w[V - 1 - i];
      __builtin_nontemporal_store(v, dst + j * kL + rl);
    }
  } else {
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
      const int e = j * kL + rl;
      const int64_t i = np - 1 - g - e;
      if (i >= 0 && i < n) y[i] = buf[(e / N) * RUN + (e % N)];
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// A forward-time group in registers (lane l holds samples lN .. lN + N - 1
// of the row's group) into the reversed-time layout of the same samples,
// out of place: lane 15 - l's run, in reverse order (DPP row_mirror moves
// lane 15 - l's value into lane l).
template <int N>
__device__ __forceinline__ void to_reversed(double (&R)[N], const double (&F)[N]) {
#pragma unroll
  for (int m = 0; m < N; ++m) R[m] = dpp<0x140, true>(F[N - 1 - m]);
}

// All-pole part of a section by PH (Section VI-B with b = (1, 0, 0)): X := (1/A) X
// on the group, ys = (y[-2], y[-1]) of the output, replaced by the group's
// last two outputs.
template <int N>
__device__ __forceinline__ void allpole_ph(double (&X)[N], ctab<double> c, double *ys) {
  typedef double T;
  const T a1 = c[OFF_A1], a2 = c[OFF_A2];
  const T ys2 = ys[0], ys1 = ys[1];
  const bool l0 = row_lane() == 0;
  particular_pass<N, T>(X, a1, a2, l0 ? ys1 : T(0), l0 ? ys2 : T(0));
  T p = X[N - 2], q = X[N - 1];
  row_scan_2x2(p, q, c + OFF_PH_POW);
  X[N - 2] = p;
  X[N - 1] = q;
  const T pr = shr<1>(p), qr = shr<1>(q);
  const ctab<T> u1 = c + OFF_U1;
  const ctab<T> u2 = c + OFF_U1 + N;
#pragma unroll
  for (int m = 0; m < N - 2; ++m) X[m] = fma_(-u2[m], pr, fma_(-u1[m], qr, X[m]));
  ys[0] = last_of_row(p);
  ys[1] = last_of_row(q);
}

// Adjoint rows per section (kBwdRow doubles): b0 b1 b2 a1 a2 (divided by a0,
// b0 not factored), the forward pass's cumulative b0 scale, the caller's a0.
enum : int { BW_B0 = 0, BW_B1 = 1, BW_B2 = 2, BW_A1 = 3, BW_A2 = 4, BW_SCALE = 5, BW_A0 = 6 };

struct BwdArgs {
  int64_t n, np;            // samples; n rounded up to the vector width
  int64_t tile, warm, ntiles;
  int64_t sstride;          // elements between saved section outputs
  int64_t shift;            // forward tiles cover [-shift, n)
  int64_t nck;              // recompute mode: group checkpoints
  int64_t stash;            // recompute mode: > 0 when the row has an LDS stash
  int64_t mid_off;          // recompute mode: doubles from the checkpoints to the kept u_H
  int32_t K, stride;
};

// Forward pass of one row's tile.  Saved-output mode: writes w_k (true
// scale, FP64) of every section k to saved + k * sstride.  Recompute mode
// (RC): writes, before each of its groups, the row's boundary values (the
// state the cascade enters the group with) as checkpoint j = (np - g)/G - 1,
// the reversed-time group that covers the same samples; the tiles start
// where the groups line up with the reversed-time ones (shift = -np mod G);
// for K >= 8 it also writes the group's input u_H of section H = K/2 to
// saved + mid_off + j G, element (m, lane) at m L + lane (adj_slots).
// PH, FP64 arithmetic, tiles as in filter_rows.  STORE_Y: also store the
// cascade's output y (the forward pass of a training step, which then
// needs no second pass for the adjoint).  st: 2 + 2K boundary values;
// rowbuf: one FP64 group.
template <int N, typename TI, bool B0ONE, bool RC, bool STORE_Y>
__device__ __forceinline__ void save_rows(const TI *__restrict__ x, double *__restrict__ saved,
                                          TI *__restrict__ y, ctab<double> ct, ctab<double> cb,
                                          const AdjView &v, int64_t tile_index, bool aligned, double *st,
                                          unsigned char *rowbuf) {
  typedef double T;
  TI *buf = reinterpret_cast<TI *>(rowbuf);
  double *dbuf = reinterpret_cast<double *>(rowbuf);
  const int SE = state_elems(v.K);
  for (int i = 0; i < SE; ++i) st[i] = T(0);
  const int64_t G = (int64_t)N * kL;
  // tiles over [-shift, n): groups start where x + g is 16-byte aligned (the
  // samples before 0 read as zeros); the saved arrays start shift elements
  // in, so that their groups are aligned too
  const int64_t t0 = tile_index * v.tile - v.shift;
  if (!RC) saved += v.shift;
  const int64_t warm_groups = v.warm / G, steps = warm_groups + v.tile / G;
  const int H = RC && adj_mid(v.K) > 0 ? adj_mid(v.K) : -1;   // RC: section whose input is kept (adj_slots)
  T X[N];
  for (int64_t it = 0; it < steps; ++it) {
    const int64_t g = t0 - v.warm + it * G;
    const bool full = aligned && __builtin_amdgcn_ballot_w64(!(g >= 0 && g + G <= v.n)) == 0;
    const bool live = it >= warm_groups;
    const int64_t j = (v.np - g) / G - 1;   // g = np mod G: exact
    const bool keep = RC && live && j >= 0 && j < v.nck;
    if (keep)
      for (int i = row_lane(); i < SE; i += kL) saved[j * SE + i] = st[i];
    load_group<N, TI, T>(X, x, g, v.n, full, buf);
    T xs2 = st[0], xs1 = st[1];
    st[0] = last_of_row(X[N - 2]);
    st[1] = last_of_row(X[N - 1]);
    for (int k = 0; k < v.K; ++k) {
      if (keep && k == H) {
        // the group's u_H for the adjoint, element (m, lane) at m * L + lane
        double *mp = saved + v.mid_off + j * G + row_lane();
#pragma unroll
        for (int m = 0; m < N; ++m) mp[m * kL] = X[m];
      }
      ph_section<N, T, B0ONE>(X, ct + (int64_t)k * v.stride, xs2, xs1, st + 2 + 2 * k);
      if (!RC && live)
        store_group<N, double, T>(X, saved + (int64_t)k * v.sstride, g, v.n, full, cb[kBwdRow * k + BW_SCALE],
                                  dbuf);
    }
    if (STORE_Y && live)
      store_group<N, TI, T>(X, y, g, v.n, full, cb[kBwdRow * (v.K - 1) + BW_SCALE], buf);
  }
}

// Reversed-time adjoint of one row's tile: run-in, then per group
// lambda = r(gy), and for k = K-1 .. 0 mu = (1/A_k) lambda, the five sums of
// section k, lambda = B_k mu; the group's final lambda is r(dL/dx).  The
// tile's sums go to sums[k][tile][0..4] (section-major, so that each
// section's reduction reads contiguous memory): sum mu[t] u[t],
// mu[t-1] u[t], mu[t-2] u[t], mu[t-1] w[t], mu[t-2] w[t] (reversed time, t
// over the tile).
// u = u_k and w = w_k come from the saved outputs, or (RC) from the group's
// checkpoint: the group's input in forward time through sections 0 .. k-1
// (and k, for w_{K-1}), then mirrored into reversed time; those values are
// in the kernels' scaled domain, so the sums take the cumulative b0 scales
// once per group.  Since w_k = u_{k+1}, two arrays take the roles of u and w
// in turn (no copies between steps).
// st: 7K values (2K all-pole output states, then 5K running sums); RC adds
// the group's checkpoint and a working copy of it (2 + 2K each).
// RC recomputes u_k from the nearest kept input at or below it, in k - s
// passes (adj_slots): u_H from the forward pass (K >= 8), the group's input
// u_0, and in each phase two inputs kept on the phase's first pass, one
// in the row's LDS stash (v.stash > 0: one FP64 group, forward layout) and
// one in registers.  rowbuf:
// the row's stage, FP64 in the saved-output mode (which reads FP64
// groups), else of the I/O type.
template <int N, typename TI, bool B0ONE, bool RC>
__device__ __forceinline__ void adjoint_rows(const TI *__restrict__ gy, TI *__restrict__ gx,
                                             const TI *__restrict__ x, const double *__restrict__ saved,
                                             ctab<double> ct, ctab<double> cb, double *__restrict__ sums,
                                             const AdjView &v, int64_t tile_index, bool aligned,
                                             double *st, unsigned char *rowbuf, double *stash) {
  typedef double T;
  TI *buf = reinterpret_cast<TI *>(rowbuf);
  double *dbuf = reinterpret_cast<double *>(rowbuf);
  // RC: the inputs kept per group (adj_slots): u_H in the workspace, and
  // per phase one input in the LDS stash and one in registers
  const int H = RC ? adj_mid(v.K) : 0;
  const bool lds_stash = RC && v.stash > 0;
  constexpr int SRUN = Stage<N, double>::RUN;   // stash doubles per lane (padded)
  double *my_stash = stash + row_lane() * SRUN;
  T *acc = st + 2 * v.K;
  const int SE = state_elems(v.K);
  T *ck = st + 7 * v.K, *cw = ck + SE;   // RC: checkpoint, working copy
  for (int i = 0; i < 7 * v.K; ++i) st[i] = T(0);
  if (!RC) saved += v.shift;   // the saved arrays' origin, as written by save_rows
  const int64_t G = (int64_t)N * kL;
  const int64_t t0 = tile_index * v.tile;
  const int64_t pad = v.np - v.n;
  const int64_t warm_groups = v.warm / G, steps = warm_groups + v.tile / G;
  T X[N], A[N], B[N], F[N], R1[N];
  int64_t g = 0, j = 0;
  bool full = false, live = false;

  // RC: F = u_from (the group's input from the stage, u_H from the
  // workspace, or a kept input), then through sections from .. upto-1
  // (capture: keep the phase's inputs on the way); the chain's input state
  // is left in xs2, xs1
  T xs2 = T(0), xs1 = T(0);
  auto forward = [&](int from, int upto, const AdjSlots &sl, bool capture) {
    if (from == 0) {
      stage_to_regs<N, TI, T>(F, buf);
    } else if (from == H) {   // (kept indices lie strictly inside a phase, never at H)
      // u_H of this group (zero past the checkpointed range)
      const bool in = j < v.nck;
      const double *mp = saved + v.mid_off + j * G + row_lane();
#pragma unroll
      for (int m = 0; m < N; ++m) F[m] = in ? mp[m * kL] : T(0);
    } else if (from == sl.lds) {
#pragma unroll
      for (int m = 0; m < N; m += 2) {
        const vd2 p = *reinterpret_cast<const vd2 *>(my_stash + m);
        F[m] = p[0];
        F[m + 1] = p[1];
      }
    } else {
#pragma unroll
      for (int m = 0; m < N; ++m) F[m] = R1[m];
    }
    for (int i = row_lane(); i < SE; i += kL) cw[i] = ck[i];
    __builtin_amdgcn_wave_barrier();
    xs2 = cw[2 * from];   // section from-1's last two outputs before the group
    xs1 = cw[2 * from + 1];
    for (int q = from; q < upto; ++q) {
      ph_section<N, T, B0ONE>(F, ct + (int64_t)q * v.stride, xs2, xs1, cw + 2 + 2 * q);
      if (capture && q + 1 == sl.lds) {
#pragma unroll
        for (int m = 0; m < N; m += 2) *reinterpret_cast<vd2 *>(my_stash + m) = vd2{F[m], F[m + 1]};
      }
      if (capture && q + 1 == sl.regs) {
#pragma unroll
        for (int m = 0; m < N; ++m) R1[m] = F[m];
      }
    }
  };
  // U = u_k in reversed time
  auto input_of = [&](int k, T (&U)[N]) {
    if constexpr (RC) {
      const AdjSlots sl = adj_slots(v.K, lds_stash, H > 0 && k >= H ? 1 : 0);
      int from = sl.base;
      if (k != sl.top) {   // the phase's top keeps the others on its way
        if (sl.lds && sl.lds <= k && sl.lds > from) from = sl.lds;
        if (sl.regs && sl.regs <= k && sl.regs > from) from = sl.regs;
      }
      forward(from, k, sl, k == sl.top);
      to_reversed<N>(U, F);
      __builtin_amdgcn_wave_barrier();
    } else {
      if (k == 0)
        load_group_rev<N, TI, T>(U, x, g, v.n, v.np, full, buf);
      else
        load_group_rev<N, double, T>(U, saved + (int64_t)(k - 1) * v.sstride, g, v.n, v.np, full, dbuf);
    }
  };
  // the adjoint of section k on X, with U = u_k, W = w_k.  B0ONE: the
  // transposed FIR runs with b0 factored out (the sub-plan's b1 / b0,
  // b2 / b0), so X carries lambda and mu divided by pk = the product of b0
  // over the sections after k; the sums take pk back, and gx the product
  // over all sections.  (The plan factors b0 only where every product of
  // the first sections' b0 lies within 2^-400 .. 2^400, so pk, a ratio of
  // two of them, lies within 2^-800 .. 2^800.)
  T pk = T(1);
  auto step = [&](int k, const T (&U)[N], const T (&W)[N]) {
    const ctab<T> c = ct + (int64_t)k * v.stride;
    const ctab<T> b = cb + kBwdRow * k;
    T *ys = st + 2 * k;
    const T old2 = ys[0], old1 = ys[1];
    allpole_ph<N>(X, c, ys);                                 // X = mu_k (/ pk)
    const T m1 = shift_r(X[N - 1], old1), m2 = shift_r(X[N - 2], old2);
    const T b0 = b[BW_B0];
    const T b1 = B0ONE ? c[OFF_B1] : b[BW_B1], b2 = B0ONE ? c[OFF_B2] : b[BW_B2];
    if (live) {
      T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0), s4 = T(0);
#pragma unroll
      for (int m = N - 1; m >= 0; --m) {
        const T p1 = m >= 1 ? X[m - 1] : m1;
        const T p2 = m >= 2 ? X[m - 2] : (m == 1 ? m1 : m2);
        s0 = fma_(X[m], U[m], s0);
        s1 = fma_(p1, U[m], s1);
        s2 = fma_(p2, U[m], s2);
        s3 = fma_(p1, W[m], s3);
        s4 = fma_(p2, W[m], s4);
        X[m] = fma_(b2, p2, fma_(b1, p1, B0ONE ? X[m] : b0 * X[m]));
      }
      // the row's totals reach its last lane, which adds them (unscaled:
      // the scales are the same in every group and are applied once, when
      // the tile's sums are written)
      s0 = row_total(s0);
      s1 = row_total(s1);
      s2 = row_total(s2);
      s3 = row_total(s3);
      s4 = row_total(s4);
      if (row_lane() == kL - 1) {
        T *ak = acc + 5 * k;
        ak[0] += s0;
        ak[1] += s1;
        ak[2] += s2;
        ak[3] += s3;
        ak[4] += s4;
      }
    } else {
#pragma unroll
      for (int m = N - 1; m >= 0; --m) {
        const T p1 = m >= 1 ? X[m - 1] : m1;
        const T p2 = m >= 2 ? X[m - 2] : (m == 1 ? m1 : m2);
        X[m] = fma_(b2, p2, fma_(b1, p1, B0ONE ? X[m] : b0 * X[m]));
      }
    }
    if (B0ONE) pk *= b0;
  };

  for (int64_t it = 0; it < steps; ++it) {
    g = t0 - v.warm + it * G;
    full = aligned && __builtin_amdgcn_ballot_w64(!(g >= pad && g + G <= v.np)) == 0;
    live = it >= warm_groups;   // uniform per wave
    pk = T(1);
    load_group_rev<N, TI, T>(X, gy, g, v.n, v.np, full, buf);
    if (live) {
      // A = u_{K-1}, B = w_{K-1}
      if constexpr (RC) {
        // the group covers forward samples [np - g - G, np - g): its input in
        // forward order (kept in the row's stage until the group's gx is
        // stored) and the state the cascade enters it with
        load_group<N, TI, T>(F, x, v.np - g - G, v.n, full, buf);
        j = g / G;
        for (int i = row_lane(); i < SE; i += kL) ck[i] = j < v.nck ? saved[j * SE + i] : T(0);
        __builtin_amdgcn_wave_barrier();
        const AdjSlots top = adj_slots(v.K, lds_stash, H > 0 ? 1 : 0);
        forward(top.base, v.K - 1, top, true);
        to_reversed<N>(A, F);
        ph_section<N, T, B0ONE>(F, ct + (int64_t)(v.K - 1) * v.stride, xs2, xs1, cw + 2 + 2 * (v.K - 1));
        to_reversed<N>(B, F);
        __builtin_amdgcn_wave_barrier();
      } else {
        input_of(v.K - 1, A);
        load_group_rev<N, double, T>(B, saved + (int64_t)(v.K - 1) * v.sstride, g, v.n, v.np, full, dbuf);
      }
    }
    for (int k = v.K - 1;;) {
      step(k, A, B);
      if (--k < 0) break;
      if (live) input_of(k, B);   // w_k = u_{k+1} is in A
      step(k, B, A);
      if (--k < 0) break;
      if (live) input_of(k, A);
    }
    if (live) store_group_rev<N, TI, T>(X, gx, g, v.n, v.np, full, buf, pk);
  }
  // one lane per row writes the row's sums (rows past the last tile have
  // none), scaled: in RC u_k and w_k are in the scaled domain (w_k =
  // scale_k W, u_k = scale_{k-1} U), and with B0ONE mu_k = pk X, pk the
  // product of b0 over the sections after k
  __builtin_amdgcn_wave_barrier();
  if (row_lane() == 0 && tile_index < v.ntiles) {
    T p = T(1);
    for (int k = v.K - 1; k >= 0; --k) {
      T su = RC ? (k > 0 ? cb[kBwdRow * (k - 1) + BW_SCALE] : T(1)) : T(1);
      T sw = RC ? cb[kBwdRow * k + BW_SCALE] : T(1);
      if (B0ONE) {
        su *= p;
        sw *= p;
        p *= cb[kBwdRow * k + BW_B0];
      }
      double *o = sums + ((int64_t)k * v.ntiles + tile_index) * 5;
      for (int j = 0; j < 5; ++j) o[j] = acc[5 * k + j] * (j < 3 ? su : sw);
    }
  }
}

// LDS doubles per row of the adjoint pass: all-pole states and sums, and
// in recompute mode the group's checkpoint and its working copy.
__host__ __device__ constexpr int adj_row_elems(int K, bool rc) { return 7 * K + (rc ? 2 * state_elems(K) : 0); }

// LDS of the adjoint pass per workgroup: the rows' stages (FP64 in the
// saved-output mode, the I/O type in recompute mode), then the rows' states
// (adj_row_elems each), then, with a stash, one padded FP64 group per row.
template <int N, typename TI, bool RC>
struct AdjLds {
  typedef typename std::conditional<RC, TI, double>::type SI;
  static constexpr int ROWBUF_BYTES = Stage<N, SI>::ROWBUF * (int)sizeof(SI);
  static constexpr int STAGE_BYTES = kWavesPerBlock * kRows * ROWBUF_BYTES;
  static constexpr int STASH_ROW = Stage<N, double>::ROWBUF;   // doubles per row
  static __host__ __device__ constexpr size_t bytes(int kmax, bool stash) {
    return (size_t)STAGE_BYTES + (size_t)kWavesPerBlock * kRows * adj_row_elems(kmax, RC) * sizeof(double) +
           (stash ? (size_t)kWavesPerBlock * kRows * STASH_ROW * sizeof(double) : 0);
  }
  // row r (0 .. 15) of the workgroup
  static __device__ unsigned char *rowbuf(unsigned char *smem, int r) { return smem + r * ROWBUF_BYTES; }
  static __device__ double *states(unsigned char *smem, int r, int kmax) {
    return reinterpret_cast<double *>(smem + STAGE_BYTES) + r * adj_row_elems(kmax, RC);
  }
  static __device__ double *stash(unsigned char *smem, int r, int kmax) {
    return reinterpret_cast<double *>(smem + STAGE_BYTES) + kWavesPerBlock * kRows * adj_row_elems(kmax, RC) +
           r * STASH_ROW;
  }
};

__device__ __forceinline__ AdjView adj_view(const BwdArgs &a) {
  AdjView v;
  v.n = a.n;
  v.np = a.np;
  v.tile = a.tile;
  v.warm = a.warm;
  v.ntiles = a.ntiles;
  v.sstride = a.sstride;
  v.shift = a.shift;
  v.nck = a.nck;
  v.stash = a.stash;
  v.mid_off = a.mid_off;
  v.K = a.K;
  v.stride = a.stride;
  return v;
}

// Single signal: row r of wavefront w takes tile 4w + r.
template <int N, typename TI, bool B0ONE, bool RC, bool STORE_Y>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_save_kernel(
    const TI *__restrict__ x, double *__restrict__ saved, TI *__restrict__ y, const double *__restrict__ tab,
    const double *__restrict__ bwd, BwdArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  // the stage holds one group per row in FP64 (the saved outputs, in that
  // mode), which also fits the input's group
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wave * kRows >= a.ntiles) return;
  const int row = lane_id() >> 4;
  double *st = reinterpret_cast<double *>(smem + stage_bytes<N, double>()) +
               (int64_t)(w * kRows + row) * state_elems(a.K);
  unsigned char *rowbuf = smem + (w * kRows + row) * Stage<N, double>::ROWBUF * 8;
  save_rows<N, TI, B0ONE, RC, STORE_Y>(x, saved, y, as_ctab(tab), as_ctab(bwd), adj_view(a), wave * kRows + row,
                                       true, st, rowbuf);
}

template <int N, typename TI, bool B0ONE, bool RC>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_adjoint_kernel(
    const TI *__restrict__ gy, TI *__restrict__ gx, const TI *__restrict__ x,
    const double *__restrict__ saved, const double *__restrict__ tab, const double *__restrict__ bwd,
    double *__restrict__ partials, BwdArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wave * kRows >= a.ntiles) return;
  const int row = lane_id() >> 4;
  const int64_t tile_index = wave * kRows + row;
  typedef AdjLds<N, TI, RC> Lds;
  const int r = w * kRows + row;
  adjoint_rows<N, TI, B0ONE, RC>(gy, gx, x, saved, as_ctab(tab), as_ctab(bwd), partials,
                                 adj_view(a), tile_index, true, Lds::states(smem, r, a.K), Lds::rowbuf(smem, r),
                                 Lds::stash(smem, r, a.K));
}

__device__ __forceinline__ AdjView adj_view(const AdjChan &c) {
  AdjView v;
  v.n = c.n;
  v.np = c.np;
  v.tile = c.tile;
  v.warm = c.warm;
  v.ntiles = c.ntiles;
  v.sstride = c.sstride;
  v.shift = c.shift;
  v.nck = c.nck;
  v.stash = c.stash;
  v.mid_off = c.mid_off;
  v.K = c.K;
  v.stride = c.stride;
  return v;
}

// The batched adjoint's launches follow the channel set they were enqueued
// for (grids, workspace, gsos rows).  hdr[1] is the batch's current
// schedule generation and gen the one at the launch: a launch replayed
// from a graph captured before a replan finds them different and writes
// nothing.
template <int N, typename TI, bool B0ONE, bool RC, bool STORE_Y>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_save_batched_kernel(
    const TI *__restrict__ x, double *__restrict__ ws, TI *__restrict__ y, const AdjChan *__restrict__ chans,
    const int32_t *__restrict__ item_chan, int64_t items, int32_t kmax, const int64_t *__restrict__ hdr,
    int64_t gen) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  if (hdr[1] != gen) return;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (item >= items) return;
  const AdjChan &c = chans[item_chan[item]];
  const int row = lane_id() >> 4;
  const int64_t tile_index = (item - c.first_item) * kRows + row;
  double *st = reinterpret_cast<double *>(smem + stage_bytes<N, double>()) +
               (int64_t)(w * kRows + row) * state_elems(kmax);
  unsigned char *rowbuf = smem + (w * kRows + row) * Stage<N, double>::ROWBUF * 8;
  save_rows<N, TI, B0ONE, RC, STORE_Y>(x + c.off, ws + c.saved_off, STORE_Y ? y + c.off : nullptr, as_ctab(c.tab),
                                       as_ctab(c.bwd), adj_view(c), tile_index, true, st, rowbuf);
}

template <int N, typename TI, bool B0ONE, bool RC>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_adjoint_batched_kernel(
    const TI *__restrict__ gy, TI *__restrict__ gx, const TI *__restrict__ x, double *__restrict__ ws,
    const AdjChan *__restrict__ chans, const int32_t *__restrict__ item_chan, int64_t items,
    int32_t kmax, const int64_t *__restrict__ hdr, int64_t gen) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  if (hdr[1] != gen) return;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (item >= items) return;
  const AdjChan &c = chans[item_chan[item]];
  const int row = lane_id() >> 4;
  const int64_t tile_index = (item - c.first_item) * kRows + row;
  typedef AdjLds<N, TI, RC> Lds;
  const int r = w * kRows + row;
  adjoint_rows<N, TI, B0ONE, RC>(gy + c.off, gx + c.off, x + c.off, ws + c.saved_off, as_ctab(c.tab),
                                 as_ctab(c.bwd), ws + c.partial_off, adj_view(c),
                                 tile_index, true, Lds::states(smem, r, kmax), Lds::rowbuf(smem, r),
                                 Lds::stash(smem, r, kmax));
}

// dL/d(sos) from the per-tile sums of one section: the block sums
// sums[k][t][j] over the tiles in a fixed order (deterministic), then
// applies the chain rule through the division by a0: with normalised
// c = (b0, b1, b2, a1, a2)/a0, dL/db_j = gb_j / a0, dL/da_j = ga_j / a0
// (j = 1, 2) and dL/da0 = -(gb . (b0, b1, b2) + ga . (a1, a2)) / a0.
// THREADS: the block size (a power of two); the order of the sums depends
// on it and on nothing else.
template <int THREADS>
__device__ __forceinline__ void adjoint_reduce(const double *__restrict__ partials, int64_t ntiles, int32_t K,
                                               int k, const double *__restrict__ bwd,
                                               double *__restrict__ g) {
  __shared__ double red[5][THREADS];
  const int tid = threadIdx.x;
  double s[5] = {0, 0, 0, 0, 0};
  for (int64_t t = tid; t < ntiles; t += THREADS)
    for (int j = 0; j < 5; ++j) s[j] += partials[((int64_t)k * ntiles + t) * 5 + j];
  for (int j = 0; j < 5; ++j) red[j][tid] = s[j];
  __syncthreads();
  for (int h = THREADS / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int j = 0; j < 5; ++j) red[j][tid] += red[j][tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    const double *b = bwd + kBwdRow * k;
    const double a0 = b[BW_A0];
    const double gb0 = red[0][0], gb1 = red[1][0], gb2 = red[2][0];
    const double ga1 = -red[3][0], ga2 = -red[4][0];
    g[0] = gb0 / a0;
    g[1] = gb1 / a0;
    g[2] = gb2 / a0;
    g[3] = -(gb0 * b[BW_B0] + gb1 * b[BW_B1] + gb2 * b[BW_B2] + ga1 * b[BW_A1] + ga2 * b[BW_A2]) / a0;
    g[4] = ga1 / a0;
    g[5] = ga2 / a0;
  }
}

// block k: section k of the single signal (one block per section, so a
// wide one: a long signal has tens of thousands of tiles)
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void sos_adjoint_reduce_kernel(const double *__restrict__ partials,
                                                                            int64_t ntiles, int32_t K,
                                                                            const double *__restrict__ bwd,
                                                                            double *__restrict__ gsos) {
  adjoint_reduce<kReduceThreads>(partials, ntiles, K, blockIdx.x, bwd, gsos + 6 * blockIdx.x);
}

// block b: row b of the batch's gsos, i.e. section b - gsos_row of channel
// red_chan[b]
__global__ __launch_bounds__(256) void sos_adjoint_reduce_batched_kernel(
    double *__restrict__ ws, const AdjChan *__restrict__ chans, const int32_t *__restrict__ red_chan,
    double *__restrict__ gsos, const int64_t *__restrict__ hdr, int64_t gen) {
  if (hdr[1] != gen) return;
  const AdjChan &c = chans[red_chan[blockIdx.x]];
  const int k = (int)blockIdx.x - c.gsos_row;
  adjoint_reduce<256>(ws + c.partial_off, c.ntiles, c.K, k, c.bwd, gsos + 6 * (int64_t)blockIdx.x);
}

}  // namespace sosf
