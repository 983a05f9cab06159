// Device code: the multi-block filter on lane groups of L = 16, 32 or 64.
//
// Layout (Section V, block size L): a 64-wide wavefront holds 64 / L
// independent signal block groups, one per group of L lanes ("row": for
// L = 16 a DPP row).  In row r, lane l (0..L-1) holds the l-th run of N
// consecutive samples of that row's group in registers X[0..N-1]; X[m] on
// lane l is x[m + l N], the l-th element of the stride-N block xbar_m.
// Moving a register one lane down inside the row (lane l receives lane
// l-1, lane 0 a fill value) is the shift matrix R.  With L = 16 every
// cross-lane step is a DPP row operation; with L = 32 or 64 the one-lane
// shift is a DPP wave shift and the longer shifts of the log-depth scans go
// through ds_bpermute.  The layout is kept across all K sections (Section
// VII-B): one permutation when a group is loaded, one de-permutation when
// it is stored.
//
// The rows of a wavefront work on different tiles of the signal, so
// nothing couples them; groups inside a tile are chained through the
// sections' boundary values (Section V), kept per row in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.hpp"

#ifndef SOSF_SCHED_CHUNK
#define SOSF_SCHED_CHUNK 4
#endif

namespace sosf {

// Fused multiply-add in the compute type (the generic builtin would promote
// float operands to double).
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Coefficient tables are read through the constant address space: they are
// never written while a kernel runs, and uniform loads from it go through
// the scalar cache.
template <typename T>
using ctab = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ ctab<T> as_ctab(const T *p) {
  return (ctab<T>)(p);
}

// ------------------------------------------------------------ lane moves

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
template <int L = kL>
__device__ __forceinline__ int row_lane() { return (int)(threadIdx.x & (L - 1)); }

// DPP controls (GFX9 encoding): row_shr:d = 0x110 + d, row_newbcast:15 = 0x15f.
template <int CTRL, bool ZERO>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, ZERO));
}
template <int CTRL, bool ZERO>
__device__ __forceinline__ double dpp(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, ZERO);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, ZERO);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// 32 bits from lane (lane - D) of the same row; lanes whose source lies
// before the row's first lane take `fill`.  L = 16: DPP row_shr:D, whose
// keep-old form leaves exactly those lanes at the old value, the fill.
// L = 32, 64: D = 1 is the DPP wave shift (a lane at a row start takes the
// fill by a select), longer shifts go through ds_bpermute (no LDS memory
// is touched; a negative source wraps inside the wavefront and is then
// replaced by the fill).
template <int L, int D>
__device__ __forceinline__ uint32_t lane_shift_u32(uint32_t v, uint32_t fill) {
  if constexpr (L == 16) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x110 + D, 0xf, 0xf, false);
  } else if constexpr (D == 1) {
    const uint32_t s = (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x138, 0xf, 0xf, false);
    return row_lane<L>() == 0 ? fill : s;
  } else {
    const uint32_t s = (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() - D) << 2, (int)v);
    return row_lane<L>() < D ? fill : s;
  }
}
template <int L, int D>
__device__ __forceinline__ float lane_shift(float v, float fill) {
  return __uint_as_float(lane_shift_u32<L, D>(__float_as_uint(v), __float_as_uint(fill)));
}
template <int L, int D>
__device__ __forceinline__ double lane_shift(double v, double fill) {
  const uint64_t b = (uint64_t)__double_as_longlong(v), f = (uint64_t)__double_as_longlong(fill);
  const uint32_t lo = lane_shift_u32<L, D>((uint32_t)b, (uint32_t)f);
  const uint32_t hi = lane_shift_u32<L, D>((uint32_t)(b >> 32), (uint32_t)(f >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Row shift by D with zeros entering the first D lanes of the row.
template <int D, typename T, int L = kL>
__device__ __forceinline__ T shr(T v) {
  if constexpr (L == 16) return dpp<0x110 + D, true>(v);
  else return lane_shift<L, D>(v, T(0));
}

// R with a fill value for lane 0 of the row.
template <int L = kL, typename T>
__device__ __forceinline__ T shift_r(T v, T fill) { return lane_shift<L, 1>(v, fill); }

// The row's last lane in every lane of the row.  L = 16: row_newbcast:15
// (a 64-bit value moves in one instruction); L = 64: the wavefront's lane
// 63, read into scalar registers; L = 32: lane 31 or 63 by half.
template <int L = kL>
__device__ __forceinline__ float last_of_row(float v) {
  if constexpr (L == 16) return dpp<0x15f, false>(v);
  const int a = __builtin_amdgcn_readlane(__float_as_int(v), 63);
  if constexpr (L == 64) return __int_as_float(a);
  const int b = __builtin_amdgcn_readlane(__float_as_int(v), 31);
  return __int_as_float(lane_id() < 32 ? b : a);
}
template <int L = kL>
__device__ __forceinline__ double last_of_row(double v) {
  if constexpr (L == 16)
    return __longlong_as_double(__builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), 0x15f, 0xf, 0xf, false));
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo63 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
  const uint32_t hi63 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
  if constexpr (L == 64) return __longlong_as_double((long long)(((uint64_t)hi63 << 32) | lo63));
  const uint32_t lo31 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 31);
  const uint32_t hi31 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 31);
  const bool first = lane_id() < 32;
  return __longlong_as_double(
      (long long)(((uint64_t)(first ? hi31 : hi63) << 32) | (first ? lo31 : lo63)));
}

// 1 in lane 0 of the row, 0 elsewhere: multiplies the previous group's
// boundary values into the first lane only.
template <typename T, int L = kL>
__device__ __forceinline__ T lane0_mask() { return row_lane<L>() == 0 ? T(1) : T(0); }

// Log-depth solve along the row of z_l = A z_{l-1} + z_l (z_{-1} = 0) for
// 2-vectors z = (p, q): round j adds A^(2^j) times the value 2^j lanes below
// (Kogge-Stone doubling).  pw holds A^(2^j) row-major for j = 0..log2(L)-1.
template <typename T, int L = kL>
__device__ __forceinline__ void row_scan_2x2(T &p, T &q, ctab<T> pw) {
#define SOSF_ROUND(J, D)                                                          \
  if constexpr (D < L) {                                                          \
    const T m00 = pw[4 * J], m01 = pw[4 * J + 1], m10 = pw[4 * J + 2], m11 = pw[4 * J + 3]; \
    const T ps = shr<D, T, L>(p), qs = shr<D, T, L>(q);                           \
    const T np = fma_(m00, ps, fma_(m01, qs, p));               \
    q = fma_(m10, ps, fma_(m11, qs, q));                        \
    p = np;                                                                       \
  }
  SOSF_ROUND(0, 1) SOSF_ROUND(1, 2) SOSF_ROUND(2, 4) SOSF_ROUND(3, 8) SOSF_ROUND(4, 16) SOSF_ROUND(5, 32)
#undef SOSF_ROUND
}

// ------------------------------------------------------------ one section

// Boundary values carried from group to group (Section V), one set per
// row: x[-2], x[-1] of each section's input and y[-2], y[-1] of its output.
// A section's input is the previous section's output, so the row keeps the
// raw input's pair and every section's output pair (2 + 2K values).

// The block loops below are fully unrolled; left alone, the scheduler hoists
// the FIR of every block ahead of the recursion, which keeps inputs and FIR
// outputs live together.  A scheduling barrier every kSchedChunk blocks
// bounds that lookahead (and the register pressure it costs).
constexpr int kSchedChunk = SOSF_SCHED_CHUNK;

// Non-recursive stage (eq. feedforward_block_uniform) in place, in
// descending m so that every input is read before it is overwritten:
//   v_m = b0 x_m + b1 x_{m-1} + b2 x_{m-2},
// with the extended blocks x_{-1} = R x_{N-1} + e0 x[-1] and
// x_{-2} = R x_{N-2} + e0 x[-2] passed in.  The recursive pass that follows
// then also runs in place, so no register is live twice and the section
// loop needs no copies.
template <int N, typename T, bool B0ONE>
__device__ __forceinline__ void fir_pass(T (&X)[N], ctab<T> c, T xm1, T xm2) {
  const T b0 = c[OFF_B0], b1 = c[OFF_B1], b2 = c[OFF_B2];
#pragma unroll
  for (int m = N - 1; m >= 0; --m) {
    const T p1 = m >= 1 ? X[m - 1] : xm1;
    const T p2 = m >= 2 ? X[m - 2] : (m == 1 ? xm1 : xm2);
    T v = B0ONE ? X[m] : b0 * X[m];
    v = fma_(b1, p1, v);
    X[m] = fma_(b2, p2, v);
    if ((m & (kSchedChunk - 1)) == 0) __builtin_amdgcn_sched_barrier(0);
  }
}

// Particular solution, eq. particular_recurrence, in place:
// w_m = v_m - a1 w_{m-1} - a2 w_{m-2} from (w_{-1}, w_{-2}) = (w1, w2).
// The y[n-2] term is added first, so one FMA per step is on the
// recurrence's critical path.
template <int N, typename T>
__device__ __forceinline__ void particular_pass(T (&X)[N], T a1, T a2, T w1, T w2) {
#pragma unroll
  for (int m = 0; m < N; ++m) {
    T v = fma_(-a2, w2, X[m]);
    v = fma_(-a1, w1, v);
    X[m] = v;
    w2 = w1;
    w1 = v;
    if ((m & (kSchedChunk - 1)) == kSchedChunk - 1) __builtin_amdgcn_sched_barrier(0);
  }
}

// PH factorisation (Section VI-B) of one section on one group per row.
//
// Boundary values: (xs2, xs1) = (x[-2], x[-1]) of this section's input on
// entry; ys = (y[-2], y[-1]) of its output, read and then replaced by the
// group's last two outputs.  Section k's input is section k-1's output, so
// on exit (xs2, xs1) holds the old ys: the next section's input state.
template <int N, typename T, bool B0ONE, int L = kL>
__device__ __forceinline__ void ph_section(T (&X)[N], ctab<T> c, T &xs2, T &xs1, T *ys) {
  const T a1 = c[OFF_A1], a2 = c[OFF_A2];
  const T ys2 = ys[0], ys1 = ys[1];
  fir_pass<N, T, B0ONE>(X, c, shift_r<L>(X[N - 1], xs1), shift_r<L>(X[N - 2], xs2));
  __builtin_amdgcn_sched_barrier(0);
  // step 1, eq. particular_recurrence: every lane a zero-state recurrence
  // over its own N samples.  On lane 0 of the row the recurrence starts from
  // the previous group's outputs, which is the same arithmetic as the state
  // correction of v_0[0] and v_1[0].
  const T m0 = lane0_mask<T, L>();
  particular_pass<N, T>(X, a1, a2, m0 * ys1, m0 * ys2);
  // step 2, eq. recursive_doubling_equation: y_e[l] = w_e[l] - C y_e[l-1]
  // along the row, with y_e[l] = (y[(l+1)N-2], y[(l+1)N-1])
  T p = X[N - 2], q = X[N - 1];
  row_scan_2x2<T, L>(p, q, c + OFF_PH_POW);
  X[N - 2] = p;
  X[N - 1] = q;
  // step 3, eq. PH_forward: the homogeneous correction from the true
  // terminal values of the preceding lane (R y_{N-2}, R y_{N-1})
  const T pr = shr<1, T, L>(p), qr = shr<1, T, L>(q);
  const ctab<T> u1 = c + OFF_U1;
  const ctab<T> u2 = c + OFF_U1 + N;
#pragma unroll
  for (int m = 0; m < N - 2; ++m) X[m] = fma_(-u2[m], pr, fma_(-u1[m], qr, X[m]));
  ys[0] = last_of_row<L>(p);
  ys[1] = last_of_row<L>(q);
  xs2 = ys2;
  xs1 = ys1;
}

// PH over the cascade with each section's homogeneous correction (step 3)
// applied inside the next section's pass: one ascending pass per section
// corrects the section's input (the previous section's particular
// solution, from that section's terminal values pr, qr and coefficients
// cp), forms the non-recursive stage and runs the particular recurrence
// (step 1); then the terminal scan (step 2).  The arithmetic is
// ph_section's except that the correction comes from its own recurrence
// rather than the u tables; fewer values are live at once, which is what a
// run too long for the architectural registers (N = 128) needs.
// FIRST: the input is the raw signal (nothing to correct).  On exit X holds
// the section's particular solution with its true last two blocks, and
// (pr, qr) the correction's inputs for the next pass (or for
// ph_last_correction).  Boundary values as for ph_section.
template <int N, typename T, bool B0ONE, bool FIRST, int L = kL>
__device__ __forceinline__ void ph_fused_section(T (&X)[N], ctab<T> c, ctab<T> cp, T &pr, T &qr, T &xs2,
                                                 T &xs1, T *ys) {
  const T b0 = c[OFF_B0], b1 = c[OFF_B1], b2 = c[OFF_B2], a1 = c[OFF_A1], a2 = c[OFF_A2];
  const T ys2 = ys[0], ys1 = ys[1];
  // the extended blocks: the input's last two blocks in the previous lane
  // (true values: the raw input, or the previous section's scanned ones)
  T p1 = shift_r<L>(X[N - 1], xs1), p2 = shift_r<L>(X[N - 2], xs2);
  const T m0 = lane0_mask<T, L>();
  T w1 = m0 * ys1, w2 = m0 * ys2;
  // the correction e_m = -(u1_m qr + u2_m pr) is the previous section's
  // homogeneous response to (e_-1, e_-2) = (qr, pr): generated by its own
  // recurrence instead of read from the u tables, whose scalar loads a lone
  // wavefront per SIMD would wait on
  const T pa1 = cp[OFF_A1], pa2 = cp[OFF_A2];
  T e1 = qr, e2 = pr;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    T xin = X[m];
    if (!FIRST && m < N - 2) {
      const T e = fma_(-pa1, e1, -pa2 * e2);
      e2 = e1;
      e1 = e;
      xin += e;
    }
    T v = B0ONE ? xin : b0 * xin;
    v = fma_(b1, p1, v);
    v = fma_(b2, p2, v);
    v = fma_(-a2, w2, v);
    v = fma_(-a1, w1, v);
    X[m] = v;
    p2 = p1;
    p1 = xin;
    w2 = w1;
    w1 = v;
    if ((m & (kSchedChunk - 1)) == kSchedChunk - 1) __builtin_amdgcn_sched_barrier(0);
  }
  T p = X[N - 2], q = X[N - 1];
  row_scan_2x2<T, L>(p, q, c + OFF_PH_POW);
  X[N - 2] = p;
  X[N - 1] = q;
  pr = shr<1, T, L>(p);
  qr = shr<1, T, L>(q);
  ys[0] = last_of_row<L>(p);
  ys[1] = last_of_row<L>(q);
  xs2 = ys2;
  xs1 = ys1;
}

// The last section's homogeneous correction (step 3, eq. PH_forward), by
// the same recurrence as in ph_fused_section.
template <int N, typename T>
__device__ __forceinline__ void ph_last_correction(T (&X)[N], ctab<T> cp, T pr, T qr) {
  const T pa1 = cp[OFF_A1], pa2 = cp[OFF_A2];
  T e1 = qr, e2 = pr;
#pragma unroll
  for (int m = 0; m < N - 2; ++m) {
    const T e = fma_(-pa1, e1, -pa2 * e2);
    e2 = e1;
    e1 = e;
    X[m] += e;
  }
}

// Cyclic reduction (Section VI-C) of one section on one group per row.
// Level i works on the blocks m = s(j+1)-1 (s = 2^i, j = 0..N/s-1); even j
// are eliminated, odd j retained.  A reference below j = 0 wraps to the last
// blocks through R.
// Boundary values as for ph_section.
template <int N, typename T, bool B0ONE, int L = kL>
__device__ __forceinline__ void cr_section(T (&X)[N], ctab<T> c, T &xs2, T &xs1, T *ys) {
  constexpr int LG = __builtin_ctz(N);
  const T a1 = c[OFF_A1], a2 = c[OFF_A2];
  const T ys2 = ys[0], ys1 = ys[1];
  fir_pass<N, T, B0ONE>(X, c, shift_r<L>(X[N - 1], xs1), shift_r<L>(X[N - 2], xs2));
  __builtin_amdgcn_sched_barrier(0);
  // the previous group's outputs enter the first element of blocks 0 and 1
  const T m0 = lane0_mask<T, L>(), z1 = m0 * ys1, z2 = m0 * ys2;
  X[0] = fma_(-a1, z1, fma_(-a2, z2, X[0]));
  X[1] = fma_(-a2, z1, X[1]);
  // reduction, eq. cr_coeff_update coefficients per level
#pragma unroll
  for (int i = 0; i < LG; ++i) {
    const int s = 1 << i, ni = N >> i;
    const T fe = c[OFF_CR_LVL + 4 * i], e = c[OFF_CR_LVL + 4 * i + 1];
    const T wrap = shr<1, T, L>(X[N - 1]);
#pragma unroll
    for (int j = 0; j < ni; j += 2) {
      const int m = s * (j + 1) - 1;
      X[m] = fma_(-fe, j == 0 ? wrap : X[m - s], X[m]);
    }
#pragma unroll
    for (int j = 1; j < ni; j += 2) {
      const int m = s * (j + 1) - 1;
      X[m] = fma_(-e, X[m - s], X[m]);
    }
  }
  // terminal block, eq. cr_terminal_block: (I + e R + f R^2) y = v' on block
  // N-1, a second-order recurrence along the row; solved by the log-depth
  // scan of z_l = (y_{l-1}, y_l) = T z_{l-1} + (0, v'_l)
  {
    T p = T(0), q = X[N - 1];
    row_scan_2x2<T, L>(p, q, c + OFF_CR_POW);
    X[N - 1] = q;
  }
  // back substitution, eqs. cr_companion_block .. cr_backsub_final
  const T r1 = shr<1, T, L>(X[N - 1]);   // R y_{N-1}, reused at every level
#pragma unroll
  for (int i = LG - 1; i >= 0; --i) {
    const int s = 1 << i, ni = N >> i;
    const T cc = c[OFF_CR_LVL + 4 * i + 2], dd = c[OFF_CR_LVL + 4 * i + 3];
    T w3;   // the once-wrapped block for j = 0
    if (ni == 2) w3 = shr<1, T, L>(r1);                 // R^2 y_{N-1}
    else w3 = shr<1, T, L>(X[N - 2 * s - 1]);           // R y at position ni-3
#pragma unroll
    for (int j = 0; j < ni; j += 2) {
      const int m = s * (j + 1) - 1;
      const T y1 = (j >= 1) ? X[m - s] : r1;
      const T y3 = (j >= 3) ? X[m - 3 * s] : (j == 0 ? w3 : r1);
      X[m] = fma_(-cc, y1, fma_(-dd, y3, X[m]));
    }
  }
  ys[0] = last_of_row<L>(X[N - 2]);
  ys[1] = last_of_row<L>(X[N - 1]);
  xs2 = ys2;
  xs1 = ys1;
}

// ------------------------------------------------------------ memory

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));

template <typename TI>
struct Vec16;
template <>
struct Vec16<float> { typedef vf4 type; static constexpr int n = 4; };
template <>
struct Vec16<double> { typedef vd2 type; static constexpr int n = 2; };

// A group (L N samples per row) is moved between HBM and registers through
// a per-wave LDS buffer.  Global accesses are 16-byte vectors, the L lanes
// of a row covering 16 L consecutive bytes of that row's group per
// instruction; the stride-N permutation happens in LDS, where lane l reads
// or writes its own run of N samples.  Each run is padded by 16 bytes so
// that the 16-byte LDS accesses of 16 lanes fall on distinct banks.
template <int N, typename TI, int L = kL>
struct Stage {
  static constexpr int V = Vec16<TI>::n;        // elements per 16-byte vector
  static constexpr int RUN = N + V;             // padded run length (elements)
  static constexpr int ROWBUF = L * RUN;        // per row
  static constexpr int ROWS = 64 / L;           // rows per wave
  static constexpr int ELEMS = ROWS * ROWBUF;   // per wave
};

// Lane l's run of the row's staged group <-> its N registers.
template <int N, typename TI, typename T, int L = kL>
__device__ __forceinline__ void stage_to_regs(T (&X)[N], const TI *__restrict__ buf) {
  typedef typename Vec16<TI>::type VT;
  constexpr int V = Stage<N, TI, L>::V, RUN = Stage<N, TI, L>::RUN;
  const int rl = row_lane<L>();
#pragma unroll
  for (int j = 0; j < N / V; ++j) {
    VT v = *reinterpret_cast<const VT *>(buf + rl * RUN + j * V);
#pragma unroll
    for (int i = 0; i < V; ++i) X[j * V + i] = T(v[i]);
  }
}
template <int N, typename TI, typename T, int L = kL>
__device__ __forceinline__ void regs_to_stage(const T (&X)[N], T gain, TI *__restrict__ buf) {
  typedef typename Vec16<TI>::type VT;
  constexpr int V = Stage<N, TI, L>::V, RUN = Stage<N, TI, L>::RUN;
  const int rl = row_lane<L>();
#pragma unroll
  for (int j = 0; j < N / V; ++j) {
    VT v;
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = (TI)(X[j * V + i] * gain);
    *reinterpret_cast<VT *>(buf + rl * RUN + j * V) = v;
  }
}

// g: this row's group start (may be negative or run past n in the run-in
// and at the end; those samples read as zero).  full: every row of the wave
// has a whole group inside [0, n).
template <int N, typename TI, typename T, int L = kL>
__device__ __forceinline__ void load_group(T (&X)[N], const TI *__restrict__ x, int64_t g,
                                           int64_t n, bool full, TI *__restrict__ buf) {
  typedef typename Vec16<TI>::type VT;
  constexpr int V = Stage<N, TI, L>::V, RUN = Stage<N, TI, L>::RUN;
  const int rl = row_lane<L>();
  if (full) {
    const VT *src = reinterpret_cast<const VT *>(x + g);
#pragma unroll
    for (int j = 0; j < N / V; ++j) {
      const int e = (j * L + rl) * V;             // element of the row's group
      VT v = __builtin_nontemporal_load(src + j * L + rl);
      *reinterpret_cast<VT *>(buf + (e / N) * RUN + (e % N)) = v;
    }
  } else {
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
      const int e = j * L + rl;
      const int64_t i = g + e;
      buf[(e / N) * RUN + (e % N)] = (i >= 0 && i < n) ? x[i] : TI(0);
    }
  }
  __builtin_amdgcn_wave_barrier();
  stage_to_regs<N, TI, T, L>(X, buf);
  __builtin_amdgcn_wave_barrier();
}

template <int N, typename TI, typename T, int L = kL>
__device__ __forceinline__ void store_group(const T (&X)[N], TI *__restrict__ y, int64_t g,
                                            int64_t n, bool full, T gain, TI *__restrict__ buf) {
  typedef typename Vec16<TI>::type VT;
  constexpr int V = Stage<N, TI, L>::V, RUN = Stage<N, TI, L>::RUN;
  const int rl = row_lane<L>();
  regs_to_stage<N, TI, T, L>(X, gain, buf);
  __builtin_amdgcn_wave_barrier();
  if (full) {
    VT *dst = reinterpret_cast<VT *>(y + g);
#pragma unroll
    for (int j = 0; j < N / V; ++j) {
      const int e = (j * L + rl) * V;
      VT v = *reinterpret_cast<const VT *>(buf + (e / N) * RUN + (e % N));
      __builtin_nontemporal_store(v, dst + j * L + rl);
    }
  } else {
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
      const int e = j * L + rl;
      const int64_t i = g + e;
      if (i >= 0 && i < n) y[i] = buf[(e / N) * RUN + (e % N)];
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------ kernel

struct FiltArgs {
  int64_t n;
  int32_t K;
  int32_t stride;
  int64_t tile;             // samples per tile, a multiple of the group (16 N)
  int64_t warm;             // run-in samples before each tile, a multiple of the group
  int64_t ntiles;
  double gain;
};

constexpr int kWavesPerBlock = 4;

template <int N, typename TI, int L = kL>
__host__ __device__ constexpr int stage_bytes() {
  return kWavesPerBlock * Stage<N, TI, L>::ELEMS * (int)sizeof(TI);
}
// Boundary values per row: the raw input's (x[-2], x[-1]), then every
// section's (y[-2], y[-1]).
__host__ __device__ constexpr int state_elems(int K) { return 2 + 2 * K; }
template <int N, typename TI, typename T, int L = kL>
__host__ __device__ constexpr int lds_bytes(int K) {
  return stage_bytes<N, TI, L>() + kWavesPerBlock * (64 / L) * state_elems(K) * (int)sizeof(T);
}

// One wavefront filters four tiles, one per row: row r's tile starts at
// sample t0 (per lane row).  The row first runs the cascade from zero state
// over the `warm` samples that precede its tile (its carry-in: after `warm`
// samples the cascade state no longer depends, to the working precision, on
// anything earlier), then filters the tile, chaining groups through each
// section's boundary values.  All four rows run the same number of groups;
// samples outside [0, n) are zeros and are not stored.  `aligned`: x and y
// are 16-byte aligned, so whole groups may use vector loads and stores.
//
// SOLVER: SOS_PH or SOS_CR when every section uses that solver (no branch
// in the section loop), SOS_AUTO for a per-section choice.
template <int N, typename TI, typename T, bool B0ONE, int SOLVER, int L = kL>
__device__ __forceinline__ void filter_rows(const TI *__restrict__ x, TI *__restrict__ y,
                                            ctab<T> tab, const int32_t *__restrict__ solver,
                                            int64_t n, int K,
                                            int stride, int64_t t0, int64_t warm, int64_t tile,
                                            bool aligned, T gain, T *st, TI *buf) {
  for (int i = 0; i < state_elems(K); ++i) st[i] = T(0);   // the row's lanes write the same value
  const int64_t G = (int64_t)N * L;
  const int64_t warm_groups = warm / G, steps = warm_groups + tile / G;
  T X[N];
  for (int64_t it = 0; it < steps; ++it) {
    const int64_t g = t0 - warm + it * G;
    const bool full = aligned && __builtin_amdgcn_ballot_w64(!(g >= 0 && g + G <= n)) == 0;
    load_group<N, TI, T, L>(X, x, g, n, full, buf);
    T xs2 = st[0], xs1 = st[1];
    st[0] = last_of_row<L>(X[N - 2]);
    st[1] = last_of_row<L>(X[N - 1]);
    if constexpr (SOLVER == SOS_PH && N >= 128) {
      // a run that needs the accumulation registers: one pass per section
      T pr = T(0), qr = T(0);
      ph_fused_section<N, T, B0ONE, true, L>(X, tab, tab, pr, qr, xs2, xs1, st + 2);
      for (int k = 1; k < K; ++k) {
        const ctab<T> c = tab + (int64_t)k * stride;
        ph_fused_section<N, T, B0ONE, false, L>(X, c, c - stride, pr, qr, xs2, xs1, st + 2 + 2 * k);
      }
      if (it >= warm_groups) ph_last_correction<N, T>(X, tab + (int64_t)(K - 1) * stride, pr, qr);
    } else {
      for (int k = 0; k < K; ++k) {
        const ctab<T> c = tab + (int64_t)k * stride;
        if (SOLVER == SOS_CR || (SOLVER == SOS_AUTO && solver[k] == SOS_CR))
          cr_section<N, T, B0ONE, L>(X, c, xs2, xs1, st + 2 + 2 * k);
        else
          ph_section<N, T, B0ONE, L>(X, c, xs2, xs1, st + 2 + 2 * k);
      }
    }
    if (it >= warm_groups) store_group<N, TI, T, L>(X, y, g, n, full, gain, buf);
  }
}

// Single signal: tile t = [t*tile, (t+1)*tile) is filtered by row (t mod 4)
// of wavefront t / 4.
//
// The pointers are separate restrict-qualified arguments so that the
// compiler may read the coefficient table (uniform addresses, never
// written here) through the scalar cache.
template <int N, typename TI, typename T, bool B0ONE, int SOLVER, int L = kL>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_kernel(
    const TI *__restrict__ x, TI *__restrict__ y, const T *__restrict__ tab,
    const int32_t *__restrict__ solver, FiltArgs a) {
  constexpr int R = 64 / L;   // rows (tiles) per wave
  // dynamic LDS: the staging buffers, then the boundary values of every
  // section of every row (sized for the plan's K at launch)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  TI *stage = reinterpret_cast<TI *>(smem);
  T *state = reinterpret_cast<T *>(smem + stage_bytes<N, TI, L>());
  // the wave index is uniform across the wave; say so, so that everything
  // derived from it stays in scalar registers
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wave * R >= a.ntiles) return;   // uniform per wave
  const int row = lane_id() / L;
  const int64_t t0 = (wave * R + row) * a.tile;   // this row's tile
  T *st = state + (int64_t)(w * R + row) * state_elems(a.K);
  TI *buf = stage + (w * R + row) * Stage<N, TI, L>::ROWBUF;
  filter_rows<N, TI, T, B0ONE, SOLVER, L>(x, y, as_ctab(tab), solver, a.n, a.K, a.stride, t0, a.warm, a.tile,
                                          true, (T)a.gain, st, buf);
}

// Batched ragged channels.  Each channel c has its own plan (K, tables, b0
// gain), length and offset into the concatenated x and y.  Its tiles are
// taken four at a time as wave items; item i belongs to channel
// item_chan[i], and the channels are ordered so that costly items come
// first.
struct BatchChan {
  const void *tab;          // the channel plan's device table (compute dtype; block filtering: its block table)
  const int32_t *solver;    // device [K]
  const void *aop;          // block filtering: the MFMA A operands of the channel's Toeplitz products
  int64_t off, n;           // first sample in x / y, length
  int64_t tile, warm;       // samples per row tile and of run-in (multiples of the group)
  int64_t first_item;       // the channel's first wave item
  int32_t K, stride;
  double gain;
  int32_t shift;            // (off mod samples per 16 bytes): the tiles cover [-shift, n)
  int32_t mix;              // SOS_CR / SOS_PH when every section uses it, else SOS_AUTO
};

// hdr: the batch's device header, hdr[0] the live item count (the grid is
// sized for the batch's room, so that one launch, captured once, serves
// every channel set the batch is replanned to).
template <int N, typename TI, typename T, bool B0ONE, int SOLVER, int L = kL>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_rows_batched_kernel(
    const TI *__restrict__ x, TI *__restrict__ y, const BatchChan *__restrict__ chans,
    const int32_t *__restrict__ item_chan, const int64_t *__restrict__ hdr, int32_t kmax) {
  constexpr int R = 64 / L;   // rows (tiles) per wave
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  TI *stage = reinterpret_cast<TI *>(smem);
  T *state = reinterpret_cast<T *>(smem + stage_bytes<N, TI, L>());
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (item >= hdr[0]) return;   // uniform per wave
  const BatchChan &ch = chans[item_chan[item]];
  const int64_t quad = item - ch.first_item;
  // the tiles cover [-shift, n), so that with x and y 16-byte aligned every
  // group starts on a 16-byte boundary; samples before 0 read as zeros and
  // are not stored
  const int64_t ntiles = (ch.n + ch.shift + ch.tile - 1) / ch.tile;
  const int row = lane_id() / L;
  const int64_t t0 = (quad * R + row) * ch.tile - ch.shift;
  // rows past the channel's end idle; the run-in never reaches before the
  // channel's start (the state there is zero)
  const int64_t last = (quad * R + R - 1 < ntiles - 1 ? quad * R + R - 1 : ntiles - 1);
  const int64_t warm = ch.warm < last * ch.tile ? ch.warm : last * ch.tile;
  T *st = state + (int64_t)(w * R + row) * state_elems(kmax);
  TI *buf = stage + (w * R + row) * Stage<N, TI, L>::ROWBUF;
  const ctab<T> tab = as_ctab(static_cast<const T *>(ch.tab));
#define SOSF_BATCH_ROWS(S)                                                                       \
  filter_rows<N, TI, T, B0ONE, S, L>(x + ch.off, y + ch.off, tab, ch.solver, ch.n, ch.K, ch.stride, t0, warm, \
                                     ch.tile, true, (T)ch.gain, st, buf)
  if (SOLVER != SOS_AUTO) {
    SOSF_BATCH_ROWS(SOLVER);
  } else {
    // channels of several classes: one uniform branch per wavefront to the
    // code specialised for this channel's class, so that a channel whose
    // sections all use one solver runs without a per-section branch
    const int mix = __builtin_amdgcn_readfirstlane(ch.mix);
    if (mix == SOS_CR) SOSF_BATCH_ROWS(SOS_CR);
    else if (mix == SOS_PH) SOSF_BATCH_ROWS(SOS_PH);
    else SOSF_BATCH_ROWS(SOS_AUTO);
  }
#undef SOSF_BATCH_ROWS
}

}  // namespace sosf
