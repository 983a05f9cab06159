// Device code: one 64-wide wavefront filters one tile of the signal through
// all K sections, one signal block group of N*64 samples at a time.
//
// Layout (Section V): lane l holds the l-th run of N consecutive samples of
// the group in registers X[0..N-1], i.e. X[m] on lane l is x[m + l N], the
// l-th element of the stride-N block xbar_m.  A lane shift by one (lane l
// receives lane l-1, lane 0 receives a fill value) is the shift matrix R.
// The layout is kept across all K sections (Section VII-B): one
// permutation on load, one de-permutation on store.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.hpp"

namespace sosf {

// ------------------------------------------------------------ lane moves

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// R applied to a register: out[l] = v[l-1], out[0] = fill.  DPP wave_shr:1
// with bound_ctrl writes 0 into lane 0; the fill is merged afterwards.
__device__ __forceinline__ float shift_r(float v, float fill) {
  int r = __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true);
  return lane_id() == 0 ? fill : __int_as_float(r);
}
__device__ __forceinline__ double shift_r(double v, double fill) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, 0x138, 0xf, 0xf, true);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), 0x138, 0xf, 0xf, true);
  double r = __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
  return lane_id() == 0 ? fill : r;
}

// Lane shift by d >= 2 with zeros entering lanes 0..d-1 (ds_bpermute).
__device__ __forceinline__ float shift_d(float v, int d) {
  int l = lane_id();
  int r = __builtin_amdgcn_ds_bpermute(((l - d) & 63) << 2, __float_as_int(v));
  return l >= d ? __int_as_float(r) : 0.0f;
}
__device__ __forceinline__ double shift_d(double v, int d) {
  int l = lane_id();
  int addr = ((l - d) & 63) << 2;
  uint64_t b = (uint64_t)__double_as_longlong(v);
  int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)b);
  int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(b >> 32));
  double r = __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
  return l >= d ? r : 0.0;
}
template <typename T>
__device__ __forceinline__ T shift_any(T v, int d) {
  return d == 1 ? shift_r(v, T(0)) : shift_d(v, d);
}

// Value of lane 63 in every lane.
__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double lane63(double v) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Log-depth solve across the 64 lanes of z_l = A z_{l-1} + z_l (z_{-1} = 0)
// for 2-vectors z = (p, q): Kogge-Stone doubling, round j adds A^(2^j) times
// the value 2^j lanes below.  pw holds A^(2^j) row-major for j = 0..5.
template <typename T>
__device__ __forceinline__ void lane_scan_2x2(T &p, T &q, const T *__restrict__ pw) {
#pragma unroll
  for (int j = 0; j < kLogLanes; ++j) {
    const int d = 1 << j;
    const T m00 = pw[4 * j], m01 = pw[4 * j + 1], m10 = pw[4 * j + 2], m11 = pw[4 * j + 3];
    T ps = shift_any(p, d);
    T qs = shift_any(q, d);
    T np = __builtin_fma(m00, ps, __builtin_fma(m01, qs, p));
    T nq = __builtin_fma(m10, ps, __builtin_fma(m11, qs, q));
    p = np;
    q = nq;
  }
}

// ------------------------------------------------------------ one section

// Per-section boundary values carried from group to group (Section V):
// st[0] = x[-2], st[1] = x[-1], st[2] = y[-2], st[3] = y[-1].

// Non-recursive stage, eq. feedforward_block_uniform: v_m = b0 x_m +
// b1 x_{m-1} + b2 x_{m-2} with the extended blocks x_{-1} = R x_{N-1} +
// e0 x[-1], x_{-2} = R x_{N-2} + e0 x[-2]; then the previous group's outputs
// enter the first element of blocks 0 and 1.
template <int N, typename T, bool B0ONE>
__device__ __forceinline__ void nonrecursive(T (&X)[N], const T *__restrict__ c, T *st) {
  const T b0 = c[OFF_B0], b1 = c[OFF_B1], b2 = c[OFF_B2];
  const T a1 = c[OFF_A1], a2 = c[OFF_A2];
  const T xs2 = st[0], xs1 = st[1], ys2 = st[2], ys1 = st[3];
  const T nx2 = lane63(X[N - 2]), nx1 = lane63(X[N - 1]);
  const T xm1 = shift_r(X[N - 1], xs1);
  const T xm2 = shift_r(X[N - 2], xs2);
#pragma unroll
  for (int m = N - 1; m >= 2; --m) {
    T acc = B0ONE ? X[m] : b0 * X[m];
    acc = __builtin_fma(b1, X[m - 1], acc);
    X[m] = __builtin_fma(b2, X[m - 2], acc);
  }
  {
    T acc = B0ONE ? X[1] : b0 * X[1];
    acc = __builtin_fma(b1, X[0], acc);
    X[1] = __builtin_fma(b2, xm1, acc);
    acc = B0ONE ? X[0] : b0 * X[0];
    acc = __builtin_fma(b1, xm1, acc);
    X[0] = __builtin_fma(b2, xm2, acc);
  }
  const bool l0 = lane_id() == 0;
  const T c0 = __builtin_fma(a1, ys1, a2 * ys2);
  const T c1 = a2 * ys1;
  X[0] -= l0 ? c0 : T(0);
  X[1] -= l0 ? c1 : T(0);
  st[0] = nx2;
  st[1] = nx1;
}

// PH factorisation (Section VI-B).
template <int N, typename T>
__device__ __forceinline__ void ph_solve(T (&X)[N], const T *__restrict__ c, T *st) {
  const T a1 = c[OFF_A1], a2 = c[OFF_A2];
  // step 1, eq. particular_recurrence: every lane runs the zero-state
  // recurrence over its own N samples
  X[1] = __builtin_fma(-a1, X[0], X[1]);
#pragma unroll
  for (int m = 2; m < N; ++m) X[m] = __builtin_fma(-a2, X[m - 2], __builtin_fma(-a1, X[m - 1], X[m]));
  // step 2, eq. recursive_doubling_equation: y_e[l] = w_e[l] - C y_e[l-1]
  // over the lanes, with y_e[l] = (y[(l+1)N-2], y[(l+1)N-1])
  T p = X[N - 2], q = X[N - 1];
  lane_scan_2x2(p, q, c + OFF_PH_POW);
  X[N - 2] = p;
  X[N - 1] = q;
  // step 3, eq. PH_forward: the homogeneous correction from the true
  // terminal values of the preceding lane (R y_{N-2}, R y_{N-1})
  const T pr = shift_r(p, T(0)), qr = shift_r(q, T(0));
  const T *__restrict__ u1 = c + OFF_U1;
  const T *__restrict__ u2 = c + OFF_U1 + N;
#pragma unroll
  for (int m = 0; m < N - 2; ++m) X[m] = __builtin_fma(-u2[m], pr, __builtin_fma(-u1[m], qr, X[m]));
  st[2] = lane63(p);
  st[3] = lane63(q);
}

// Cyclic reduction (Section VI-C).  Level i works on the blocks m = s(j+1)-1
// (s = 2^i, j = 0..N/s-1); even j are eliminated, odd j retained.  A
// reference below j = 0 wraps to the last blocks through R.
template <int N, typename T>
__device__ __forceinline__ void cr_solve(T (&X)[N], const T *__restrict__ c, T *st) {
  constexpr int LG = __builtin_ctz(N);
  // reduction, eq. cr_coeff_update coefficients per level
#pragma unroll
  for (int i = 0; i < LG; ++i) {
    const int s = 1 << i, ni = N >> i;
    const T fe = c[OFF_CR_LVL + 4 * i], e = c[OFF_CR_LVL + 4 * i + 1];
    const T wrap = shift_r(X[N - 1], T(0));
#pragma unroll
    for (int j = 0; j < ni; j += 2) {
      const int m = s * (j + 1) - 1;
      X[m] = __builtin_fma(-fe, j == 0 ? wrap : X[m - s], X[m]);
    }
#pragma unroll
    for (int j = 1; j < ni; j += 2) {
      const int m = s * (j + 1) - 1;
      X[m] = __builtin_fma(-e, X[m - s], X[m]);
    }
  }
  // terminal block, eq. cr_terminal_block: (I + e R + f R^2) y = v' on block
  // N-1, a second-order recurrence over the lanes; solved by the log-depth
  // scan of z_l = (y_{l-1}, y_l) = T z_{l-1} + (0, v'_l)
  {
    T p = T(0), q = X[N - 1];
    lane_scan_2x2(p, q, c + OFF_CR_POW);
    X[N - 1] = q;
  }
  // back substitution, eqs. cr_companion_block .. cr_backsub_final
  const T r1 = shift_r(X[N - 1], T(0));   // R y_{N-1}, reused at every level
#pragma unroll
  for (int i = LG - 1; i >= 0; --i) {
    const int s = 1 << i, ni = N >> i;
    const T cc = c[OFF_CR_LVL + 4 * i + 2], dd = c[OFF_CR_LVL + 4 * i + 3];
    T w3;   // the once-wrapped block for j = 0
    if (ni == 2) w3 = shift_r(r1, T(0));                 // R^2 y_{N-1}
    else w3 = shift_r(X[N - 2 * s - 1], T(0));           // R y at position ni-3
#pragma unroll
    for (int j = 0; j < ni; j += 2) {
      const int m = s * (j + 1) - 1;
      const T y1 = (j >= 1) ? X[m - s] : r1;
      const T y3 = (j >= 3) ? X[m - 3 * s] : (j == 0 ? w3 : r1);
      X[m] = __builtin_fma(-cc, y1, __builtin_fma(-dd, y3, X[m]));
    }
  }
  st[2] = lane63(X[N - 2]);
  st[3] = lane63(X[N - 1]);
}

// ------------------------------------------------------------ memory

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));

template <int N, typename TI, typename T>
__device__ __forceinline__ void load_group(T (&X)[N], const TI *__restrict__ x, int64_t g,
                                           int64_t n) {
  const int64_t base = g + (int64_t)lane_id() * N;
  if (g + (int64_t)N * kLanes <= n) {
    if constexpr (sizeof(TI) == 4) {
      const vf4 *p = reinterpret_cast<const vf4 *>(x + base);
#pragma unroll
      for (int j = 0; j < N / 4; ++j) {
        vf4 v = __builtin_nontemporal_load(p + j);
        X[4 * j] = T(v.x); X[4 * j + 1] = T(v.y); X[4 * j + 2] = T(v.z); X[4 * j + 3] = T(v.w);
      }
    } else {
      const vd2 *p = reinterpret_cast<const vd2 *>(x + base);
#pragma unroll
      for (int j = 0; j < N / 2; ++j) {
        vd2 v = __builtin_nontemporal_load(p + j);
        X[2 * j] = T(v.x); X[2 * j + 1] = T(v.y);
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const int64_t i = base + m;
      X[m] = (i < n) ? T(x[i]) : T(0);
    }
  }
}

template <int N, typename TI, typename T>
__device__ __forceinline__ void store_group(const T (&X)[N], TI *__restrict__ y, int64_t g,
                                            int64_t n, T gain) {
  const int64_t base = g + (int64_t)lane_id() * N;
  if (g + (int64_t)N * kLanes <= n) {
    if constexpr (sizeof(TI) == 4) {
      vf4 *p = reinterpret_cast<vf4 *>(y + base);
#pragma unroll
      for (int j = 0; j < N / 4; ++j) {
        vf4 v;
        v.x = (float)(X[4 * j] * gain); v.y = (float)(X[4 * j + 1] * gain);
        v.z = (float)(X[4 * j + 2] * gain); v.w = (float)(X[4 * j + 3] * gain);
        __builtin_nontemporal_store(v, p + j);
      }
    } else {
      vd2 *p = reinterpret_cast<vd2 *>(y + base);
#pragma unroll
      for (int j = 0; j < N / 2; ++j) {
        vd2 v;
        v.x = (double)(X[2 * j] * gain); v.y = (double)(X[2 * j + 1] * gain);
        __builtin_nontemporal_store(v, p + j);
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const int64_t i = base + m;
      if (i < n) y[i] = (TI)(X[m] * gain);
    }
  }
}

// ------------------------------------------------------------ kernel

struct FiltArgs {
  int64_t n;
  int32_t K;
  int32_t stride;
  int64_t tile;             // samples per tile, multiple of N*64
  int64_t warm;             // run-in samples before each tile, multiple of N*64
  int64_t ntiles;
  double gain;
};

constexpr int kWavesPerBlock = 4;

// One wavefront per tile [t*tile, (t+1)*tile).  The wave first runs the
// cascade from zero state over the `warm` samples that precede the tile
// (its carry-in: the cascade state after `warm` samples no longer depends,
// to the working precision, on anything earlier), then filters the tile,
// chaining groups by each section's boundary values.
//
// The pointers are separate restrict-qualified arguments so that the
// compiler may read the coefficient table (uniform addresses, never
// written here) through the scalar cache.
template <int N, typename TI, typename T, bool B0ONE>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_tiles_kernel(
    const TI *__restrict__ x, TI *__restrict__ y, const T *__restrict__ tab,
    const int32_t *__restrict__ solver, FiltArgs a) {
  __shared__ T state[kWavesPerBlock][SOS_MAX_SECTIONS][4];
  // the wave index is uniform across the wave; say so, so that everything
  // derived from it (tile bounds, table addresses) stays in scalar registers
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (tile >= a.ntiles) return;   // uniform per wave
  T(*st)[4] = state[w];
  for (int i = 0; i < a.K * 4; ++i) st[i >> 2][i & 3] = T(0);   // every lane writes the same value
  const int64_t t0 = tile * a.tile;
  const int64_t t1 = (t0 + a.tile < a.n) ? t0 + a.tile : a.n;
  const int64_t NL = (int64_t)N * kLanes;
  const T gain = (T)a.gain;
  T X[N];
  for (int64_t g = (t0 > a.warm ? t0 - a.warm : 0); g < t1; g += NL) {
    load_group<N, TI, T>(X, x, g, a.n);
    for (int k = 0; k < a.K; ++k) {
      const T *__restrict__ c = tab + (int64_t)k * a.stride;
      nonrecursive<N, T, B0ONE>(X, c, st[k]);
      if (solver[k] == SOS_CR) cr_solve<N, T>(X, c, st[k]);
      else ph_solve<N, T>(X, c, st[k]);
    }
    if (g >= t0) store_group<N, TI, T>(X, y, g, a.n, gain);
  }
}

}  // namespace sosf
