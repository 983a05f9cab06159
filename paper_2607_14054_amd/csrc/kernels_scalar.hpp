// Scalar filtering: the plain recurrence of Sec. II (eq.
// general_cascaded_equation), one lane per segment.  The comparison point the
// paper calls scalar filtering (Table overall_complexity): 4 FMA per sample
// and section with b0 factored out, no parallelism inside a segment.
//
// Each lane owns one contiguous segment of the signal and runs the whole
// cascade over it sample by sample, after a run-in of W samples from zero
// state (the same carry rule as the tile kernels).  A wavefront's 64
// segments move through LDS in chunks of 32 samples, so that global accesses
// stay 16-byte vectors: eight lanes cover one segment's 128-byte chunk.
#pragma once

#include "kernels.hpp"

namespace sosf {

constexpr int kScalarChunk = 32;
constexpr int kScalarKMax = 16;

struct ScalarArgs {
  int64_t n;
  int64_t seg;       // samples per lane segment (multiple of the chunk)
  int64_t warm;      // run-in samples (multiple of the chunk)
  int64_t nseg;      // segments
  int32_t K, stride;
  double gain;
};

template <typename TI>
struct ScalarStage {
  static constexpr int V = Vec16<TI>::n;
  static constexpr int RUN = kScalarChunk + V;   // padded per-lane run
  static constexpr int ELEMS = 64 * RUN;         // per wavefront
};

// KMAX: compile-time bound on K, so that every section's state stays in
// registers.
template <typename TI, typename T, bool B0ONE, int KMAX>
__global__ __launch_bounds__(kWavesPerBlock * 64) void sos_scalar_kernel(const TI *__restrict__ x,
                                                                         TI *__restrict__ y,
                                                                         const T *__restrict__ tab,
                                                                         ScalarArgs a) {
  typedef typename Vec16<TI>::type VT;
  constexpr int C = kScalarChunk, V = ScalarStage<TI>::V, RUN = ScalarStage<TI>::RUN;
  constexpr int PER = C / V;   // vectors per segment chunk
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
  if (wave * 64 >= a.nseg) return;
  const int lane = lane_id();
  TI *buf = reinterpret_cast<TI *>(smem) + w * ScalarStage<TI>::ELEMS;
  const ctab<T> ct = as_ctab(tab);
  const T gain = (T)a.gain;
  // raw input state, then each section's output state (y[-2], y[-1])
  T st[2 + 2 * KMAX];
#pragma unroll
  for (int i = 0; i < 2 + 2 * KMAX; ++i) st[i] = T(0);
  const int64_t steps = (a.warm + a.seg) / C;
  T X[C];
  for (int64_t it = 0; it < steps; ++it) {
    const int64_t off = it * C - a.warm;   // chunk start relative to each segment start
    // cooperative load: vector f = lane + 64 v is part f % PER of segment f / PER
#pragma unroll
    for (int v = 0; v < PER; ++v) {
      const int f = lane + 64 * v, s = f / PER, part = f % PER;
      const int64_t gi = (wave * 64 + s) * a.seg + off + part * V;
      TI *dst = buf + s * RUN + part * V;
      if (gi >= 0 && gi + V <= a.n) {
        *reinterpret_cast<VT *>(dst) = __builtin_nontemporal_load(reinterpret_cast<const VT *>(x + gi));
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i) dst[i] = (gi + i >= 0 && gi + i < a.n) ? x[gi + i] : TI(0);
      }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < C; t += V) {
      const VT v = *reinterpret_cast<const VT *>(buf + lane * RUN + t);
#pragma unroll
      for (int i = 0; i < V; ++i) X[t + i] = T(v[i]);
    }
    __builtin_amdgcn_wave_barrier();
    T xp2 = st[0], xp1 = st[1];
    st[0] = X[C - 2];
    st[1] = X[C - 1];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < a.K) {
        const ctab<T> c = ct + (int64_t)k * a.stride;
        const T b0 = c[OFF_B0], b1 = c[OFF_B1], b2 = c[OFF_B2], a1 = c[OFF_A1], a2 = c[OFF_A2];
        const T oy2 = st[2 + 2 * k], oy1 = st[3 + 2 * k];
        T yp2 = oy2, yp1 = oy1;
#pragma unroll
        for (int t = 0; t < C; ++t) {
          const T xi = X[t];
          T v = B0ONE ? xi : b0 * xi;
          v = fma_(b1, xp1, v);
          v = fma_(b2, xp2, v);
          v = fma_(-a2, yp2, v);
          v = fma_(-a1, yp1, v);
          X[t] = v;
          xp2 = xp1;
          xp1 = xi;
          yp2 = yp1;
          yp1 = v;
        }
        st[2 + 2 * k] = yp2;
        st[3 + 2 * k] = yp1;
        // the next section's input state is this section's previous output
        xp2 = oy2;
        xp1 = oy1;
      }
    }
    if (off >= 0) {   // uniform: every segment is at the same offset
#pragma unroll
      for (int t = 0; t < C; t += V) {
        VT v;
#pragma unroll
        for (int i = 0; i < V; ++i) v[i] = (TI)(X[t + i] * gain);
        *reinterpret_cast<VT *>(buf + lane * RUN + t) = v;
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int v = 0; v < PER; ++v) {
        const int f = lane + 64 * v, s = f / PER, part = f % PER;
        const int64_t gi = (wave * 64 + s) * a.seg + off + part * V;
        const TI *src = buf + s * RUN + part * V;
        if (gi >= 0 && gi + V <= a.n) {
          __builtin_nontemporal_store(*reinterpret_cast<const VT *>(src), reinterpret_cast<VT *>(y + gi));
        } else {
#pragma unroll
          for (int i = 0; i < V; ++i)
            if (gi + i >= 0 && gi + i < a.n) y[gi + i] = src[i];
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

}  // namespace sosf
