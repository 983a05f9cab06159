// Host side of the plan: coefficient validation and normalisation, the FP64
// tables of the PH factorisation and of cyclic reduction, the CR guard, and
// the cascade's state transition that fixes the tile run-in length.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.hpp"

namespace sosf {
namespace {

struct Mat2 { double a, b, c, d; };   // [[a, b], [c, d]]

Mat2 mul(const Mat2 &x, const Mat2 &y) {
  return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d,
          x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}

// u_{1,m}, u_{2,m} (Section VI-A): u_{2,0} = a2, u_{1,0} = a1,
// u_{2,1} = -a1 a2, u_{1,1} = a2 - a1^2, u_{l,m} = -a2 u_{l,m-2} - a1 u_{l,m-1}.
void u_tables(double a1, double a2, int N, double *u1, double *u2) {
  u2[0] = a2;
  u1[0] = a1;
  if (N > 1) {
    u2[1] = -a1 * a2;
    u1[1] = a2 - a1 * a1;
  }
  for (int m = 2; m < N; ++m) {
    u1[m] = -a2 * u1[m - 2] - a1 * u1[m - 1];
    u2[m] = -a2 * u2[m - 2] - a1 * u2[m - 1];
  }
}

double inf_norm(const std::vector<double> &M, int n) {
  double best = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += std::fabs(M[i * n + j]);
    if (s > best) best = s;
  }
  return best;
}

std::vector<double> matmul(const std::vector<double> &A, const std::vector<double> &B, int n) {
  std::vector<double> C(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double a = A[i * n + k];
      if (a == 0.0) continue;
      for (int j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
    }
  return C;
}

}  // namespace

sos_status build_plan_tables(sos_plan_s &p, const double *sos) {
  const int K = p.K, N = p.N;
  // 1. validation and a0 normalisation (eq. complex_second_order)
  std::vector<double> nrm(K * 5);
  for (int k = 0; k < K; ++k) {
    const double *r = sos + 6 * k;
    for (int j = 0; j < 6; ++j)
      if (!std::isfinite(r[j])) return SOS_E_COEF;
    double a0 = r[3];
    if (a0 == 0.0) return SOS_E_COEF;
    double b0 = r[0] / a0, b1 = r[1] / a0, b2 = r[2] / a0, a1 = r[4] / a0, a2 = r[5] / a0;
    if (!(std::fabs(a2) < 1.0 && std::fabs(a1) < 1.0 + a2)) return SOS_E_UNSTABLE;
    double *o = &nrm[5 * k];
    o[0] = b0; o[1] = b1; o[2] = b2; o[3] = a1; o[4] = a2;
  }
  // 2. b0 factoring (eq. simple_second_order) when it keeps every
  //    intermediate scale within range of the compute dtype
  const double lim = (p.compute_dtype == SOS_F64) ? 0x1p400 : 0x1p60;
  bool factor = true;
  double run = 1.0;
  for (int k = 0; k < K && factor; ++k) {
    double b0 = nrm[5 * k];
    if (b0 == 0.0) { factor = false; break; }
    run /= b0;
    if (!(std::fabs(run) < lim && std::fabs(run) > 1.0 / lim)) factor = false;
  }
  p.b0_factored = factor;
  p.gain = 1.0;
  p.rows = nrm;
  p.rows_norm = nrm;
  p.a0.resize(K);
  for (int k = 0; k < K; ++k) p.a0[k] = sos[6 * k + 3];
  if (factor) {
    for (int k = 0; k < K; ++k) {
      double *o = &p.rows[5 * k];
      p.gain *= o[0];
      o[1] /= o[0];
      o[2] /= o[0];
      o[0] = 1.0;
    }
  }
  // 3. per-section tables
  p.stride = tab_stride(N);
  p.table.assign((size_t)K * p.stride, 0.0);
  p.solver.assign(K, SOS_PH);
  p.C.assign(K * 4, 0.0);
  p.cr_term.assign(K * 2, 0.0);
  const double tau = 64.0;          // CR guard on |f/e|, |c|, |d|
  const double flush = 0x1p-60;     // r^(2^i) below this: level decoupled
  for (int k = 0; k < K; ++k) {
    const double *o = &p.rows[5 * k];
    double *t = &p.table[(size_t)k * p.stride];
    const double a1 = o[3], a2 = o[4];
    t[OFF_B0] = o[0]; t[OFF_B1] = o[1]; t[OFF_B2] = o[2];
    t[OFF_A1] = a1; t[OFF_A2] = a2;
    // PH: u tables, C = [[e, g], [f, d]] = [[u2(N-2), u1(N-2)], [u2(N-1), u1(N-1)]]
    double *u1 = t + OFF_U1, *u2 = t + off_u2(N);
    u_tables(a1, a2, N, u1, u2);
    Mat2 C{u2[N - 2], u1[N - 2], u2[N - 1], u1[N - 1]};
    p.C[4 * k + 0] = C.a; p.C[4 * k + 1] = C.b; p.C[4 * k + 2] = C.c; p.C[4 * k + 3] = C.d;
    // terminal-block scan y_e[l] = w_e[l] - C y_e[l-1] with powers of A = -C
    Mat2 A{-C.a, -C.b, -C.c, -C.d};
    for (int j = 0; j < kMaxLogL; ++j) {
      double *q = t + OFF_PH_POW + 4 * j;
      q[0] = A.a; q[1] = A.b; q[2] = A.c; q[3] = A.d;
      A = mul(A, A);
    }
    // CR: eq. cr_coeff_update, with the flush and the guard
    // largest pole magnitude of 1 + a1 z^-1 + a2 z^-2; at level i the reduced
    // polynomial has the poles raised to the power 2^i
    double disc = a1 * a1 - 4.0 * a2, rho = 0.0;
    if (disc < 0.0) rho = std::sqrt(a2);
    else rho = std::max(std::fabs(-a1 + std::sqrt(disc)), std::fabs(-a1 - std::sqrt(disc))) * 0.5;
    double e = a1, f = a2;
    bool cr_ok = true, flushed = false;
    for (int i = 0; i < p.lgN; ++i) {
      double *q = t + OFF_CR_LVL + 4 * i;
      if (flushed || rho < flush) flushed = true;
      rho = rho * rho;
      if (flushed) {
        q[0] = q[1] = q[2] = q[3] = 0.0;
        e = f = 0.0;
        continue;
      }
      if (e == 0.0) { cr_ok = false; q[0] = q[1] = q[2] = q[3] = 0.0; e = 2 * f; f = f * f; continue; }
      double fe = f / e, c = e - f / e, d = -f * f / e;
      if (!(std::fabs(fe) <= tau && std::fabs(c) <= tau && std::fabs(d) <= tau)) cr_ok = false;
      q[0] = fe; q[1] = e; q[2] = c; q[3] = d;
      double en = 2 * f - e * e, fn = f * f;
      e = en;
      f = fn;
    }
    if (flushed || rho < flush) { e = 0.0; f = 0.0; }
    p.cr_term[2 * k] = e;
    p.cr_term[2 * k + 1] = f;
    Mat2 T{0.0, 1.0, -f, -e};
    for (int j = 0; j < kMaxLogL; ++j) {
      double *q = t + OFF_CR_POW + 4 * j;
      q[0] = T.a; q[1] = T.b; q[2] = T.c; q[3] = T.d;
      T = mul(T, T);
    }
    // AUTO takes PH: on MI355X it is the faster of the two at every N (1-8%
    // ahead at N = 4 .. 64, 17% at N = 128, several times with the runs in
    // the workspace), and it needs no guard.  CR is used where asked for
    // and the guard allows it.  (Where the runs live in the workspace, AUTO
    // plans take the deferred-correction PH instead, chosen at plan
    // creation.)
    p.solver[k] = (p.solver_opt == SOS_CR && cr_ok) ? SOS_CR : SOS_PH;
  }
  // 4. cascade state s = (y_1[n-2], y_1[n-1], ..., y_K[n-2], y_K[n-1]) in the
  //    scaled domain the kernels use; one step with zero raw input.
  const int D = 2 * K;
  p.phi.assign((size_t)D * D, 0.0);
  for (int col = 0; col < D; ++col) {
    std::vector<double> s(D, 0.0), s2(D, 0.0);
    s[col] = 1.0;
    double in_prev2 = 0.0, in_prev1 = 0.0, in_now = 0.0;   // raw input is zero
    for (int k = 0; k < K; ++k) {
      const double *o = &p.rows[5 * k];
      double y2 = s[2 * k], y1 = s[2 * k + 1];
      double yn = o[0] * in_now + o[1] * in_prev1 + o[2] * in_prev2 - o[3] * y1 - o[4] * y2;
      s2[2 * k] = y1;
      s2[2 * k + 1] = yn;
      in_prev2 = y2; in_prev1 = y1; in_now = yn;   // this section's output feeds the next
    }
    for (int row = 0; row < D; ++row) p.phi[(size_t)row * D + col] = s2[row];
  }
  // 5. run-in length W: smallest W (to a power-of-two search) with
  //    ||Phi^W||_inf below eps; rounded up to whole groups.  eps sits 2^16
  //    below the unit roundoff of what is stored (FP32: 2^-24) and 2^-64
  //    for FP64 throughout, so a tile's truncated history stays far below
  //    the rounding of its own outputs.
  const double eps = p.runin_eps > 0.0                                            ? p.runin_eps
                     : (p.compute_dtype == SOS_F64 && p.io_dtype == SOS_F64) ? 0x1p-64
                                                                             : 0x1p-40;
  std::vector<std::vector<double>> pw;   // Phi^(2^j)
  pw.push_back(p.phi);
  int64_t w = 1;
  while (inf_norm(pw.back(), D) >= eps && w < ((int64_t)1 << 40)) {
    pw.push_back(matmul(pw.back(), pw.back(), D));
    w <<= 1;
  }
  // binary refinement below the first power of two that meets eps
  int64_t lo = 0;
  std::vector<double> acc;   // Phi^lo (empty = identity)
  for (int j = (int)pw.size() - 2; j >= 0; --j) {
    std::vector<double> cand = acc.empty() ? pw[j] : matmul(acc, pw[j], D);
    if (inf_norm(cand, D) >= eps) {
      acc = cand;
      lo += (int64_t)1 << j;
    }
  }
  int64_t W = lo + 1;
  const int64_t NL = (int64_t)N * p.L;
  p.warm = ((W + NL - 1) / NL) * NL;
  // the norm over the rounded length, for reporting
  {
    std::vector<double> r;
    int64_t rem = p.warm;
    std::vector<double> base = p.phi;
    bool have = false;
    for (int j = 0; rem && j < 62; ++j) {
      if (rem & 1) {
        r = have ? matmul(r, base, D) : base;
        have = true;
      }
      rem >>= 1;
      if (rem) base = matmul(base, base, D);
    }
    p.warm_norm = have ? inf_norm(r, D) : 1.0;
  }
  return SOS_OK;
}

// Tables of the deferred homogeneous correction.  Inside a group each lane
// runs the whole cascade from zero state over its N samples (raw input
// history taken from the data); the true output is that zero-state output
// plus the response to the segment's entry state, the 2K values
// (y_j[-2], y_j[-1]) of every section j.  A unit entry component of section
// j sets y_j's history and, because x_{j+1} = y_j, x_{j+1}'s history too.
//   theta[m][2j+c]      response of the last section at block m (m < N)
//   coupling(j, k)[t][c] response of section k at block N-2+t, for j < k
// (the diagonal blocks j = k are -C of the PH factorisation).
void build_deferred_tables(sos_plan_s &p) {
  const int K = p.K, N = p.N, D = 2 * K;
  p.kb = (D + 3) / 4;
  p.theta.assign((size_t)N * D, 0.0);
  p.coupling.assign((size_t)2 * K * (K - 1), 0.0);
  std::vector<double> out((size_t)K * N);
  for (int col = 0; col < D; ++col) {
    const int j = col / 2, c = col % 2;
    std::vector<double> xh(2 * K, 0.0), yh(2 * K, 0.0);   // (x[-2], x[-1]), (y[-2], y[-1])
    yh[2 * j + c] = 1.0;
    if (j + 1 < K) xh[2 * (j + 1) + c] = 1.0;
    for (int k = 0; k < K; ++k) {
      const double *o = &p.rows[5 * k];
      double x2 = xh[2 * k], x1 = xh[2 * k + 1], y2 = yh[2 * k], y1 = yh[2 * k + 1];
      for (int m = 0; m < N; ++m) {
        const double in = (k == 0) ? 0.0 : out[(size_t)(k - 1) * N + m];
        const double v = o[0] * in + o[1] * x1 + o[2] * x2 - o[3] * y1 - o[4] * y2;
        x2 = x1; x1 = in; y2 = y1; y1 = v;
        out[(size_t)k * N + m] = v;
      }
    }
    for (int m = 0; m < N; ++m) p.theta[(size_t)m * D + col] = out[(size_t)(K - 1) * N + m];
    for (int k = j + 1; k < K; ++k) {
      double *blk = &p.coupling[4 * ((size_t)k * (k - 1) / 2 + j)];
      blk[0 * 2 + c] = out[(size_t)k * N + N - 2];
      blk[1 * 2 + c] = out[(size_t)k * N + N - 1];
    }
  }
  // MFMA A operand (16 x 4 FP64 tile, lane l holds A[l % 16][l / 16]) for
  // each 16-block of m and 4-block of state components, zero-padded to the
  // kernel's compile-time block count (2, 4 or 8)
  const int MB = N / 16;
  const int kbm = K <= 4 ? 2 : (K <= 8 ? 4 : 8);
  p.kb = kbm;
  p.theta_mfma.assign((size_t)(MB > 0 ? MB : 0) * kbm * 64, 0.0);
  for (int mb = 0; mb < MB; ++mb)
    for (int b = 0; b < kbm; ++b)
      for (int l = 0; l < 64; ++l) {
        const int m = 16 * mb + l % 16, comp = 4 * b + l / 16;
        p.theta_mfma[((size_t)mb * kbm + b) * 64 + l] = comp < D ? p.theta[(size_t)m * D + comp] : 0.0;
      }
}

}  // namespace sosf
