// Internal plan structure and the per-section coefficient table layout that
// the host plan writes and the kernels read.
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/sosfilt.h"

namespace sosf {

constexpr int kL = 16;           // default block size L = lanes of one DPP row
constexpr int kLogL = 4;
constexpr int kRows = 4;         // independent blocks (rows) per 64-wide wavefront at L = 16
constexpr int kMaxLogL = 6;      // largest L is 64, a whole wavefront
constexpr int kMaxLevels = 10;   // log2 of the largest N the tables hold
constexpr int kBwdN = 16;        // N of the adjoint kernels
constexpr int kBwdRow = 8;       // doubles per section in the adjoint rows

// Offsets (in elements of the compute dtype) inside one section's row of the
// device table.  Row length = tab_stride(N).
enum : int {
  OFF_B0 = 0, OFF_B1 = 1, OFF_B2 = 2, OFF_A1 = 3, OFF_A2 = 4,
  OFF_PH_POW = 8,                              // 6 x 4: (-C)^(2^j), j < log2 L
  OFF_CR_POW = OFF_PH_POW + 4 * kMaxLogL,      // 6 x 4: T^(2^j), j < log2 L
  OFF_CR_LVL = OFF_CR_POW + 4 * kMaxLogL,      // 10 x 4: f/e, e, c, d
  OFF_U1 = OFF_CR_LVL + 4 * kMaxLevels,        // N
};
inline int off_u2(int N) { return OFF_U1 + N; }
inline int tab_stride(int N) { return (OFF_U1 + 2 * N + 7) & ~7; }

}  // namespace sosf

struct sos_plan_s {
  int K = 0, N = 0, L = 0, lgN = 0;
  int io_dtype = SOS_F32, compute_dtype = SOS_F64, solver_opt = SOS_AUTO;
  int tile_groups = 0;
  uint32_t flags = 0;
  bool b0_factored = false;
  double gain = 1.0;
  std::vector<double> rows;        // K x 5: b0 b1 b2 a1 a2 as the kernel uses them
  std::vector<double> rows_norm;   // K x 5: b0 b1 b2 a1 a2 divided by a0, b0 not factored
  std::vector<double> a0;          // K: the caller's a0
  std::vector<int32_t> solver;     // K: SOS_PH or SOS_CR
  std::vector<double> C;           // K x 4
  std::vector<double> cr_term;     // K x 2: e, f at the terminal level
  std::vector<double> table;       // K x stride, FP64 master copy of the device table
  int stride = 0;
  std::vector<double> phi;         // (2K)^2 one-step cascade state transition
  // deferred homogeneous correction (solver SOS_PH_DEFERRED, N >= 16)
  std::vector<double> theta;       // N x 2K: output at block m from a unit entry state
  std::vector<double> theta_mfma;  // theta in MFMA A-operand order [mb][kb][lane]
  std::vector<double> coupling;    // K(K-1)/2 blocks of 2x2: terminal of k from entry state j < k
  int kb = 0;                      // 4-wide state blocks: ceil(2K / 4)
  void *d_theta = nullptr;
  void *d_coupling = nullptr;
  int64_t warm = 0;                // run-in samples, multiple of N*L
  double runin_eps = 0.0;          // bound on ||Phi^warm||_inf (0: by the I/O type)
  double warm_norm = 0.0;
  int device = -1;
  int simds = 1024, waves_per_simd = 4;   // residency of the plan's kernel (launch-shape model)
  void *d_table = nullptr;         // device copy in the compute dtype
  void *d_solver = nullptr;        // device int8 per section: 1 = PH, 2 = CR
  // adjoint support (device plans only): a PH plan of the same cascade with
  // N = kBwdN and FP64 arithmetic, and per section the rows of the adjoint
  // (b0 b1 b2 a1 a2 unfactored, the cumulative b0 gain of the forward
  // pass's scaling, the caller's a0)
  sos_plan_s *bwd = nullptr;
  void *d_bwd_rows = nullptr;
  // block filtering (solver SOS_BLOCK): product type, FP64 block tables and
  // the MFMA A operands of the Toeplitz products
  int block_pt = 0;
  int block_slices = 1;            // slices per operand of FP16 / BF16 products (1: rounded once)
  std::vector<double> block_tab;
  std::vector<unsigned char> block_aop;
  void *d_block = nullptr;
  void *d_aop = nullptr;
  // exact inter-tile carry: the one-step state transition phi on the device
  void *d_phi = nullptr;
};

namespace sosf {
sos_status build_plan_tables(sos_plan_s &p, const double *sos);
void build_deferred_tables(sos_plan_s &p);
// the adjoint's sub-plan and rows (sosfilt_backward.hip)
sos_status attach_adjoint(sos_plan_s &p, const double *sos);
bool adjoint_recompute(const sos_plan_s &p);
double adjoint_cost_saved(int K, int io_dtype);
double adjoint_cost_recompute(int K, int io_dtype, bool stash);
bool adjoint_stash(bool rc, int io_dtype, int kmax);
// block filtering plans (sosfilt_block.hip)
sos_status build_block_plan(sos_plan_s &p);
sos_status upload_block_plan(sos_plan_s &p);
int64_t block_tile(const sos_plan_s &p, int64_t n);
sos_status launch_block(const sos_plan_s &p, const void *x, void *y, int64_t n, hipStream_t s);
// exact inter-tile carry (sosfilt_carry.hip): whether a plan can use it, the
// tiles, scan rounds and workspace for n samples (use = false: run-in), and
// the launches
struct CarryLayout {
  bool use = false;
  int64_t tile = 0, ntiles = 0;
  int rounds = 0;
  size_t aggs_off = 0, buf_off = 0, pow_off = 0, bytes = 0;
};
bool carry_supported(const sos_plan_s &p);
CarryLayout carry_layout(const sos_plan_s &p, int64_t n, int64_t runin_tile);
sos_status launch_carry(const sos_plan_s &p, const CarryLayout &l, const void *x, void *y, int64_t n, void *ws,
                        hipStream_t s);
}
namespace sosf {
sos_status check_filt_args(const sos_plan_s &p, const void *x, const void *y, int64_t n);
// wide groups, N > 64 (sosfilt_wide.hip): the lane runs live in the caller's workspace
bool wide_plan(const sos_plan_s &p);
int64_t wide_tile(const sos_plan_s &p, int64_t n);
size_t wide_workspace(const sos_plan_s &p, int64_t n);
sos_status launch_wide(const sos_plan_s &p, const void *x, void *y, int64_t n, void *ws, hipStream_t s);
// narrow groups, N = 4 (sosfilt_narrow.hip): single signals on 16-lane rows
bool narrow_plan(const sos_plan_s &p);
}
// runin_eps > 0 replaces the run-in bound that build_plan_tables picks.
sos_status create_plan(const double *sos, int32_t K, const sos_opts *opts, bool adjoint,
                       sos_plan_t *out, double runin_eps = 0.0);
