// Internal declarations shared by the IPFP library's HIP sources (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ipfp.h"

namespace ipfp {

// Device-side control block of one resident market. The sweep loop is driven
// entirely on the device: every kernel of a sweep reads `done` first and
// returns at once when the solve has finished, so the host can enqueue (or
// replay through a graph) more sweeps than remain without changing results.
struct Ctl {
  int32_t sweep;        // index i of the state (u^(i), v^(i)) currently held
  int32_t done;         // 1 once converged, max_sweeps reached or failed
  int32_t stop_sweep;   // sweep index of the returned state
  int32_t n_checks;     // residual checks recorded so far
  int32_t nonfinite;    // 1 if a non-finite intermediate was produced
  int32_t bad_margin;   // 1 if a margin was not > 0 and finite, or an FP8
                        // input row scale not a positive power of two
  int32_t arrive;       // combine workgroups of the row pass that have finished
                        // (the last one runs the convergence check)
  int32_t fix_total;    // rows recomputed by the fallback over the solve
  int32_t wexp[2];      // fused path: largest binary exponent of u (0), v (1)
  double last_res;      // most recent recorded residual
};

// Sweep parameters that are constant for a solve.
struct SweepParams {
  double tol;
  int32_t max_sweeps;
  int32_t check_every;
  int32_t hist_cap;     // capacity of the device residual history
};

// The positive root of w^2 + 2 s w - marg = 0 (eq. 6), evaluated as
// marg / (s + sqrt(s^2 + marg)) so that it does not cancel for s >> sqrt(marg).
__device__ __forceinline__ double quad_root(double marg, double s) {
  if (s > 1e150) return marg / (2.0 * s);
  return marg / (s + sqrt(s * s + marg));
}

// True when sweep i's state gets a residual check.
__device__ __forceinline__ bool is_check(int i, const SweepParams& sp) {
  return i >= 1 && (i % sp.check_every == 0 || i == sp.max_sweeps);
}

// Value of an OCP e4m3fn code (1 sign, 4 exponent bits with bias 7, 3
// significand bits; subnormals (f/8) 2^-6; the NaN codes 0x7F / 0xFF are
// decoded as 480 and never produced by the packer).
__device__ __forceinline__ float e4m3_val(uint8_t c) {
  const int e = (c >> 3) & 0xF, f = c & 7;
  const float v = e == 0 ? ldexpf((float)f, -9) : ldexpf((float)(8 + f), e - 10);
  return (c & 0x80) ? -v : v;
}

// A row scale of FP8 input: a positive, normal power of two.
__device__ __forceinline__ bool pow2_scale_ok(float s) {
  const uint32_t b = __float_as_uint(s);
  return (b >> 31) == 0 && (b & 0x7FFFFFu) == 0 && ((b >> 23) & 0xFF) != 0 &&
         ((b >> 23) & 0xFF) != 0xFF;
}

constexpr int kWave = 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = w > v ? w : v;
  }
  return v;
}

// One workgroup: reduce the residual maxima of the row pass that just ran
// (they belong to state i = ctl->sweep), record them at check sweeps, decide
// whether the solve stops at state i, and otherwise advance to state i + 1.
// The residual of state i is available here because the row pass of sweep
// i + 1 computes K v^(i) anyway; u^(i) is kept in the other half of a double
// buffer, so stopping at i returns exactly (u^(i), v^(i)).
__device__ __forceinline__ void check_body(Ctl* ctl, const double* res_block, int nblocks,
                                           double* hist, const SweepParams& sp) {
  __shared__ double red[256];
  if (ctl->done) return;
  const int i = ctl->sweep;
  const bool chk = is_check(i, sp);
  double r = 0.0;
  if (chk) {
    for (int k = threadIdx.x; k < nblocks; k += blockDim.x) {
      double x = res_block[k];
      // NaN compares false: keep it visible
      r = (x > r || x != x) ? x : r;
    }
  }
  red[threadIdx.x] = r;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      double a = red[threadIdx.x], b = red[threadIdx.x + o];
      red[threadIdx.x] = (b > a || b != b) ? b : a;
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (ctl->nonfinite || ctl->bad_margin) {
    ctl->done = 1;
    ctl->stop_sweep = i;
    return;
  }
  if (chk) {
    r = red[0];
    if (ctl->n_checks < sp.hist_cap) hist[ctl->n_checks] = r;
    ctl->n_checks += 1;
    ctl->last_res = r;
    if (r != r) ctl->nonfinite = 1;
    if (r < sp.tol || i >= sp.max_sweeps || r != r) {
      ctl->done = 1;
      ctl->stop_sweep = i;
      return;
    }
  }
  ctl->sweep = i + 1;
}

// ---- launchers implemented in the .hip sources ----------------------------

// residual / convergence control (control.hip)
hipError_t launch_check(Ctl* ctl, const double* res_block, int nblocks,
                        double* hist, SweepParams sp, hipStream_t s);
hipError_t launch_init_vec(double* v, const double* src, int64_t len,
                           hipStream_t s);
// Zero `bytes` (rounded up to whole 32-bit words) of device memory.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_validate_margins(const double* n, int64_t N, const double* m,
                                   int64_t M, Ctl* ctl, hipStream_t s);
hipError_t launch_validate_scales(const float* sx, int64_t N, const float* sy, int64_t M,
                                  Ctl* ctl, hipStream_t s);
hipError_t launch_mu_pairs(const void* U, const void* Q, const void* V,
                           const void* P, ipfp_dtype dt, const float* scale_x,
                           const float* scale_y, int64_t ld_x,
                           int64_t ld_y, int64_t N, int64_t M, int64_t d,
                           double sigma, const double* a, const double* b,
                           const int64_t* xs, const int64_t* ys, int64_t count,
                           double* mu, int32_t* bad, hipStream_t s);

// Margin residuals of eq. 5 for the output side (rows of A|B) against the
// other side (rows of C|D), from the factors as given; max_out (device, may be
// null) receives their maximum.
hipError_t launch_margin_residual(const void* A, const void* B, const float* sa, int64_t lda,
                                  const void* C, const void* D, const float* sc, int64_t ldc,
                                  ipfp_dtype dt, int64_t R, int64_t L, int64_t d, double sigma,
                                  const double* w_out, const double* w_red, const double* marg,
                                  double* res, double* max_out, hipStream_t s);

// plain path (plain.hip)
hipError_t launch_phi_from_factors(const void* U, const void* Q, const void* V,
                                   const void* P, ipfp_dtype dt, const float* scale_x,
                                   const float* scale_y, int64_t ld_x,
                                   int64_t ld_y, int64_t N, int64_t M,
                                   int64_t d, void* Kbuf, ipfp_dtype kdt,
                                   int64_t ldk, hipStream_t s);
hipError_t launch_materialize(const void* Phi, ipfp_dtype pdt, int64_t ldp,
                              void* Kbuf, ipfp_dtype kdt, int64_t ldk,
                              int64_t N, int64_t M, double sigma,
                              double* cshift, Ctl* ctl, hipStream_t s);
hipError_t launch_plain_row(const void* K, ipfp_dtype kdt, int64_t ldk,
                            int64_t N, int64_t M, const double* cshift,
                            const double* v, const double* n, double* u2,
                            double* ut, double* res_block, int* nblocks,
                            Ctl* ctl, hipStream_t s);
hipError_t launch_plain_col(const void* K, ipfp_dtype kdt, int64_t ldk,
                            int64_t N, int64_t M, const double* ut, int splits,
                            double* part, const double* m, double* v, Ctl* ctl,
                            hipStream_t s);
int plain_splits(int64_t N, int64_t M, ipfp_dtype kdt);

// fused path (fused.hip)
struct FusedSide {
  const void* ops;      // packed operand rows (rows x kpad codes)
  const float* scale;   // FP8: per-row power-of-two scale, else null
  int64_t rows;
};
int64_t fused_kpad(int64_t d, ipfp_dtype compute);
float fused_prescale(double sigma);
hipError_t launch_pack(const void* A, const void* B, ipfp_dtype in_dt,
                       const float* in_scale, int64_t ld, int64_t rows, int64_t d, ipfp_dtype compute,
                       int64_t kpad, float prescale, void* out, float* scale,
                       Ctl* ctl, hipStream_t s);

struct FusedPass {
  FusedSide out, red;       // output side (its scalings are updated) and
                            // reduced side (summed over)
  ipfp_dtype compute;
  int64_t kpad;
  const double* w_red;      // reduced side's scaling (FP64); for a double-
                            // buffered side the base of both halves
  int red_dbuf;             // 1: w_red holds two halves, pick by sweep parity
  int exp_red, exp_out;     // Ctl::wexp indices of the two sides
  float* shift;             // out.rows: -max_r T_or (log2 units), fixed
  const double* marg;       // out.rows margins
  double* part;             // splits x out.rows partial sums
  double* res_block;        // per-combine-block residual maxima
  int splits;
  int tile_rows;            // requested output rows per workgroup
  bool residual;            // compute the row residual of the old scaling
};
hipError_t launch_fused_pass(const FusedPass& fp, Ctl* ctl, hipStream_t s);
hipError_t launch_fused_shift(const FusedPass& fp, Ctl* ctl, hipStream_t s);
// Combine of a pass's partial sums, the quadratic update of its output side,
// the exact fallback for rows out of the shift's range and, for the row pass
// (fp.residual), the convergence check: one launch.
hipError_t launch_fused_combine(const FusedPass& fp, double* w2, int dbuf, Ctl* ctl,
                                double* hist, SweepParams sp, hipStream_t s);
int fused_combine_blocks(int64_t rows);
hipError_t launch_init_exp(const double* w, int64_t len, Ctl* ctl, int idx,
                           hipStream_t s);

// Recommendation lists (top-k per output row of a pass's output side): the
// k reduced rows with the largest mu, as (index, log mu). Scratch: splits x
// rows x topk_width(k) floats (pscore) and int32 (pidx).
int topk_width(int k);
int topk_splits(int64_t R, int64_t L);
hipError_t launch_topk(const FusedPass& fp, const double* a_out, int k, int splits,
                       float* pscore, int32_t* pidx, int32_t* idx_out, float* score_out,
                       hipStream_t s);
// Welfare gradient of the output side, G = mu Y (N x width FP64, width = 2d):
// BF16 operands only. Scratch: splits x rows x kpad doubles (gpart) and
// gradient_scratch_bytes(kpad, reduced rows) bytes (img, the reduced side's
// stage image: per stage, its packed rows and value columns as LDS holds
// them, 16-byte aligned); *Eptr is the largest binary exponent of fp.w_red.
size_t gradient_scratch_bytes(int kpad, int64_t L);
// Split count of the gradient pass (at most max_splits), from its occupancy.
int gradient_splits(int64_t R, int64_t L, int kpad, int max_splits);
hipError_t launch_gradient(const FusedPass& fp, const int* Eptr, const double* a_out,
                           double inv_p, int splits, double* gpart, uint8_t* img, int width,
                           double* g, int64_t ld_g, hipStream_t s);
hipError_t launch_stable_factors(const void* A, const void* B, ipfp_dtype dt,
                                 const float* in_scale, int64_t ld,
                                 int64_t rows, int64_t d, double sigma, const double* w,
                                 int log_col, double* out, int64_t ld_out, hipStream_t s);

// ---- grouped launches (many resident markets per kernel launch) -------------

// One market's half-sweep as the grouped pass and combine kernels read it
// (and, passed by value, as the single-market combine reads it).
struct GroupHalf {
  const uint8_t* Xo;        // output side operands (rows R)
  const float* xscale;
  const uint8_t* Yr;        // reduced side operands (rows L)
  const float* yscale;
  const double* wred;       // reduced side scaling (double-buffered if red_dbuf)
  const float* shift;       // R fixed row shifts
  double* part;             // nsplit x R partial sums
  Ctl* ctl;
  const double* marg;       // R margins
  double* w2;               // output side scaling (double-buffered if dbuf)
  double* res_block;        // combine blocks' residual maxima
  double* hist;             // residual history (row pass)
  SweepParams sp;
  int32_t red_dbuf, exp_red, exp_out, R, L, tiles_per_split, nsplit, dbuf, residual,
      kpad;
};
GroupHalf fused_half(const FusedPass& fp, Ctl* ctl, double* w2, int dbuf, double* hist,
                     SweepParams sp);

// Pass over markets idx[0..count) of table g; market idx[j] owns grid blocks
// [first[j], first[j+1]), first[count] = total. All share kpad and waves.
hipError_t launch_group_pass(const GroupHalf* g, const int32_t* idx, const int32_t* first,
                             int count, int total, int64_t kpad, ipfp_dtype compute,
                             int tile_rows, hipStream_t s);
// Combine (with fallback and, for row halves, the check) over markets
// 0..count of g with block ranges first[] (256 rows each).
hipError_t launch_group_combine(const GroupHalf* g, const int32_t* first, int count,
                                int total, ipfp_dtype compute, hipStream_t s);
// Grid size and split bookkeeping of a single-market pass (what the grouped
// pass must reproduce for bitwise-identical results).
void fused_pass_grid(const FusedPass& fp, int64_t* blocks, int* tiles_per_split);
int fused_auto_splits(int64_t R, int64_t L, int rows_per_wg);
// Split count of the sum pass for a market side (automatic splits).
int fused_pass_splits(int64_t R, int64_t L, int64_t kpad, ipfp_dtype compute, int tile_rows);
int fused_rows_per_wg(int64_t kpad, ipfp_dtype compute, int tile_rows);
int fused_default_tile_rows(int64_t kpad, ipfp_dtype compute);

}  // namespace ipfp
