/*
 * ipfp.h -- C ABI of the MI355X (gfx950) IPFP library for Choo-Siow
 * transferable-utility matching markets.
 *
 * The library solves the welfare program of the paper's Sec. 3.1 (eq. 2-3)
 * by the IPFP sweep of Sec. 3.2 (eq. 6-7): with u_x = sqrt(mu_x0) and
 * v_y = sqrt(mu_0y), every sweep sets
 *     u_x <- n_x / (s_x + sqrt(s_x^2 + n_x)),  s_x = (1/2) sum_y K_xy v_y,
 *     v_y <- m_y / (s_y + sqrt(s_y^2 + m_y)),  s_y = (1/2) sum_x K_xy u_x,
 * with K = exp(Phi / (2 sigma)) and v starting at 1. The root is the
 * rationalised form of eq. 6's sqrt(n + s^2) - s (the same number, without
 * the cancellation). The surplus is either given as a dense matrix (batch
 * IPFP, eq. 7) or as the low-rank product Phi = U V^T + Q P^T of eq. 8, in
 * which case the fused path never stores K (mini-batch IPFP, eq. 9-10).
 * Matching masses follow eq. 4: mu_xy = K_xy a_x b_y, mu_x0 = a_x^2,
 * mu_0y = b_y^2, with a = u and b = v.
 *
 * Names: n (length N) are the row (candidate) margins and m (length M) the
 * column (employer) margins, as in eq. 2 (the appendix's algorithms swap the
 * two letters). sigma is the paper's entropy scale beta.
 *
 * Convergence: after sweep i, when i is a multiple of check_every or equals
 * max_sweeps, the residual r = max_x |a_x^2 + a_x (K b)_x - n_x| / n_x of the
 * current (a, b) is recorded (eq. 5's row equation; its column equation holds
 * to rounding right after each v update). The solve stops when r < tol and
 * returns that sweep's (a, b); tol = 0 runs exactly max_sweeps sweeps.
 * r is measured on the kernel the path computes: on the FUSED path that is
 * 2^T of the rounded operands, summed from hardware exp2 values and FP32
 * partial sums of 16 terms, so r settles at a floor of a few 1e-7 (the FP64
 * oracle on the same operands agrees to 3e-7): a tol below that floor
 * returns IPFP_NOT_CONVERGED after max_sweeps. The distance to the exact
 * surplus (ipfp_margin_residuals) is set by the operand rounding instead.
 *
 * Conventions for every entry point:
 *  - Return value: IPFP_OK (0), a positive status (results valid), or a
 *    negative error code; nothing is thrown across the ABI.
 *  - Pointers named "device" are HIP device pointers on the context's device;
 *    "host" pointers are ordinary host memory. The caller owns every input
 *    and output buffer; the library owns only its scratch memory, which is
 *    charged against the context's HBM budget.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). All
 *    device work is ordered on it. Calls that return results to the host
 *    synchronise that stream before returning.
 *  - Matrices are row-major with a leading dimension (row stride) given in
 *    elements, >= the row length.
 *  - Inputs are validated before any launch: N, M >= 1; 1 <= d <= 256
 *    (fused path: d <= 128);
 *    sigma > 0 and finite; n and m must be > 0 and finite (checked on the
 *    device; a violation gives IPFP_EINVAL). Non-finite factor or surplus
 *    values give IPFP_ENONFINITE.
 */
#ifndef IPFP_H
#define IPFP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IPFP_ABI_VERSION 2

typedef enum {
  IPFP_F64 = 0,      /* IEEE binary64 */
  IPFP_F32 = 1,      /* IEEE binary32 */
  IPFP_BF16 = 2,     /* bfloat16 (upper half of binary32) */
  IPFP_FP8E4M3 = 3   /* OCP FP8 e4m3fn codes with a power-of-two scale per row */
} ipfp_dtype;

typedef enum {
  IPFP_PATH_FUSED = 0, /* factors -> on-the-fly MFMA tiles, K never stored */
  IPFP_PATH_PLAIN = 1  /* K = exp(Phi/2sigma) materialised, two matvecs/sweep */
} ipfp_path;

enum {
  IPFP_OK = 0,
  IPFP_NOT_CONVERGED = 1,   /* tol > 0 not reached in max_sweeps; a, b valid */
  IPFP_EINVAL = -1,         /* invalid argument */
  IPFP_EBUDGET = -2,        /* scratch would exceed the context's HBM budget */
  IPFP_EHIP = -3,           /* a HIP runtime call failed */
  IPFP_ENONFINITE = -4,     /* non-finite input or non-finite intermediate */
  IPFP_ECANCELLED = -5,     /* serving request cancelled */
  IPFP_EBUSY = -6,          /* serving request still queued or running */
  IPFP_ENOTFOUND = -7       /* unknown serving ticket */
};

typedef struct ipfp_ctx ipfp_ctx;       /* one per device; internally locked */
typedef struct ipfp_handle ipfp_handle; /* a market held resident on device */

/* A market given by its factors (eq. 8): Phi = U V^T + Q P^T.
 * U, Q: N x d device matrices with row stride ld_x; V, P: M x d with ld_y.
 * All four have dtype `in_dtype` (F64, F32, BF16 or FP8E4M3). n (N) and m (M)
 * are device FP64 margins.
 * FP8E4M3 input: the factors hold 1-byte OCP e4m3fn codes and the value of
 * row x's entries is code value x scale_x[x] (one scale per concatenated row
 * [U|Q]_x), of row y's entries code value x scale_y[y] ([V|P]_y). scale_x
 * (N) and scale_y (M) are device FP32 arrays, required for FP8 input and not
 * read otherwise; every scale must be a positive normal power of two, so the
 * values are exact in FP32 (checked on the device; a violation gives
 * IPFP_EINVAL). Such a market solves exactly as the same values given in
 * FP32 would (bitwise, for every path and compute type). */
typedef struct {
  int64_t N, M, d;
  ipfp_dtype in_dtype;
  const void *U, *Q, *V, *P;
  int64_t ld_x, ld_y;
  const double *n, *m;
  double sigma;
  const float *scale_x, *scale_y;
} ipfp_market;

typedef struct {
  ipfp_path path;        /* FUSED (factors) or PLAIN (materialised K)         */
  ipfp_dtype compute;    /* FUSED: BF16, FP8E4M3 or F32 operands for the
                            surplus tiles (BF16 and FP8 on their MFMAs, F32 on
                            the FP32 MFMA v_mfma_f32_32x32x2_f32; FP32
                            accumulate, FP32 exp2, FP64 sums and updates).
                            PLAIN: F32 or F64 storage of K (FP64 sums and
                            updates either way).                              */
  double tol;            /* stop when the row residual < tol; 0 = never       */
  int32_t max_sweeps;    /* >= 1                                              */
  int32_t check_every;   /* >= 1: residual cadence (and host sync cadence)    */
  int32_t splits;        /* reduction splits of the row half-sweep (and of
                            the column one unless splits_col is set); 0 =
                            automatic (chosen from the shape and the device's
                            compute units and occupancy). Results are bitwise
                            reproducible for fixed splits; across splits they
                            agree to rounding.                                */
  int32_t splits_col;    /* FUSED: splits of the column half-sweep; 0 = as
                            `splits` (automatic when that is 0)               */
  int32_t tile_rows;     /* FUSED: output rows per workgroup (128, 256 or
                            512); 0 = a per-type default (256 for BF16 with
                            2d = 64 and FP8 up to 2d = 128, else 512). F32
                            compute always uses 128 (one tile of 32 rows per
                            wave, four waves)                                 */
  const double *b0;      /* optional device warm start for v (length M);
                            NULL = ones. The initial u is never read.         */
  int32_t use_graph;     /* 1 = replay sweeps through a captured hipGraph     */
  int32_t time_passes;   /* 1 = bracket every reduction-pass launch with HIP
                            events and report their total in the result       */
} ipfp_options;

typedef struct {
  double *a;             /* device, length N: a = u = sqrt(mu_x0) (output)    */
  double *b;             /* device, length M: b = v = sqrt(mu_0y) (output)    */
  double *res_hist;      /* host, capacity res_cap: residual at every check   */
  int32_t res_cap;
  /* filled by the library */
  int32_t sweeps;        /* sweeps whose (a, b) are returned                  */
  int32_t n_res;         /* residuals recorded (may exceed res_cap; only the
                            first res_cap are stored)                         */
  double final_res;      /* residual of the returned (a, b)                   */
  double setup_ms;       /* packing / K materialisation time (host clock)     */
  double loop_ms;        /* sweep-loop time (HIP events on `stream`)          */
  double pass_ms;        /* sum of timed reduction-pass launches (ms)         */
  int32_t pass_launches; /* number of timed reduction-pass launches           */
  int32_t fixups;        /* rows recomputed by the exact-shift fallback (a row
                            whose shifted sum left [2^-60, inf): two FP64
                            passes over the reduced side inside its combine
                            workgroup, four rows at a time, one for FP8; about
                            2.7 ms per row at L = 2e5, d = 32 on MI355X, so a
                            count well above zero signals a slow solve)      */
} ipfp_result;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `hip_device` whose scratch allocations may
 * total at most `hbm_budget_bytes` (0 = no limit beyond the device's). */
int ipfp_create(ipfp_ctx **out, int hip_device, size_t hbm_budget_bytes);
void ipfp_destroy(ipfp_ctx *ctx);
const char *ipfp_strerror(int code);
int ipfp_abi_version(void);
/* The default options: FUSED, BF16, tol 0, 100 sweeps, check every sweep,
 * automatic splits and tiles, no warm start, no graph, no pass timing. */
void ipfp_default_options(ipfp_options *opt);

/* Scratch bytes a solve of this market with these options needs. */
int ipfp_footprint(const ipfp_market *mk, const ipfp_options *opt,
                   size_t *bytes_out);

/* How a fused solve of this market with these options would be laid out on
 * the current device (host-side only, nothing is launched): the packed width,
 * the workgroup height, the automatic and the chosen reduction splits of each
 * half-sweep, their grid sizes and the scratch footprint. */
typedef struct {
  int64_t kpad;              /* packed operand width (2d rounded up)         */
  int32_t rows_per_workgroup;
  int32_t auto_splits_row, auto_splits_col;
  int32_t splits_row, splits_col;
  int64_t blocks_row, blocks_col;   /* workgroups of each reduction pass     */
  size_t footprint_bytes;
} ipfp_plan;
int ipfp_plan_market(const ipfp_market *mk, const ipfp_options *opt, ipfp_plan *out);

/* ---- one-call solves ------------------------------------------------------ */

/* Solve a factor market (eq. 8-10). opt->path selects the fused on-the-fly
 * kernels (K never stored, mini-batch IPFP of Sec. 3.3) or the plain path,
 * which materialises K once from the factors (batch IPFP, eq. 7).
 * Returns IPFP_OK, IPFP_NOT_CONVERGED or an error. */
int ipfp_solve_market(ipfp_ctx *ctx, const ipfp_market *mk,
                      const ipfp_options *opt, ipfp_result *res, void *stream);

/* Allocation-free variant of ipfp_solve_market, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). It runs the same set-up, sweep kernels
 * and read-out, so its (a, b), residual history and sweep count equal
 * ipfp_solve_market's bit for bit, but the market's scratch is carved from a
 * fixed array of IPFP_NOALLOC_BYTES in device memory that every device the
 * library runs on holds for the life of the process (its address is looked up
 * by ipfp_create), and the call allocates nothing: no hipMalloc or hipFree,
 * no pinned host memory, no events or graphs (opt->use_graph and
 * opt->time_passes are ignored; loop_ms is host-clock time). The caller still
 * owns every input and output. A market whose footprint (ipfp_footprint)
 * exceeds IPFP_NOALLOC_BYTES is refused with IPFP_EBUDGET before any launch.
 * All calls on one device share that device's array, which keeps the last
 * call's contents (the set-up initialises everything a solve reads): calls
 * that overlap on one device, from any thread or stream, race and must be
 * serialised by the caller. Returns as ipfp_solve_market. */
#define IPFP_NOALLOC_BYTES ((size_t)64 << 20)
int ipfp_solve_market_noalloc(ipfp_ctx *ctx, const ipfp_market *mk,
                              const ipfp_options *opt, ipfp_result *res,
                              void *stream);

/* Autotuner for the fused path: times whole sweeps of this market (opened on
 * scratch memory, then freed) over candidate layouts and returns *opt with
 * the fastest tile_rows, splits and splits_col in *best and that sweep time in
 * *best_ms (may be NULL). Candidates: workgroup heights 256 and 512 (FP32:
 * its fixed 128) times the row pass's automatic split count, its half and its
 * double; then, for the best of those, the column pass's automatic split
 * count, its half and its double. Results of a solve depend on the choice
 * only through the split counts, to rounding (bitwise reproducible for a
 * fixed choice). Callers cache the choice per market shape as multiples of
 * the automatic counts (ipfp_plan_market); the Python binding keeps a JSON
 * cache. */
int ipfp_tune(ipfp_ctx *ctx, const ipfp_market *mk, const ipfp_options *opt,
              ipfp_options *best, double *best_ms, void *stream);

/* Solve a market given by a dense surplus Phi (N x M device matrix, dtype
 * F32 or F64, row stride ld_phi): batch IPFP of eq. 7 / Alg. 1 on the plain
 * path. opt->path is ignored; opt->compute chooses F32 or F64 storage of K. */
int ipfp_solve_market_phi(ipfp_ctx *ctx, int64_t N, int64_t M,
                          ipfp_dtype phi_dtype, const void *Phi,
                          int64_t ld_phi, const double *n, const double *m,
                          double sigma, const ipfp_options *opt,
                          ipfp_result *res, void *stream);

/* ---- resident markets (kept on device between calls) ---------------------- */

/* Pack the market's operands (fused path) or materialise K (plain path),
 * allocate its scratch and set v to b0 (or 1). The caller's factor and margin
 * buffers must stay valid until ipfp_market_close. */
int ipfp_market_open(ipfp_ctx *ctx, const ipfp_market *mk,
                     const ipfp_options *opt, ipfp_handle **out, void *stream);
/* Enqueue up to `sweeps` more sweeps (stopping early once converged or at
 * max_sweeps), then synchronise and report progress. *done is set to 1 when
 * the solve has finished (converged, or max_sweeps reached and the final
 * residual recorded). */
int ipfp_market_run(ipfp_handle *h, int32_t sweeps, int *done, void *stream);
/* Copy the current (a, b) to caller device buffers and fill `res` (res->a and
 * res->b are ignored; residual history goes to res->res_hist). */
int ipfp_market_read(ipfp_handle *h, double *a, double *b, ipfp_result *res,
                     void *stream);
void ipfp_market_close(ipfp_handle *h);

/* ---- outputs -------------------------------------------------------------- */

/* Matching masses at `count` requested pairs (eq. 4):
 * mu_out[i] = exp(Phi_{xs[i], ys[i]} / (2 sigma)) a_{xs[i]} b_{ys[i]}, where
 * Phi is formed in FP64 from the market's factors as given (in_dtype values,
 * not the packed compute operands). xs, ys: device int64 indices; a, b:
 * device FP64 scalings; mu_out: device FP64. The indices live in device
 * memory, so they are checked by the kernel: an out-of-range pair gets NaN
 * and the call returns IPFP_EINVAL after the stream has synchronised (the
 * other pairs are still written). The margins of mk are not read. */
int ipfp_mu_pairs(ipfp_ctx *ctx, const ipfp_market *mk, const double *a,
                  const double *b, const int64_t *xs, const int64_t *ys,
                  int64_t count, double *mu_out, void *stream);

/* Margin residuals of eq. 5 for given scalings (a, b), against the surplus
 * formed in FP64 from the market's factors as given (in_dtype values, not the
 * fused path's rounded operands): with mu_xy = exp(Phi_xy / (2 sigma)) a_x b_y
 * (eq. 4),
 *   row_res[x] = |a_x^2 + sum_y mu_xy - n_x| / n_x,
 *   col_res[y] = |b_y^2 + sum_x mu_xy - m_y| / m_y,
 * every mu formed in the log domain and summed in FP64 (O(N M d) FP64 work:
 * the exact check of any solve, whatever precision it ran in). a (N), b (M):
 * device FP64, > 0; row_res (N), col_res (M): caller-owned device FP64
 * outputs; max_row, max_col: host, may be NULL, receive the maxima (the
 * stream is synchronised). Scratch of 16 bytes is allocated for the call. */
int ipfp_margin_residuals(ipfp_ctx *ctx, const ipfp_market *mk, const double *a,
                          const double *b, double *row_res, double *col_res,
                          double *max_row, double *max_col, void *stream);

/* Stable factors of eq. 11 (Alg. 2's outputs), with which the matching of
 * eq. 4 factorises as log mu_xy = <psi_x, xi_y> / (2 sigma):
 *   psi_x = [U_x, Q_x, 2 sigma log a_x, 1],  xi_y = [V_y, P_y, 1, 2 sigma log b_y].
 * The paper prints sigma log u in place of 2 sigma log u; with u = sqrt(mu_x0)
 * only the factor 2 reproduces eq. 4, so that is what is written.
 * psi: N x (2d + 2) FP64 device matrix with row stride ld_psi; xi: M x (2d + 2)
 * with ld_xi (both caller-owned). Factors are read as given (mk->in_dtype);
 * the margins are not read. */
int ipfp_stable_factors(ipfp_ctx *ctx, const ipfp_market *mk, const double *a,
                        const double *b, double *psi, int64_t ld_psi, double *xi,
                        int64_t ld_xi, void *stream);

/* Recommendation lists of a resident fused market at its current state: for
 * side 0 every candidate x gets the k employers y with the largest mu_xy, for
 * side 1 every employer y the k candidates x with the largest mu_xy (the
 * reciprocal recommendation of Sec. 4.1, ranked by the stable matching).
 * Scores are formed from the packed operands the solve uses: log mu_xy =
 * ln 2 (T_xy + log2 a_x + log2 b_y), T from the matrix cores in FP32 (for
 * BF16 and FP32 operands the reduced side's log2 weight is the MFMA chain's
 * initial accumulator; for FP8 it is added after the chain). idx_out
 * (rows x k int32, device) lists indices best first, score_out (rows x k
 * float, device) the matching log mu; entries beyond the other side's size
 * are -1 / -inf. Equal scores keep the lower index of a lane's stream, so the
 * order among exact ties is implementation-defined. 1 <= k <= 32. Scratch of
 * splits x rows x (4 + 4) x k' bytes (k' = 8, 12, 16 or 32) is allocated for the
 * call and charged to the context budget. */
int ipfp_market_topk(ipfp_handle *h, int side, int32_t k, int32_t *idx_out,
                     float *score_out, void *stream);

/* Gradient of the optimal welfare with respect to the factors (Sec. 5 names
 * back-propagation into the recommender as future work). At the optimum of
 * eq. 2-3, dW/dPhi_xy = mu_xy (envelope theorem), and Phi = [U|Q][V|P]^T
 * (eq. 8), so side 0 gives G = mu [V|P] = [dW/dU | dW/dQ] (N x 2d) and side
 * 1 gives G = mu^T [U|Q] = [dW/dV | dW/dP] (M x 2d). Computed for a resident
 * fused BF16 market at its current state, from the operands the solve uses:
 * mu = 2^T a b with T from the packed rows, and the packed rows divided by
 * their prescale as the factor values (the factors as the matrix cores see
 * them). g_out: rows x 2d FP64 device, row stride ld_g >= 2d. Scratch of
 * splits x rows x kpad doubles plus a stage image of the other side's packed
 * rows (its rows and its value columns laid out per stage as the kernel's
 * LDS holds them: (2 kpad + 16) + kpad (2 s + 16) / s bytes per row for
 * stage height s, 544 at kpad 128; its row count rounded up to the stage
 * height) is allocated for the call and charged to the context budget.
 * IPFP_EINVAL for the plain path or FP8 operands. */
int ipfp_market_gradient(ipfp_handle *h, int side, double *g_out, int64_t ld_g,
                         void *stream);

/* The fused path's packed operand of one side (Sec. 3.3's factor matrices as
 * the matrix cores read them): rows p [A|B] concatenated, zero-padded to
 * `kpad` columns and rounded to `compute`, where p = sqrt(log2(e)/(2 sigma))
 * rounded to FP32 (p = 1 when sigma = 0), applied in FP32 after rounding the
 * input to FP32. BF16: 2-byte codes of the round-to-nearest-even value.
 * FP8E4M3: 1-byte e4m3fn codes of p x / s, with one FP32 power-of-two scale
 * s per row (the smallest with max |p x| <= 448 s) written to `scale_out`.
 * F32: the FP32 values p x. `out` is a device buffer of rows * kpad codes
 * (values for F32); kpad is returned through *kpad_out (pass out = NULL to
 * query it). FP8E4M3 input takes its per-row scales from `in_scale` (as
 * ipfp_market's scale_x; NULL otherwise). The solver packs with the market's
 * sigma, so this reproduces its operands bit for bit. */
int ipfp_pack_side(ipfp_ctx *ctx, int64_t rows, int64_t d, ipfp_dtype in_dtype,
                   const void *A, const void *B, const float *in_scale, int64_t ld,
                   ipfp_dtype compute, double sigma, void *out, float *scale_out,
                   int64_t *kpad_out, void *stream);

/* ---- roofline probes ------------------------------------------------------
 *
 * Measured ceilings of the operations the passes are bound by, taken on the
 * context's device: one kernel at full occupancy doing only that operation,
 * timed with HIP events on `stream` after a warm-up launch.
 *   EXP2: v_exp_f32 results per second; `work` = iterations per thread
 *         (8 independent chains each).
 *   MFMA_BF16 / MFMA_FP8 / MFMA_F32: dense flops per second of the fused
 *         paths' matrix instructions (32x32x16 BF16, 32x32x64 FP8 with unit
 *         scales, 32x32x2 FP32), four independent accumulators per wave;
 *         `work` = MFMAs per accumulator.
 *   HBM_READ: bytes per second of a streaming read (16-byte nontemporal loads,
 *         lane-contiguous as in the plain path, four in flight per thread) of
 *         a `work`-byte buffer (a multiple of 32 MiB, allocated for the call
 *         and charged to the context budget).
 *   MFMA_BF16_2W / MFMA_BF16_EPI / MFMA_FP8_EPI: the matrix stream at the
 *         fused passes' occupancy (two waves per SIMD, two independent
 *         accumulators per wave), bare or with the sum pass's epilogue beside
 *         it: after each MFMA, 2 exp2 and 2 FMAs (BF16, the ratio at
 *         2d = 128) or 8 exp2 and 8 FMAs (FP8 at 2d = 128), on independent
 *         registers; MFMA flops per second, `work` = rounds of two MFMAs.
 * *rate_out receives the rate, *ms_out (may be NULL) the timed launch. */
enum {
  IPFP_PROBE_EXP2 = 0,
  IPFP_PROBE_MFMA_BF16 = 1,
  IPFP_PROBE_MFMA_FP8 = 2,
  IPFP_PROBE_MFMA_F32 = 3,
  IPFP_PROBE_HBM_READ = 4,
  IPFP_PROBE_MFMA_BF16_2W = 5,
  IPFP_PROBE_MFMA_BF16_EPI = 6,
  IPFP_PROBE_MFMA_FP8_EPI = 7
};
int ipfp_probe(ipfp_ctx *ctx, int kind, int64_t work, double *rate_out, double *ms_out,
               void *stream);

/* ---- serving: continuous batching of many markets ------------------------
 *
 * The paper solves one market at a time; a server solves a stream of
 * independent markets (requests) concurrently on one device. It owns one slab
 * of device memory (its arena) and a scheduler thread. Each request belongs
 * to one of `lanes` HIP streams chosen by its size N*M. The scheduler admits
 * queued requests smallest first, where a request's size counts as
 * log2(N*M) minus its waiting time over aging_ms (so nothing waits forever),
 * while its footprint (ipfp_footprint) fits the arena, fewer than max_active
 * markets are resident and its lane holds fewer than lane_blocks reduction
 * workgroups per pass (a lane with no market always takes one). A request
 * that can never fit the arena is refused at submission with IPFP_EBUDGET.
 * Each lane advances all of its resident markets together: every kernel of a
 * sweep is one grouped launch over the lane's markets, `chunk` sweeps per
 * scheduling round. Markets join and leave a lane at round boundaries. Each
 * market keeps
 * its own convergence state on the device and stops by itself (tol,
 * max_sweeps), and its arithmetic -- splits, tiles, reduction order -- is the
 * one ipfp_solve_market uses with the same options, so a request's (a, b) are
 * bitwise identical to solving it alone.
 *
 * Ownership: the market's input buffers (factors, margins, b0) must stay
 * valid, and its ipfp_result (with its device a, b and host res_hist) must
 * stay allocated, until the request is reported finished. */
typedef struct ipfp_server ipfp_server;

typedef struct {
  size_t arena_bytes;   /* device memory for resident markets; 0 = 1 GiB.
                           Charged against the context's budget.            */
  int32_t max_active;   /* resident markets at once, 1..1024; 0 = 256       */
  int32_t lanes;        /* concurrent streams, 1..4; 0 = 3                  */
  int32_t chunk;        /* sweeps per scheduling round, 1..64; 0 = 4        */
  ipfp_dtype compute;   /* BF16 or FP8E4M3, for every request               */
  int32_t tile_rows;    /* as ipfp_options.tile_rows, for every request     */
  double lane_pairs[3]; /* rising upper bounds of N*M for lanes 0..lanes-2;
                           0 = split log2(N*M) in [20, 36] evenly           */
  int32_t lane_blocks;  /* reduction workgroups per pass a lane admits up
                           to; 0 = 2048 (8 per compute unit)                */
  double aging_ms;      /* waiting time worth a halving of N*M; 0 = 4000    */
} ipfp_server_options;

enum { IPFP_REQ_QUEUED = 0, IPFP_REQ_RUNNING = 1, IPFP_REQ_FINISHED = 2 };

typedef struct {
  int32_t state;        /* IPFP_REQ_*                                       */
  int32_t code;         /* once finished: the solve's return code          */
  int32_t lane;         /* lane the market runs on (-1 before admission)   */
  double t_submit;      /* host CLOCK_MONOTONIC, milliseconds              */
  double t_admit;       /* its set-up was enqueued                         */
  double t_done;        /* its outputs were written                        */
} ipfp_request_info;

typedef struct {
  int64_t submitted, admitted, finished, queued, active, rounds;
  size_t arena_bytes, arena_used, arena_peak;
  double pair_evals;    /* sum over finished requests of 2 N M sweeps      */
} ipfp_server_stats;

void ipfp_default_server_options(ipfp_server_options *opt);
/* Allocates the arena and starts the scheduler thread. */
int ipfp_server_create(ipfp_ctx *ctx, const ipfp_server_options *opt,
                       ipfp_server **out);
/* Cancels queued and running requests, waits for the scheduler to drain and
 * frees the server. Tickets are invalid afterwards. */
void ipfp_server_destroy(ipfp_server *srv);
/* Queues a fused-path solve (validated as ipfp_solve_market; opt->compute
 * must be the server's, opt->tile_rows 0 or the server's; use_graph and
 * time_passes are ignored). The inputs are read after the work enqueued on
 * `stream` so far has completed (an event is recorded there). Never blocks on
 * the device. */
int ipfp_submit(ipfp_server *srv, const ipfp_market *mk, const ipfp_options *opt,
                ipfp_result *res, uint64_t *ticket, void *stream);
/* IPFP_EBUSY while queued or running. Once finished: the request's return
 * code (IPFP_OK, IPFP_NOT_CONVERGED, IPFP_ECANCELLED or an error), after
 * which the ticket is forgotten (IPFP_ENOTFOUND). `info` may be NULL. */
int ipfp_poll(ipfp_server *srv, uint64_t ticket, ipfp_request_info *info);
/* As ipfp_poll, blocking up to timeout_ms (< 0: no limit). */
int ipfp_wait(ipfp_server *srv, uint64_t ticket, double timeout_ms,
              ipfp_request_info *info);
/* A queued request finishes at once with IPFP_ECANCELLED; a running one at
 * the end of its lane's round (its outputs are then not written). */
int ipfp_cancel(ipfp_server *srv, uint64_t ticket);
int ipfp_server_get_stats(ipfp_server *srv, ipfp_server_stats *out);
/* The host clock the request times use (CLOCK_MONOTONIC), in ms. */
double ipfp_clock_ms(void);

#ifdef __cplusplus
}
#endif
#endif /* IPFP_H */
