// C ABI: contexts, resident markets, the device-driven sweep loop, the
// one-call solves, the outputs (stable factors, recommendation lists,
// gradient) and the autotuner. Every sweep is a fixed sequence of kernels on
// the caller's stream; the only host/device synchronisation is a 64-byte read
// of the control block after each batch of enqueued sweeps.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "handle.h"

using namespace ipfp;

// Scratch of the allocation-free solve (ipfp_solve_market_noalloc): one array
// in device memory, a copy of which every device the library runs on holds
// until the process ends. In host code this name is only a handle for the
// symbol lookup below, never an address: the array's device address is
// looked up once per device (with that device current) and kept in
// g_noalloc, and only that address is passed to kernels.
static __device__ __align__(256) char scratch[IPFP_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void* g_noalloc[kMaxDevices];
std::mutex g_noalloc_mu;

// The device address of `scratch` on device `dev` (looked up on first use).
int noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return IPFP_EINVAL;
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  if (!g_noalloc[dev]) {
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(dev) != hipSuccess) {
      (void)hipGetLastError();
      return IPFP_EHIP;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return IPFP_EHIP;
    }
    g_noalloc[dev] = p;
  }
  *out = g_noalloc[dev];
  return IPFP_OK;
}
}  // namespace

#define HIPCHK(expr)                         \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return IPFP_EHIP;  \
  } while (0)

// ---- sizes -------------------------------------------------------------------

void ipfp::handle_layout(ipfp_handle* h, Carver& cv) {
  const int64_t N = h->N, M = h->M;
  h->ctl = cv.take<Ctl>(1);
  if (h->ext_ctl) h->ctl = h->ext_ctl;
  h->hist = cv.take<double>(kHistCap);
  h->u2 = cv.take<double>(2 * N);
  h->v = cv.take<double>(M);
  if (h->plain) {
    const int64_t vn = h->kdt == IPFP_F64 ? 2 : 4;
    h->ldk = align_up((size_t)M, 64);
    (void)vn;
    h->K = cv.take<char>((size_t)N * h->ldk * dtype_size(h->kdt));
    h->cshift = cv.take<double>(N);
    h->ut = cv.take<double>(N);
    h->psplits = plain_splits(N, M, h->kdt);
    h->part = cv.take<double>((size_t)h->psplits * M);
    h->nres_row = (int)((N + 15) / 16);
    h->res_block = cv.take<double>(h->nres_row);
  } else {
    const ipfp_dtype cd = h->opt.compute;
    const size_t es = cd == IPFP_FP8E4M3 ? 1 : (cd == IPFP_F32 ? 4 : 2);
    h->kpad = fused_kpad(h->mk.d, cd);
    h->xop = cv.take<char>((size_t)N * h->kpad * es);
    h->yop = cv.take<char>((size_t)M * h->kpad * es);
    h->xscale = cv.take<float>(N);
    h->yscale = cv.take<float>(M);
    h->xshift = cv.take<float>(N);
    h->yshift = cv.take<float>(M);
    const int tr = h->opt.tile_rows > 0 ? h->opt.tile_rows : fused_default_tile_rows(h->kpad, cd);
    const int rx = fused_rows_per_wg(h->kpad, cd, tr);
    const int scol = h->opt.splits_col > 0 ? h->opt.splits_col : h->opt.splits;
    int sx = h->opt.splits > 0 ? h->opt.splits : fused_pass_splits(N, M, h->kpad, cd, tr);
    int sy = scol > 0 ? scol : fused_pass_splits(M, N, h->kpad, cd, tr);
    h->xpart = cv.take<double>((size_t)sx * N);
    h->ypart = cv.take<double>((size_t)sy * M);
    h->row_combine_blocks = fused_combine_blocks(N);
    h->col_combine_blocks = fused_combine_blocks(M);
    h->nres_row = h->row_combine_blocks;
    h->res_block = cv.take<double>(h->nres_row);
    h->res_dummy = cv.take<double>(h->col_combine_blocks);
    h->rowp.splits = sx;
    h->colp.splits = sy;
    h->rowp.tile_rows = h->colp.tile_rows = tr;
  }
}

int ipfp::validate_market(const ipfp_market* mk, const ipfp_options* opt, bool factors) {
  if (!mk || !opt) return IPFP_EINVAL;
  if (mk->N < 1 || mk->M < 1) return IPFP_EINVAL;
  if (mk->N > INT32_MAX || mk->M > INT32_MAX) return IPFP_EINVAL;
  if (!(mk->sigma > 0.0) || !(mk->sigma < INFINITY)) return IPFP_EINVAL;
  if (!mk->n || !mk->m) return IPFP_EINVAL;
  if (opt->max_sweeps < 1 || opt->check_every < 1) return IPFP_EINVAL;
  if (!(opt->tol >= 0.0)) return IPFP_EINVAL;
  if (opt->splits < 0 || opt->splits > 256) return IPFP_EINVAL;
  if (opt->splits_col < 0 || opt->splits_col > 256) return IPFP_EINVAL;
  if (factors) {
    if (mk->d < 1 || mk->d > 256) return IPFP_EINVAL;
    if (!mk->U || !mk->Q || !mk->V || !mk->P) return IPFP_EINVAL;
    if (mk->ld_x < mk->d || mk->ld_y < mk->d) return IPFP_EINVAL;
    if (mk->in_dtype != IPFP_F64 && mk->in_dtype != IPFP_F32 &&
        mk->in_dtype != IPFP_BF16 && mk->in_dtype != IPFP_FP8E4M3)
      return IPFP_EINVAL;
    if (mk->in_dtype == IPFP_FP8E4M3 && (!mk->scale_x || !mk->scale_y)) return IPFP_EINVAL;
  }
  if (opt->path == IPFP_PATH_PLAIN) {
    if (opt->compute != IPFP_F32 && opt->compute != IPFP_F64) return IPFP_EINVAL;
  } else if (opt->path == IPFP_PATH_FUSED) {
    if (opt->compute != IPFP_BF16 && opt->compute != IPFP_FP8E4M3 &&
        opt->compute != IPFP_F32)
      return IPFP_EINVAL;
    if (mk->d > 128) return IPFP_EINVAL;
    if (opt->tile_rows != 0 && opt->tile_rows != 128 && opt->tile_rows != 256 &&
        opt->tile_rows != 512)
      return IPFP_EINVAL;
  } else {
    return IPFP_EINVAL;
  }
  return IPFP_OK;
}

// ---- sweep units ---------------------------------------------------------------

SweepParams ipfp::handle_sweep_params(const ipfp_handle* h) {
  SweepParams sp;
  sp.tol = h->opt.tol;
  sp.max_sweeps = h->opt.max_sweeps;
  sp.check_every = h->opt.check_every;
  sp.hist_cap = kHistCap;
  return sp;
}

// Runs `fn` (one kernel launch on `s`), bracketed by HIP events when timing;
// the event pairs are summed after the next synchronisation.
template <typename F>
static hipError_t timed(ipfp_handle* h, bool timing, hipStream_t s, F&& fn) {
  if (!timing) return fn();
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipEventRecord(a, s);
  if (e == hipSuccess) e = fn();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return e;
  }
  h->evs.push_back(a);
  h->evs.push_back(b);
  return hipSuccess;
}

// One sweep unit: the row half-sweep for the current state, the convergence
// check, then the column half-sweep (skipped on the device once done).
static hipError_t enqueue_unit(ipfp_handle* h, hipStream_t s, bool timing) {
  hipError_t e;
  const SweepParams sp = handle_sweep_params(h);
  int nb = 0;
  if (h->plain) {
    e = timed(h, timing, s, [&] {
      return launch_plain_row(h->K, h->kdt, h->ldk, h->N, h->M, h->cshift, h->v, h->mk.n,
                              h->u2, h->ut, h->res_block, &nb, h->ctl, s);
    });
    if (e != hipSuccess) return e;
    e = launch_check(h->ctl, h->res_block, nb, h->hist, sp, s);
    if (e != hipSuccess) return e;
    return timed(h, timing, s, [&] {
      return launch_plain_col(h->K, h->kdt, h->ldk, h->N, h->M, h->ut, h->psplits, h->part,
                              h->mk.m, h->v, h->ctl, s);
    });
  }
  // fused: four launches per sweep -- each combine also runs the exact
  // fallback for its rows, the row combine's last workgroup the check
  e = timed(h, timing, s, [&] { return launch_fused_pass(h->rowp, h->ctl, s); });
  if (e != hipSuccess) return e;
  e = launch_fused_combine(h->rowp, h->u2, 1, h->ctl, h->hist, sp, s);
  if (e != hipSuccess) return e;
  e = timed(h, timing, s, [&] { return launch_fused_pass(h->colp, h->ctl, s); });
  if (e != hipSuccess) return e;
  return launch_fused_combine(h->colp, h->v, 0, h->ctl, h->hist, sp, s);
}

static int read_ctl(ipfp_handle* h, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(h->host_ctl, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return IPFP_OK;
}

static void collect_events(ipfp_handle* h) {
  for (size_t k = 0; k + 1 < h->evs.size(); k += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->evs[k], h->evs[k + 1]) == hipSuccess) {
      h->pass_ms += ms;
      h->pass_launches += 1;
    }
    (void)hipEventDestroy(h->evs[k]);
    (void)hipEventDestroy(h->evs[k + 1]);
  }
  h->evs.clear();
}

int ipfp::ctx_reserve(ipfp_ctx* ctx, size_t bytes) {
  std::lock_guard<std::mutex> g(ctx->mu);
  if (ctx->budget && ctx->used + bytes > ctx->budget) return IPFP_EBUDGET;
  ctx->used += bytes;
  return IPFP_OK;
}

void ipfp::ctx_release(ipfp_ctx* ctx, size_t bytes) {
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->used -= bytes;
}

#define TRY(expr)                        \
  do {                                   \
    hipError_t e_ = (expr);              \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

hipError_t ipfp::handle_setup(ipfp_handle* h, const void* phi, ipfp_dtype phi_dt,
                              int64_t ld_phi, hipStream_t s) {
  const ipfp_market* mk = &h->mk;
  const ipfp_options* opt = &h->opt;
  TRY(launch_zero(h->ctl, sizeof(Ctl), s));
  TRY(launch_validate_margins(mk->n, h->N, mk->m, h->M, h->ctl, s));
  if (!phi && mk->in_dtype == IPFP_FP8E4M3)
    TRY(launch_validate_scales(mk->scale_x, h->N, mk->scale_y, h->M, h->ctl, s));
  TRY(launch_init_vec(h->u2, nullptr, 2 * h->N, s));
  TRY(launch_init_vec(h->v, opt->b0, h->M, s));
  if (h->plain) {
    if (phi) {
      return launch_materialize(phi, phi_dt, ld_phi, h->K, h->kdt, h->ldk, h->N, h->M,
                                mk->sigma, h->cshift, h->ctl, s);
    }
    TRY(launch_phi_from_factors(mk->U, mk->Q, mk->V, mk->P, mk->in_dtype, mk->scale_x,
                                mk->scale_y, mk->ld_x,
                                mk->ld_y, h->N, h->M, mk->d, h->K, h->kdt, h->ldk, s));
    return launch_materialize(h->K, h->kdt, h->ldk, h->K, h->kdt, h->ldk, h->N, h->M,
                              mk->sigma, h->cshift, h->ctl, s);
  }
  const ipfp_dtype cd = opt->compute;
  const float ps = fused_prescale(mk->sigma);
  TRY(launch_pack(mk->U, mk->Q, mk->in_dtype, mk->scale_x, mk->ld_x, h->N, mk->d, cd, h->kpad, ps,
                  h->xop, h->xscale, h->ctl, s));
  TRY(launch_pack(mk->V, mk->P, mk->in_dtype, mk->scale_y, mk->ld_y, h->M, mk->d, cd, h->kpad, ps,
                  h->yop, h->yscale, h->ctl, s));
  FusedSide X{h->xop, cd == IPFP_FP8E4M3 ? h->xscale : nullptr, h->N};
  FusedSide Y{h->yop, cd == IPFP_FP8E4M3 ? h->yscale : nullptr, h->M};
  FusedPass& r = h->rowp;
  r.out = X; r.red = Y; r.compute = cd; r.kpad = h->kpad;
  r.w_red = h->v; r.red_dbuf = 0; r.exp_red = 1; r.exp_out = 0;
  r.shift = h->xshift; r.marg = mk->n;
  r.part = h->xpart; r.res_block = h->res_block;
  r.residual = true;
  FusedPass& q = h->colp;
  q.out = Y; q.red = X; q.compute = cd; q.kpad = h->kpad;
  q.w_red = h->u2; q.red_dbuf = 1; q.exp_red = 0; q.exp_out = 1;
  q.shift = h->yshift; q.marg = mk->m;
  q.part = h->ypart; q.res_block = h->res_dummy;
  q.residual = false;
  // fixed row shifts h = -max T from one max pass per side; exponent of v0
  TRY(launch_fused_shift(r, h->ctl, s));
  TRY(launch_fused_shift(q, h->ctl, s));
  return launch_init_exp(h->v, h->M, h->ctl, 1, s);
}

// ---- C ABI -------------------------------------------------------------------

extern "C" {

int ipfp_abi_version(void) { return IPFP_ABI_VERSION; }

const char* ipfp_strerror(int code) {
  switch (code) {
    case IPFP_OK: return "ok";
    case IPFP_NOT_CONVERGED: return "tolerance not reached within max_sweeps";
    case IPFP_EINVAL: return "invalid argument";
    case IPFP_EBUDGET: return "scratch memory exceeds the context budget";
    case IPFP_EHIP: return "HIP runtime error";
    case IPFP_ENONFINITE: return "non-finite input or intermediate value";
    case IPFP_ECANCELLED: return "request cancelled";
    case IPFP_EBUSY: return "request not finished";
    case IPFP_ENOTFOUND: return "unknown ticket";
    default: return "unknown error code";
  }
}

void ipfp_default_options(ipfp_options* opt) {
  memset(opt, 0, sizeof(*opt));
  opt->path = IPFP_PATH_FUSED;
  opt->compute = IPFP_BF16;
  opt->tol = 0.0;
  opt->max_sweeps = 100;
  opt->check_every = 1;
}

int ipfp_create(ipfp_ctx** out, int hip_device, size_t hbm_budget_bytes) {
  if (!out) return IPFP_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n)
    return IPFP_EINVAL;
  void* sp = nullptr;
  const int rc = noalloc_scratch(hip_device, &sp);
  if (rc != IPFP_OK) return rc;
  ipfp_ctx* c = new ipfp_ctx;
  c->device = hip_device;
  c->budget = hbm_budget_bytes;
  c->used = 0;
  c->noalloc = sp;
  *out = c;
  return IPFP_OK;
}

void ipfp_destroy(ipfp_ctx* ctx) { delete ctx; }

static int footprint_impl(const ipfp_market* mk, const ipfp_options* opt,
                          bool plain, size_t* bytes) {
  ipfp_handle h;
  h.mk = *mk;
  h.opt = *opt;
  h.plain = plain;
  h.N = mk->N;
  h.M = mk->M;
  h.kdt = opt->compute == IPFP_F64 ? IPFP_F64 : IPFP_F32;
  Carver cv;
  handle_layout(&h, cv);
  *bytes = align_up(cv.off, 256);
  return IPFP_OK;
}

int ipfp_footprint(const ipfp_market* mk, const ipfp_options* opt,
                   size_t* bytes_out) {
  if (!bytes_out) return IPFP_EINVAL;
  int rc = validate_market(mk, opt, true);
  if (rc != IPFP_OK) return rc;
  return footprint_impl(mk, opt, opt->path == IPFP_PATH_PLAIN, bytes_out);
}

static void destroy_handle(ipfp_handle* h) {
  if (!h) return;
  collect_events(h);
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->host_ctl) (void)hipHostFree(h->host_ctl);
  if (!h->arena) {
    if (h->mem) (void)hipFree(h->mem);
    if (h->ctx && h->bytes) ctx_release(h->ctx, h->bytes);
  }
  delete h;
}

// Opens a market: explicit Phi (phi != null) or factors.
static int open_impl(ipfp_ctx* ctx, const ipfp_market* mk, const ipfp_options* opt,
                     const void* phi, ipfp_dtype phi_dt, int64_t ld_phi,
                     ipfp_handle** out, hipStream_t s) {
  *out = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return IPFP_EHIP;
  const double t0 = now_ms();
  ipfp_handle* h = new ipfp_handle;
  h->ctx = ctx;
  h->mk = *mk;
  h->opt = *opt;
  h->plain = phi != nullptr || opt->path == IPFP_PATH_PLAIN;
  h->N = mk->N;
  h->M = mk->M;
  h->kdt = opt->compute == IPFP_F64 ? IPFP_F64 : IPFP_F32;
  Carver cv;
  handle_layout(h, cv);
  const size_t bytes = align_up(cv.off, 256);
  int rc = ctx_reserve(ctx, bytes);
  if (rc != IPFP_OK) {
    delete h;
    return rc;
  }
  h->bytes = bytes;
  if (hipMalloc((void**)&h->mem, bytes) != hipSuccess) {
    h->mem = nullptr;
    destroy_handle(h);
    return IPFP_EBUDGET;
  }
  if (hipHostMalloc((void**)&h->host_ctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
    h->host_ctl = nullptr;
    destroy_handle(h);
    return IPFP_EHIP;
  }
  Carver real;
  real.base = h->mem;
  handle_layout(h, real);

  auto fail = [&](int code) {
    destroy_handle(h);
    return code;
  };
  if (handle_setup(h, phi, phi_dt, ld_phi, s) != hipSuccess) return fail(IPFP_EHIP);
  if (read_ctl(h, s) != IPFP_OK) return fail(IPFP_EHIP);
  if (h->host_ctl->bad_margin) return fail(IPFP_EINVAL);
  if (h->host_ctl->nonfinite) return fail(IPFP_ENONFINITE);
  h->setup_ms = now_ms() - t0;
  *out = h;
  return IPFP_OK;
}

int ipfp_market_open(ipfp_ctx* ctx, const ipfp_market* mk, const ipfp_options* opt,
                     ipfp_handle** out, void* stream) {
  if (!ctx || !out) return IPFP_EINVAL;
  int rc = validate_market(mk, opt, true);
  if (rc != IPFP_OK) return rc;
  return open_impl(ctx, mk, opt, nullptr, IPFP_F32, 0, out, (hipStream_t)stream);
}

static int run_impl(ipfp_handle* h, int32_t sweeps, int* done, hipStream_t s) {
  if (hipSetDevice(h->ctx->device) != hipSuccess) return IPFP_EHIP;
  const int total = h->opt.max_sweeps + 1;  // +1: final residual row pass
  int todo = std::min(sweeps, total - h->units);
  const bool timing = h->opt.time_passes != 0;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  if (h->opt.use_graph && !timing && todo > 0) {
    const int G = std::max(1, std::min(h->opt.check_every, 16));
    if (!h->graph && todo >= G) {
      if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
      hipGraph_t g;
      HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < G; ++k) {
        if (enqueue_unit(h, h->cap_stream, false) != hipSuccess) {
          (void)hipStreamEndCapture(h->cap_stream, &g);
          return IPFP_EHIP;
        }
      }
      HIPCHK(hipStreamEndCapture(h->cap_stream, &g));
      HIPCHK(hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0));
      (void)hipGraphDestroy(g);
      h->graph_units = G;
    }
    while (h->graph && todo >= h->graph_units) {
      HIPCHK(hipGraphLaunch(h->graph, s));
      todo -= h->graph_units;
      h->units += h->graph_units;
    }
  }
  for (; todo > 0; --todo) {
    if (enqueue_unit(h, s, timing) != hipSuccess) return IPFP_EHIP;
    h->units += 1;
  }
  HIPCHK(hipEventRecord(e1, s));
  int rc = read_ctl(h, s);
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) h->loop_ms += ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  collect_events(h);
  if (rc != IPFP_OK) return rc;
  if (done) *done = h->host_ctl->done || h->units >= total;
  if (h->host_ctl->nonfinite) return IPFP_ENONFINITE;
  return IPFP_OK;
}

int ipfp_market_run(ipfp_handle* h, int32_t sweeps, int* done, void* stream) {
  if (!h || sweeps < 0) return IPFP_EINVAL;
  return run_impl(h, sweeps, done, (hipStream_t)stream);
}

int ipfp_market_read(ipfp_handle* h, double* a, double* b, ipfp_result* res,
                     void* stream) {
  if (!h) return IPFP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(h->ctx->device) != hipSuccess) return IPFP_EHIP;
  int rc = read_ctl(h, s);
  if (rc != IPFP_OK) return rc;
  const Ctl c = *h->host_ctl;
  // the state held is c.sweep until the solve stops; then c.stop_sweep
  const int state = c.done ? c.stop_sweep : c.sweep;
  const double* u = h->u2 + (int64_t)(state & 1) * h->N;
  if (a) HIPCHK(hipMemcpyAsync(a, u, h->N * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (b) HIPCHK(hipMemcpyAsync(b, h->v, h->M * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (res) {
    res->sweeps = state;
    res->n_res = c.n_checks;
    res->final_res = c.n_checks ? c.last_res : NAN;
    res->setup_ms = h->setup_ms;
    res->loop_ms = h->loop_ms;
    res->pass_ms = h->pass_ms;
    res->pass_launches = h->pass_launches;
    res->fixups = c.fix_total;
    const int ncopy = std::min(std::min(c.n_checks, res->res_cap), kHistCap);
    if (res->res_hist && ncopy > 0)
      HIPCHK(hipMemcpyAsync(res->res_hist, h->hist, ncopy * sizeof(double),
                            hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  if (c.nonfinite) return IPFP_ENONFINITE;
  if (h->opt.tol > 0.0 && c.done && !(c.last_res < h->opt.tol)) return IPFP_NOT_CONVERGED;
  return IPFP_OK;
}

void ipfp_market_close(ipfp_handle* h) { destroy_handle(h); }

static int solve_handle(ipfp_handle* h, ipfp_result* res, hipStream_t s) {
  int done = 0;
  const int chunk = std::max(h->opt.check_every, 8);
  while (!done) {
    int rc = run_impl(h, chunk, &done, s);
    if (rc != IPFP_OK) return rc;
  }
  return ipfp_market_read(h, res->a, res->b, res, s);
}

int ipfp_solve_market(ipfp_ctx* ctx, const ipfp_market* mk, const ipfp_options* opt,
                      ipfp_result* res, void* stream) {
  if (!ctx || !res || !res->a || !res->b) return IPFP_EINVAL;
  int rc = validate_market(mk, opt, true);
  if (rc != IPFP_OK) return rc;
  ipfp_handle* h = nullptr;
  rc = open_impl(ctx, mk, opt, nullptr, IPFP_F32, 0, &h, (hipStream_t)stream);
  if (rc != IPFP_OK) return rc;
  rc = solve_handle(h, res, (hipStream_t)stream);
  destroy_handle(h);
  return rc;
}

// The one-call solve on the per-device scratch array: the same set-up, sweep
// kernels and read-out as ipfp_solve_market (so the same results, bit for
// bit), with the handle on the stack, the control block read into host stack
// memory and the loop timed on the host clock. Nothing is allocated.
int ipfp_solve_market_noalloc(ipfp_ctx* ctx, const ipfp_market* mk, const ipfp_options* opt,
                              ipfp_result* res, void* stream) {
  if (!ctx || !res || !res->a || !res->b) return IPFP_EINVAL;
  int rc = validate_market(mk, opt, true);
  if (rc != IPFP_OK) return rc;
  if (!ctx->noalloc) return IPFP_EHIP;
  hipStream_t s = (hipStream_t)stream;
  ipfp_handle h;
  h.ctx = ctx;
  h.mk = *mk;
  h.opt = *opt;
  h.opt.use_graph = 0;
  h.opt.time_passes = 0;
  h.plain = opt->path == IPFP_PATH_PLAIN;
  h.N = mk->N;
  h.M = mk->M;
  h.kdt = opt->compute == IPFP_F64 ? IPFP_F64 : IPFP_F32;
  h.arena = true;   // the memory is not the handle's
  Carver cv;
  handle_layout(&h, cv);
  h.bytes = align_up(cv.off, 256);
  if (h.bytes > (size_t)IPFP_NOALLOC_BYTES) return IPFP_EBUDGET;
  if (hipSetDevice(ctx->device) != hipSuccess) return IPFP_EHIP;
  const double t0 = now_ms();
  h.mem = static_cast<char*>(ctx->noalloc);
  Carver real;
  real.base = h.mem;
  handle_layout(&h, real);
  Ctl hc{};
  h.host_ctl = &hc;
  if (handle_setup(&h, nullptr, IPFP_F32, 0, s) != hipSuccess) return IPFP_EHIP;
  if (read_ctl(&h, s) != IPFP_OK) return IPFP_EHIP;
  if (hc.bad_margin) return IPFP_EINVAL;
  if (hc.nonfinite) return IPFP_ENONFINITE;
  h.setup_ms = now_ms() - t0;
  const int total = h.opt.max_sweeps + 1;   // +1: final residual row pass
  const int chunk = std::max(h.opt.check_every, 8);
  const double t1 = now_ms();
  for (bool done = false; !done;) {
    const int todo = std::min(chunk, total - h.units);
    for (int k = 0; k < todo; ++k) {
      if (enqueue_unit(&h, s, false) != hipSuccess) return IPFP_EHIP;
      h.units += 1;
    }
    if (read_ctl(&h, s) != IPFP_OK) return IPFP_EHIP;
    if (hc.nonfinite) return IPFP_ENONFINITE;
    done = hc.done || h.units >= total;
  }
  h.loop_ms = now_ms() - t1;
  rc = ipfp_market_read(&h, res->a, res->b, res, stream);
  h.host_ctl = nullptr;
  return rc;
}

// Sweep time of one candidate layout: open the market (set-up included in no
// timing), one warm-up sweep, then the mean of two timed sweeps. INFINITY when
// the candidate does not fit the budget.
static int time_candidate(ipfp_ctx* ctx, const ipfp_market* mk, const ipfp_options* opt,
                          int tile_rows, int splits, int splits_col, hipStream_t s,
                          double* ms) {
  const int kWarm = 1, kReps = 2;
  ipfp_options o = *opt;
  o.tile_rows = tile_rows;
  o.splits = splits;
  o.splits_col = splits_col;
  o.tol = 0.0;
  o.max_sweeps = kWarm + kReps + 1;
  o.check_every = kWarm + kReps + 1;
  o.use_graph = 0;
  o.time_passes = 0;
  ipfp_handle* h = nullptr;
  int rc = open_impl(ctx, mk, &o, nullptr, IPFP_F32, 0, &h, s);
  *ms = INFINITY;
  if (rc == IPFP_EBUDGET) return IPFP_OK;   // a candidate that does not fit is skipped
  if (rc != IPFP_OK) return rc;
  int done = 0;
  rc = run_impl(h, kWarm, &done, s);
  const double before = h->loop_ms;
  if (rc == IPFP_OK) rc = run_impl(h, kReps, &done, s);
  if (rc == IPFP_OK) *ms = (h->loop_ms - before) / kReps;
  destroy_handle(h);
  return rc;
}

int ipfp_tune(ipfp_ctx* ctx, const ipfp_market* mk, const ipfp_options* opt,
              ipfp_options* best, double* best_ms, void* stream) {
  if (!ctx || !mk || !opt || !best) return IPFP_EINVAL;
  if (opt->path != IPFP_PATH_FUSED) return IPFP_EINVAL;
  int rc = validate_market(mk, opt, true);
  if (rc != IPFP_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t kpad = fused_kpad(mk->d, opt->compute);
  double best_t = INFINITY;
  int win_tr = 0, win_sx = 0, win_sy = 0;
  // stage 1: workgroup height x row-pass splits (column pass automatic)
  std::vector<int> heights;
  if (opt->compute == IPFP_F32) heights = {128};
  else heights = {512, 256};
  for (int tr : heights) {
    const int sa = fused_pass_splits(mk->N, mk->M, kpad, opt->compute, tr);
    for (int sx : {sa, sa / 2, sa * 2}) {
      if (sx < 1 || sx > 256) continue;
      double t = 0.0;
      rc = time_candidate(ctx, mk, opt, tr, sx, 0, s, &t);
      if (rc != IPFP_OK) return rc;
      if (t < best_t) {
        best_t = t;
        win_tr = tr;
        win_sx = sx;
      }
    }
  }
  if (!(best_t < INFINITY)) return IPFP_EBUDGET;
  // stage 2: column-pass splits for the winner
  const int sc = fused_pass_splits(mk->M, mk->N, kpad, opt->compute, win_tr);
  win_sy = sc;
  for (int sy : {sc / 2, sc * 2}) {
    if (sy < 1 || sy > 256) continue;
    double t = 0.0;
    rc = time_candidate(ctx, mk, opt, win_tr, win_sx, sy, s, &t);
    if (rc != IPFP_OK) return rc;
    if (t < best_t) {
      best_t = t;
      win_sy = sy;
    }
  }
  *best = *opt;
  best->tile_rows = win_tr;
  best->splits = win_sx;
  best->splits_col = win_sy;
  if (best_ms) *best_ms = best_t;
  return IPFP_OK;
}

int ipfp_plan_market(const ipfp_market* mk, const ipfp_options* opt, ipfp_plan* out) {
  if (!out) return IPFP_EINVAL;
  int rc = validate_market(mk, opt, true);
  if (rc != IPFP_OK) return rc;
  if (opt->path != IPFP_PATH_FUSED) return IPFP_EINVAL;
  ipfp_handle h;
  h.mk = *mk;
  h.opt = *opt;
  h.N = mk->N;
  h.M = mk->M;
  Carver cv;
  handle_layout(&h, cv);
  const int tr = h.rowp.tile_rows;
  memset(out, 0, sizeof(*out));
  out->kpad = h.kpad;
  out->rows_per_workgroup = fused_rows_per_wg(h.kpad, opt->compute, tr);
  out->auto_splits_row = fused_pass_splits(mk->N, mk->M, h.kpad, opt->compute, tr);
  out->auto_splits_col = fused_pass_splits(mk->M, mk->N, h.kpad, opt->compute, tr);
  out->splits_row = h.rowp.splits;
  out->splits_col = h.colp.splits;
  const int64_t rows = out->rows_per_workgroup;
  out->blocks_row = (mk->N + rows - 1) / rows * out->splits_row;
  out->blocks_col = (mk->M + rows - 1) / rows * out->splits_col;
  out->footprint_bytes = align_up(cv.off, 256);
  return IPFP_OK;
}

int ipfp_solve_market_phi(ipfp_ctx* ctx, int64_t N, int64_t M, ipfp_dtype phi_dtype,
                          const void* Phi, int64_t ld_phi, const double* n,
                          const double* m, double sigma, const ipfp_options* opt,
                          ipfp_result* res, void* stream) {
  if (!ctx || !res || !res->a || !res->b || !Phi || !opt) return IPFP_EINVAL;
  if (phi_dtype != IPFP_F32 && phi_dtype != IPFP_F64) return IPFP_EINVAL;
  if (ld_phi < M) return IPFP_EINVAL;
  ipfp_market mk{};
  mk.N = N;
  mk.M = M;
  mk.d = 1;
  mk.n = n;
  mk.m = m;
  mk.sigma = sigma;
  ipfp_options o = *opt;
  o.path = IPFP_PATH_PLAIN;
  if (o.compute != IPFP_F64) o.compute = IPFP_F32;
  int rc = validate_market(&mk, &o, false);
  if (rc != IPFP_OK) return rc;
  ipfp_handle* h = nullptr;
  rc = open_impl(ctx, &mk, &o, Phi, phi_dtype, ld_phi, &h, (hipStream_t)stream);
  if (rc != IPFP_OK) return rc;
  rc = solve_handle(h, res, (hipStream_t)stream);
  destroy_handle(h);
  return rc;
}

int ipfp_mu_pairs(ipfp_ctx* ctx, const ipfp_market* mk, const double* a,
                  const double* b, const int64_t* xs, const int64_t* ys,
                  int64_t count, double* mu_out, void* stream) {
  if (!ctx || !mk || !a || !b || (count > 0 && (!xs || !ys || !mu_out)) || count < 0)
    return IPFP_EINVAL;
  if (!mk->U || !mk->Q || !mk->V || !mk->P || mk->d < 1 || !(mk->sigma > 0.0))
    return IPFP_EINVAL;
  if (mk->in_dtype == IPFP_FP8E4M3 && (!mk->scale_x || !mk->scale_y)) return IPFP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return IPFP_EHIP;
  int32_t* bad = nullptr;
  HIPCHK(hipMalloc((void**)&bad, sizeof(int32_t)));
  int rc = IPFP_OK;
  int32_t hb = 0;
  if (launch_zero(bad, sizeof(int32_t), s) != hipSuccess ||
      launch_mu_pairs(mk->U, mk->Q, mk->V, mk->P, mk->in_dtype, mk->scale_x, mk->scale_y,
                      mk->ld_x, mk->ld_y,
                      mk->N, mk->M, mk->d, mk->sigma, a, b, xs, ys, count, mu_out,
                      bad, s) != hipSuccess ||
      hipMemcpyAsync(&hb, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = IPFP_EHIP;
  (void)hipFree(bad);
  if (rc == IPFP_OK && hb) rc = IPFP_EINVAL;
  return rc;
}

int ipfp_margin_residuals(ipfp_ctx* ctx, const ipfp_market* mk, const double* a,
                          const double* b, double* row_res, double* col_res, double* max_row,
                          double* max_col, void* stream) {
  if (!ctx || !mk || !a || !b || !row_res || !col_res) return IPFP_EINVAL;
  if (mk->N < 1 || mk->M < 1 || mk->d < 1 || mk->d > 256 || !(mk->sigma > 0.0) ||
      !(mk->sigma < INFINITY))
    return IPFP_EINVAL;
  if (!mk->U || !mk->Q || !mk->V || !mk->P || !mk->n || !mk->m || mk->ld_x < mk->d ||
      mk->ld_y < mk->d)
    return IPFP_EINVAL;
  if (mk->in_dtype != IPFP_F64 && mk->in_dtype != IPFP_F32 && mk->in_dtype != IPFP_BF16 &&
      mk->in_dtype != IPFP_FP8E4M3)
    return IPFP_EINVAL;
  if (mk->in_dtype == IPFP_FP8E4M3 && (!mk->scale_x || !mk->scale_y)) return IPFP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return IPFP_EHIP;
  double* mx = nullptr;
  HIPCHK(hipMalloc((void**)&mx, 2 * sizeof(double)));
  double hm[2] = {0.0, 0.0};
  int rc = IPFP_OK;
  if (launch_margin_residual(mk->U, mk->Q, mk->scale_x, mk->ld_x, mk->V, mk->P, mk->scale_y,
                             mk->ld_y, mk->in_dtype, mk->N, mk->M, mk->d, mk->sigma, a, b,
                             mk->n, row_res, mx, s) != hipSuccess ||
      launch_margin_residual(mk->V, mk->P, mk->scale_y, mk->ld_y, mk->U, mk->Q, mk->scale_x,
                             mk->ld_x, mk->in_dtype, mk->M, mk->N, mk->d, mk->sigma, b, a,
                             mk->m, col_res, mx + 1, s) != hipSuccess ||
      hipMemcpyAsync(hm, mx, sizeof(hm), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = IPFP_EHIP;
  (void)hipFree(mx);
  if (rc == IPFP_OK) {
    if (max_row) *max_row = hm[0];
    if (max_col) *max_col = hm[1];
  }
  return rc;
}

int ipfp_stable_factors(ipfp_ctx* ctx, const ipfp_market* mk, const double* a,
                        const double* b, double* psi, int64_t ld_psi, double* xi,
                        int64_t ld_xi, void* stream) {
  if (!ctx || !mk || !a || !b || !psi || !xi) return IPFP_EINVAL;
  if (mk->N < 1 || mk->M < 1 || mk->d < 1 || mk->d > 256 || !(mk->sigma > 0.0)) return IPFP_EINVAL;
  if (!mk->U || !mk->Q || !mk->V || !mk->P || mk->ld_x < mk->d || mk->ld_y < mk->d)
    return IPFP_EINVAL;
  if (mk->in_dtype != IPFP_F64 && mk->in_dtype != IPFP_F32 && mk->in_dtype != IPFP_BF16 &&
      mk->in_dtype != IPFP_FP8E4M3)
    return IPFP_EINVAL;
  if (mk->in_dtype == IPFP_FP8E4M3 && (!mk->scale_x || !mk->scale_y)) return IPFP_EINVAL;
  const int64_t width = 2 * mk->d + 2;
  if (ld_psi < width || ld_xi < width) return IPFP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return IPFP_EHIP;
  HIPCHK(launch_stable_factors(mk->U, mk->Q, mk->in_dtype, mk->scale_x, mk->ld_x, mk->N,
                               mk->d, mk->sigma,
                               a, 0, psi, ld_psi, s));
  HIPCHK(launch_stable_factors(mk->V, mk->P, mk->in_dtype, mk->scale_y, mk->ld_y, mk->M,
                               mk->d, mk->sigma,
                               b, 1, xi, ld_xi, s));
  return IPFP_OK;
}

int ipfp_market_topk(ipfp_handle* h, int side, int32_t k, int32_t* idx_out, float* score_out,
                     void* stream) {
  if (!h || h->plain || (side != 0 && side != 1) || k < 1 || k > 32 || !idx_out || !score_out)
    return IPFP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(h->ctx->device) != hipSuccess) return IPFP_EHIP;
  int rc = read_ctl(h, s);
  if (rc != IPFP_OK) return rc;
  const Ctl c = *h->host_ctl;
  const int state = c.done ? c.stop_sweep : c.sweep;
  const double* u = h->u2 + (int64_t)(state & 1) * h->N;
  FusedPass fp = side == 0 ? h->rowp : h->colp;
  fp.w_red = side == 0 ? h->v : u;
  fp.red_dbuf = 0;
  const double* a_out = side == 0 ? u : h->v;
  const int64_t R = fp.out.rows, L = fp.red.rows;
  const int splits = topk_splits(R, L);
  const size_t entries = (size_t)splits * R * topk_width(k);
  const size_t bytes = align_up(entries * sizeof(float), 256) + entries * sizeof(int32_t);
  rc = ctx_reserve(h->ctx, bytes);
  if (rc != IPFP_OK) return rc;
  char* mem = nullptr;
  if (hipMalloc((void**)&mem, bytes) != hipSuccess) {
    ctx_release(h->ctx, bytes);
    return IPFP_EBUDGET;
  }
  float* pscore = (float*)mem;
  int32_t* pidx = (int32_t*)(mem + align_up(entries * sizeof(float), 256));
  rc = IPFP_OK;
  if (launch_topk(fp, a_out, k, splits, pscore, pidx, idx_out, score_out, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = IPFP_EHIP;
  (void)hipFree(mem);
  ctx_release(h->ctx, bytes);
  return rc;
}

int ipfp_market_gradient(ipfp_handle* h, int side, double* g_out, int64_t ld_g,
                         void* stream) {
  if (!h || h->plain || (side != 0 && side != 1) || !g_out) return IPFP_EINVAL;
  if (h->opt.compute != IPFP_BF16) return IPFP_EINVAL;
  const int width = (int)(2 * h->mk.d);
  if (ld_g < width) return IPFP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(h->ctx->device) != hipSuccess) return IPFP_EHIP;
  int rc = read_ctl(h, s);
  if (rc != IPFP_OK) return rc;
  const Ctl c = *h->host_ctl;
  const int state = c.done ? c.stop_sweep : c.sweep;
  const double* u = h->u2 + (int64_t)(state & 1) * h->N;
  FusedPass fp = side == 0 ? h->rowp : h->colp;
  fp.w_red = side == 0 ? h->v : u;
  fp.red_dbuf = 0;
  const double* a_out = side == 0 ? u : h->v;
  const int64_t R = fp.out.rows, L = fp.red.rows;
  // FP64 partials of at most 4 GiB
  const size_t per_split = (size_t)R * h->kpad * sizeof(double);
  const int max_splits = (int)std::max<size_t>(1, std::min<size_t>(64, ((size_t)4 << 30) / per_split));
  const int splits = gradient_splits(R, L, (int)h->kpad, max_splits);
  const size_t part = (size_t)splits * R * h->kpad * sizeof(double);
  const size_t imgb = gradient_scratch_bytes((int)h->kpad, L);
  const size_t bytes = align_up(sizeof(Ctl), 256) + align_up(part, 256) + imgb;
  rc = ctx_reserve(h->ctx, bytes);
  if (rc != IPFP_OK) return rc;
  char* mem = nullptr;
  if (hipMalloc((void**)&mem, bytes) != hipSuccess) {
    ctx_release(h->ctx, bytes);
    return IPFP_EBUDGET;
  }
  Ctl* sc = (Ctl*)mem;
  double* gpart = (double*)(mem + align_up(sizeof(Ctl), 256));
  uint8_t* img = (uint8_t*)(mem + align_up(sizeof(Ctl), 256) + align_up(part, 256));
  const double inv_p = 1.0 / (double)fused_prescale(h->mk.sigma);
  rc = IPFP_OK;
  if (launch_init_exp(fp.w_red, L, sc, 0, s) != hipSuccess ||
      launch_gradient(fp, &sc->wexp[0], a_out, inv_p, splits, gpart, img, width, g_out, ld_g,
                      s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = IPFP_EHIP;
  (void)hipFree(mem);
  ctx_release(h->ctx, bytes);
  return rc;
}

int ipfp_pack_side(ipfp_ctx* ctx, int64_t rows, int64_t d, ipfp_dtype in_dtype,
                   const void* A, const void* B, const float* in_scale, int64_t ld,
                   ipfp_dtype compute,
                   double sigma, void* out, float* scale_out, int64_t* kpad_out,
                   void* stream) {
  if (!ctx || !kpad_out || rows < 1 || d < 1 || d > 128 || ld < d) return IPFP_EINVAL;
  if (!(sigma >= 0.0) || !(sigma < INFINITY)) return IPFP_EINVAL;
  if (compute != IPFP_BF16 && compute != IPFP_FP8E4M3 && compute != IPFP_F32)
    return IPFP_EINVAL;
  const int64_t kpad = fused_kpad(d, compute);
  *kpad_out = kpad;
  if (!out) return IPFP_OK;
  if (!A || !B || (compute == IPFP_FP8E4M3 && !scale_out)) return IPFP_EINVAL;
  if (in_dtype != IPFP_F64 && in_dtype != IPFP_F32 && in_dtype != IPFP_BF16 &&
      in_dtype != IPFP_FP8E4M3)
    return IPFP_EINVAL;
  if (in_dtype == IPFP_FP8E4M3 && !in_scale) return IPFP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return IPFP_EHIP;
  char* mem = nullptr;
  const size_t bytes = align_up(sizeof(Ctl), 256) + rows * sizeof(float);
  HIPCHK(hipMalloc((void**)&mem, bytes));
  Ctl* ctl = (Ctl*)mem;
  float* sc = scale_out ? scale_out : (float*)(mem + align_up(sizeof(Ctl), 256));
  Ctl hc{};
  int rc = IPFP_OK;
  if (launch_zero(ctl, sizeof(Ctl), s) != hipSuccess ||
      launch_pack(A, B, in_dtype, in_scale, ld, rows, d, compute, kpad, fused_prescale(sigma), out,
                  sc, ctl, s) != hipSuccess ||
      hipMemcpyAsync(&hc, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = IPFP_EHIP;
  (void)hipFree(mem);
  if (rc == IPFP_OK && hc.bad_margin) rc = IPFP_EINVAL;
  if (rc == IPFP_OK && hc.nonfinite) rc = IPFP_ENONFINITE;
  return rc;
}

}  // extern "C"
