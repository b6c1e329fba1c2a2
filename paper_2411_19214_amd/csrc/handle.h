// Internal: contexts and resident-market handles, shared by the one-call
// solves (runtime.hip) and the serving scheduler (serve.hip).
#pragma once

#include <chrono>
#include <mutex>
#include <vector>

#include "common.h"

struct ipfp_ctx {
  int device;
  size_t budget;
  size_t used;
  std::mutex mu;
  void* noalloc = nullptr;  // device address of the allocation-free solve's
                            // scratch array on this context's device
};

namespace ipfp {

constexpr int kHistCap = 4096;  // device residual history entries per market

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Carves one device allocation into aligned sub-buffers.
struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

inline size_t dtype_size(ipfp_dtype t) {
  switch (t) {
    case IPFP_F64: return 8;
    case IPFP_F32: return 4;
    case IPFP_BF16: return 2;
    default: return 1;
  }
}

inline double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace ipfp

struct ipfp_handle {
  ipfp_ctx* ctx = nullptr;
  ipfp_market mk{};
  ipfp_options opt{};
  bool plain = false;
  int64_t N = 0, M = 0;
  size_t bytes = 0;
  char* mem = nullptr;
  // shared state
  ipfp::Ctl* ext_ctl = nullptr;  // control block supplied by the owner (serving)
  bool arena = false;            // `mem` belongs to a serving arena, not this handle
  ipfp::Ctl* ctl = nullptr;
  double* hist = nullptr;
  double* res_block = nullptr;   // row residual maxima, one per row-combine workgroup
  double* res_dummy = nullptr;   // column side writes its (unused) maxima here
  double* u2 = nullptr;          // 2 x N double buffer
  double* v = nullptr;           // M
  int nres_row = 0;              // entries of res_block the check reduces
  // plain path
  ipfp_dtype kdt = IPFP_F32;
  void* K = nullptr;
  int64_t ldk = 0;
  double* cshift = nullptr;
  double* ut = nullptr;
  double* part = nullptr;
  int psplits = 1;
  // fused path
  int64_t kpad = 0;
  void *xop = nullptr, *yop = nullptr;
  float *xscale = nullptr, *yscale = nullptr;
  float *xshift = nullptr, *yshift = nullptr;
  double *xpart = nullptr, *ypart = nullptr;
  ipfp::FusedPass rowp{}, colp{};
  int row_combine_blocks = 0, col_combine_blocks = 0;
  // loop state
  int units = 0;                 // sweep units enqueued so far
  ipfp::Ctl* host_ctl = nullptr; // pinned mirror
  hipGraphExec_t graph = nullptr;
  int graph_units = 0;
  hipStream_t cap_stream = nullptr;
  std::vector<hipEvent_t> evs;   // pass timing events (pairs)
  double pass_ms = 0.0;
  int pass_launches = 0;
  double loop_ms = 0.0;
  double setup_ms = 0.0;
};


namespace ipfp {

// Carves (base != null) or sizes (base == null) a handle's device memory.
void handle_layout(ipfp_handle* h, Carver& cv);
// Enqueues a market's set-up on `s`: control block, margin check, v = b0 or 1,
// then packing and the fixed shifts (fused) or K (plain). Failures of the
// device checks show up as Ctl flags, read by the caller.
hipError_t handle_setup(ipfp_handle* h, const void* phi, ipfp_dtype phi_dt, int64_t ld_phi,
                        hipStream_t s);
int validate_market(const ipfp_market* mk, const ipfp_options* opt, bool factors);
int ctx_reserve(ipfp_ctx* ctx, size_t bytes);
void ctx_release(ipfp_ctx* ctx, size_t bytes);
SweepParams handle_sweep_params(const ipfp_handle* h);

}  // namespace ipfp
