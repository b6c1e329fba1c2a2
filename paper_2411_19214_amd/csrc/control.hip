// Convergence control (single-market and grouped), small vector kernels and
// the outputs computed from the factors as given: matching masses at pairs
// and the stable factors.
#include <math.h>

#include "common.h"

namespace ipfp {

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

__global__ void __launch_bounds__(256) k_check(Ctl* ctl, const double* res_block,
                                               int nblocks, double* hist,
                                               SweepParams sp) {
  check_body(ctl, res_block, nblocks, hist, sp);
}

// One workgroup per market.
__global__ void __launch_bounds__(256) k_group_check(const GroupCheck* __restrict__ c) {
  const GroupCheck& g = c[blockIdx.x];
  check_body(g.ctl, g.res_block, g.nblocks, g.hist, g.sp);
}

hipError_t launch_group_check(const GroupCheck* c, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_group_check, dim3((unsigned)count), dim3(256), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_check(Ctl* ctl, const double* res_block, int nblocks,
                        double* hist, SweepParams sp, hipStream_t s) {
  hipLaunchKernelGGL(k_check, dim3(1), dim3(256), 0, s, ctl, res_block, nblocks,
                     hist, sp);
  return hipGetLastError();
}

// Zero fill of `words` 32-bit words (control blocks and other small scratch
// that must start at zero; a kernel rather than a memset node, so that the
// set-up can sit inside a captured graph).
__global__ void k_zero_words(int32_t* p, int64_t words) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t words = (int64_t)((bytes + 3) / 4);
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                     static_cast<int32_t*>(p), words);
  return hipGetLastError();
}

__global__ void k_init_vec(double* v, const double* src, int64_t len) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) v[i] = src ? src[i] : 1.0;
}

hipError_t launch_init_vec(double* v, const double* src, int64_t len,
                           hipStream_t s) {
  int64_t blocks = (len + 255) / 256;
  hipLaunchKernelGGL(k_init_vec, dim3((unsigned)blocks), dim3(256), 0, s, v, src,
                     len);
  return hipGetLastError();
}

__global__ void k_validate(const double* a, int64_t len, Ctl* ctl) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) {
    double x = a[i];
    if (!(x > 0.0) || !(x < INFINITY)) atomicOr(&ctl->bad_margin, 1);
  }
}

// FP8 input: every row scale must be a positive, normal power of two.
__global__ void k_validate_scales(const float* s, int64_t len, Ctl* ctl) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len && !pow2_scale_ok(s[i])) atomicOr(&ctl->bad_margin, 1);
}

hipError_t launch_validate_scales(const float* sx, int64_t N, const float* sy, int64_t M,
                                  Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_scales, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                     sx, N, ctl);
  hipLaunchKernelGGL(k_validate_scales, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s,
                     sy, M, ctl);
  return hipGetLastError();
}

hipError_t launch_validate_margins(const double* n, int64_t N, const double* m,
                                   int64_t M, Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                     s, n, N, ctl);
  hipLaunchKernelGGL(k_validate, dim3((unsigned)((M + 255) / 256)), dim3(256), 0,
                     s, m, M, ctl);
  return hipGetLastError();
}

template <typename T>
__device__ __forceinline__ double ld_as_double(const void* p, int64_t i) {
  return (double)static_cast<const T*>(p)[i];
}

__device__ __forceinline__ double ld_elem(const void* p, int64_t i,
                                          ipfp_dtype dt) {
  switch (dt) {
    case IPFP_F64:
      return static_cast<const double*>(p)[i];
    case IPFP_F32:
      return (double)static_cast<const float*>(p)[i];
    case IPFP_FP8E4M3:   // code value; the caller applies the row scale
      return (double)e4m3_val(static_cast<const uint8_t*>(p)[i]);
    default: {  // BF16 codes
      uint32_t bits = (uint32_t)static_cast<const uint16_t*>(p)[i] << 16;
      return (double)__uint_as_float(bits);
    }
  }
}

// mu_xy = exp(Phi_xy / 2 sigma) a_x b_y at requested pairs (eq. 4), with the
// surplus formed in FP64 from the factors as given.
// Stable factors (eq. 11): one output row [A_x, B_x, c0, c1] of 2d + 2 FP64
// values, with the log entry 2 sigma log w_x in column 2d + log_col and 1 in
// the other (2 sigma, not the printed sigma: with w = sqrt of the unmatched
// mass this is sigma log mu_x0, which makes the inner product reproduce
// eq. 4).
__global__ void k_stable_factors(const void* A, const void* B, ipfp_dtype dt,
                                 const float* in_scale, int64_t ld,
                                 int64_t rows, int64_t d, double sigma, const double* w,
                                 int log_col, double* out, int64_t ld_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t width = 2 * d + 2;
  if (i >= rows * width) return;
  const int64_t r = i / width, c = i % width;
  const double rs = dt == IPFP_FP8E4M3 ? (double)in_scale[r] : 1.0;
  double v;
  if (c < d) {
    v = ld_elem(A, r * ld + c, dt) * rs;
  } else if (c < 2 * d) {
    v = ld_elem(B, r * ld + (c - d), dt) * rs;
  } else if (c - 2 * d == log_col) {
    v = 2.0 * sigma * log(w[r]);
  } else {
    v = 1.0;
  }
  out[r * ld_out + c] = v;
}

hipError_t launch_stable_factors(const void* A, const void* B, ipfp_dtype dt,
                                 const float* in_scale, int64_t ld,
                                 int64_t rows, int64_t d, double sigma, const double* w,
                                 int log_col, double* out, int64_t ld_out, hipStream_t s) {
  const int64_t n = rows * (2 * d + 2);
  hipLaunchKernelGGL(k_stable_factors, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     A, B, dt, in_scale, ld, rows, d, sigma, w, log_col, out, ld_out);
  return hipGetLastError();
}

__global__ void k_mu_pairs(const void* U, const void* Q, const void* V,
                           const void* P, ipfp_dtype dt, const float* scale_x,
                           const float* scale_y, int64_t ld_x,
                           int64_t ld_y, int64_t N, int64_t M, int64_t d,
                           double sigma, const double* a, const double* b,
                           const int64_t* xs, const int64_t* ys, int64_t count,
                           double* mu, int32_t* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int64_t x = xs[i], y = ys[i];
  if (x < 0 || x >= N || y < 0 || y >= M) {
    mu[i] = NAN;
    atomicOr(bad, 1);
    return;
  }
  double phi = 0.0;
  for (int64_t k = 0; k < d; ++k) {
    phi = fma(ld_elem(U, x * ld_x + k, dt), ld_elem(V, y * ld_y + k, dt), phi);
    phi = fma(ld_elem(Q, x * ld_x + k, dt), ld_elem(P, y * ld_y + k, dt), phi);
  }
  // FP8 input: the row scales are powers of two, so scaling the sum is exact
  if (dt == IPFP_FP8E4M3) phi *= (double)scale_x[x] * (double)scale_y[y];
  mu[i] = exp(phi / (2.0 * sigma)) * a[x] * b[y];
}

hipError_t launch_mu_pairs(const void* U, const void* Q, const void* V,
                           const void* P, ipfp_dtype dt, const float* scale_x,
                           const float* scale_y, int64_t ld_x,
                           int64_t ld_y, int64_t N, int64_t M, int64_t d,
                           double sigma, const double* a, const double* b,
                           const int64_t* xs, const int64_t* ys, int64_t count,
                           double* mu, int32_t* bad, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mu_pairs, dim3((unsigned)((count + 255) / 256)), dim3(256),
                     0, s, U, Q, V, P, dt, scale_x, scale_y, ld_x, ld_y, N, M, d, sigma,
                     a, b, xs, ys, count, mu, bad);
  return hipGetLastError();
}

}  // namespace ipfp
