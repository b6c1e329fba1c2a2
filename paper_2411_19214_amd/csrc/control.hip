// Convergence control (single-market and grouped), small vector kernels and
// the outputs computed from the factors as given: matching masses at pairs
// and the stable factors.
#include <math.h>

#include <algorithm>

#include "common.h"

namespace ipfp {

__global__ void __launch_bounds__(256) k_check(Ctl* ctl, const double* res_block,
                                               int nblocks, double* hist,
                                               SweepParams sp) {
  check_body(ctl, res_block, nblocks, hist, sp);
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
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
    p[i] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t words = (int64_t)((bytes + 3) / 4);
  if (words == 0) return hipSuccess;
  // grid-stride: at most 65536 workgroups (a grid's x extent times its
  // workgroup size must stay below 2^32)
  const int64_t blocks = std::min<int64_t>((words + 255) / 256, 65536);
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, s,
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

// ---- margin residuals of eq. 5 against the surplus as given ------------------
//
// For every output row o (a candidate x: other side the employers, or an
// employer y), with mu_or = exp(Phi_or / (2 sigma) + log w_o + log w_r)
// (eq. 4) and Phi formed in FP64 from the factors as given:
//     res_o = |w_o^2 + sum_r mu_or - marg_o| / marg_o,
// the residual of eq. 5's margin equation (w_o^2 = mu_o0). Each mu is formed
// directly in the log domain, so no intermediate overflows for any scalings a
// solve returns. One workgroup per 64 output rows loops over the other side in
// 64-row tiles; 4 x 4 pairs per thread, surplus chunks of 16 factor columns
// through LDS, FP64 throughout; the 16 partial sums of a row are added in a
// fixed order, so the result is deterministic.
__global__ void __launch_bounds__(256)
    k_margin_residual(const void* A, const void* B, const float* sa, int64_t lda,
                      const void* C, const void* D, const float* sc, int64_t ldc,
                      ipfp_dtype dt, int64_t R, int64_t L, int64_t d, double inv2s,
                      const double* w_out, const double* w_red, const double* marg,
                      double* res) {
  constexpr int TB = 64, KC = 16;
  __shared__ double xs[KC][TB + 1];
  __shared__ double ys[KC][TB + 1];
  __shared__ double lw[TB];
  __shared__ double part[16][TB + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t o0 = (int64_t)blockIdx.x * TB;
  const int64_t K2 = 2 * d;
  double lo[4], rsum[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int64_t o = o0 + ty + 16 * p;
    lo[p] = o < R ? log(w_out[o]) : 0.0;
  }
  for (int64_t r0 = 0; r0 < L; r0 += TB) {
    if (threadIdx.x < TB) {
      const int64_t r = r0 + threadIdx.x;
      lw[threadIdx.x] = r < L ? log(w_red[r]) : -INFINITY;
    }
    double acc[4][4] = {};
    for (int64_t k0 = 0; k0 < K2; k0 += KC) {
      for (int e = threadIdx.x; e < TB * KC; e += 256) {
        const int i = e / KC, kk = e % KC;
        const int64_t k = k0 + kk, o = o0 + i, r = r0 + i;
        double xv = 0.0, yv = 0.0;
        if (k < K2) {
          if (o < R) {
            xv = k < d ? ld_elem(A, o * lda + k, dt) : ld_elem(B, o * lda + k - d, dt);
            if (dt == IPFP_FP8E4M3) xv *= (double)sa[o];
          }
          if (r < L) {
            yv = k < d ? ld_elem(C, r * ldc + k, dt) : ld_elem(D, r * ldc + k - d, dt);
            if (dt == IPFP_FP8E4M3) yv *= (double)sc[r];
          }
        }
        xs[kk][i] = xv;
        ys[kk][i] = yv;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        double a4[4], b4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a4[q] = xs[kk][ty + 16 * q];
          b4[q] = ys[kk][tx + 16 * q];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p][q] = fma(a4[p], b4[q], acc[p][q]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rsum[p] += exp(acc[p][q] * inv2s + lo[p] + lw[tx + 16 * q]);   // 0 past the end
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) part[tx][ty + 16 * p] = rsum[p];
  __syncthreads();
  if (threadIdx.x < TB) {
    const int64_t o = o0 + threadIdx.x;
    if (o < R) {
      double sum = 0.0;
      for (int j = 0; j < 16; ++j) sum += part[j][threadIdx.x];
      const double w = w_out[o], mg = marg[o];
      res[o] = fabs(fma(w, w, -mg) + sum) / mg;
    }
  }
}

// out[0] = max of x[0..n) (one workgroup; NaN propagates).
__global__ void __launch_bounds__(256) k_max_of(const double* x, int64_t n, double* out) {
  __shared__ double red[256];
  double r = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = x[i];
    r = (v > r || v != v) ? v : r;
  }
  red[threadIdx.x] = r;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double a = red[threadIdx.x], b = red[threadIdx.x + o];
      red[threadIdx.x] = (b > a || b != b) ? b : a;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_margin_residual(const void* A, const void* B, const float* sa, int64_t lda,
                                  const void* C, const void* D, const float* sc, int64_t ldc,
                                  ipfp_dtype dt, int64_t R, int64_t L, int64_t d, double sigma,
                                  const double* w_out, const double* w_red, const double* marg,
                                  double* res, double* max_out, hipStream_t s) {
  hipLaunchKernelGGL(k_margin_residual, dim3((unsigned)((R + 63) / 64)), dim3(256), 0, s, A, B,
                     sa, lda, C, D, sc, ldc, dt, R, L, d, 0.5 / sigma, w_out, w_red, marg, res);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !max_out) return e;
  hipLaunchKernelGGL(k_max_of, dim3(1), dim3(256), 0, s, res, R, max_out);
  return hipGetLastError();
}

}  // namespace ipfp
