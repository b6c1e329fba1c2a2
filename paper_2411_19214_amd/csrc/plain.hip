// Plain (batch) IPFP path: K = exp(Phi / 2 sigma) materialised once, then two
// HBM-streaming matrix-vector passes per sweep (eq. 7, Alg. 1).
//
// Storage: K is kept as K'_xy = exp(Phi_xy / 2 sigma - c_x) with the row
// shift c_x = max_y Phi_xy / 2 sigma, so every stored entry is in (0, 1] and
// FP32 storage cannot overflow for any surplus whose row-wise spread fits the
// format. The factor e^{c_x} is applied in FP64 on the side: the row pass
// scales its FP64 sum by e^{c_x}, the column pass multiplies by
// ut_x = e^{c_x} u_x. All sums and updates are FP64; only K is FP32 (or FP64
// for the FP64 instantiation).
#include <math.h>

#include "common.h"

namespace ipfp {

// ---- Phi from factors (one-time set-up of the plain path) ------------------

template <typename T>
__device__ __forceinline__ double to_d(T x) {
  return (double)x;
}
template <>
__device__ __forceinline__ double to_d<uint16_t>(uint16_t x) {
  return (double)__uint_as_float((uint32_t)x << 16);
}
template <>
__device__ __forceinline__ double to_d<uint8_t>(uint8_t x) {   // e4m3 code
  return (double)e4m3_val(x);
}

// Phi_xy = sum_k U_xk V_yk + Q_xk P_yk in FP64, written to K's buffer in the
// storage type TK. 64 x 64 output tile per 256 threads, 4 x 4 per thread.
// FP8 input (TIN = uint8_t codes) is scaled by its rows' scales sx, sy.
template <typename TIN, typename TK>
__global__ void __launch_bounds__(256)
    k_phi_factors(const TIN* U, const TIN* Q, const TIN* V, const TIN* P,
                  const float* sx, const float* sy,
                  int64_t ld_x, int64_t ld_y, int64_t N, int64_t M, int64_t d,
                  TK* K, int64_t ldk) {
  constexpr int TB = 64, KC = 16;
  __shared__ double xs[KC][TB + 1];
  __shared__ double ys[KC][TB + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t x0 = (int64_t)blockIdx.y * TB, y0 = (int64_t)blockIdx.x * TB;
  double acc[4][4] = {};
  const int64_t K2 = 2 * d;
  for (int64_t k0 = 0; k0 < K2; k0 += KC) {
    for (int e = threadIdx.x; e < TB * KC; e += 256) {
      int r = e / KC, kk = e % KC;
      int64_t k = k0 + kk;
      int64_t x = x0 + r, y = y0 + r;
      double xv = 0.0, yv = 0.0;
      if (k < K2) {
        if (x < N) {
          xv = k < d ? to_d(U[x * ld_x + k]) : to_d(Q[x * ld_x + k - d]);
          if (sx) xv *= (double)sx[x];
        }
        if (y < M) {
          yv = k < d ? to_d(V[y * ld_y + k]) : to_d(P[y * ld_y + k - d]);
          if (sy) yv *= (double)sy[y];
        }
      }
      xs[kk][r] = xv;
      ys[kk][r] = yv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = xs[kk][ty + 16 * q];
        b[q] = ys[kk][tx + 16 * q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    int64_t x = x0 + ty + 16 * p;
    if (x >= N) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int64_t y = y0 + tx + 16 * q;
      if (y < M) K[x * ldk + y] = (TK)acc[p][q];
    }
  }
}

template <typename TIN, typename TK>
static hipError_t phi_factors_t(const void* U, const void* Q, const void* V,
                                const void* P, const float* sx, const float* sy,
                                int64_t ld_x, int64_t ld_y, int64_t N, int64_t M, int64_t d,
                                void* K, int64_t ldk, hipStream_t s) {
  dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
  hipLaunchKernelGGL((k_phi_factors<TIN, TK>), grid, dim3(256), 0, s,
                     (const TIN*)U, (const TIN*)Q, (const TIN*)V, (const TIN*)P, sx, sy,
                     ld_x, ld_y, N, M, d, (TK*)K, ldk);
  return hipGetLastError();
}

template <typename TK>
static hipError_t phi_factors_k(const void* U, const void* Q, const void* V, const void* P,
                                ipfp_dtype dt, const float* sx, const float* sy,
                                int64_t ld_x, int64_t ld_y, int64_t N, int64_t M, int64_t d,
                                void* K, int64_t ldk, hipStream_t s) {
  switch (dt) {
    case IPFP_F64:
      return phi_factors_t<double, TK>(U, Q, V, P, nullptr, nullptr, ld_x, ld_y, N, M, d, K,
                                       ldk, s);
    case IPFP_F32:
      return phi_factors_t<float, TK>(U, Q, V, P, nullptr, nullptr, ld_x, ld_y, N, M, d, K,
                                      ldk, s);
    case IPFP_FP8E4M3:
      return phi_factors_t<uint8_t, TK>(U, Q, V, P, sx, sy, ld_x, ld_y, N, M, d, K, ldk, s);
    default:
      return phi_factors_t<uint16_t, TK>(U, Q, V, P, nullptr, nullptr, ld_x, ld_y, N, M, d,
                                         K, ldk, s);
  }
}

hipError_t launch_phi_from_factors(const void* U, const void* Q, const void* V,
                                   const void* P, ipfp_dtype dt, const float* scale_x,
                                   const float* scale_y, int64_t ld_x,
                                   int64_t ld_y, int64_t N, int64_t M,
                                   int64_t d, void* Kbuf, ipfp_dtype kdt,
                                   int64_t ldk, hipStream_t s) {
  if (kdt == IPFP_F64)
    return phi_factors_k<double>(U, Q, V, P, dt, scale_x, scale_y, ld_x, ld_y, N, M, d, Kbuf,
                                 ldk, s);
  return phi_factors_k<float>(U, Q, V, P, dt, scale_x, scale_y, ld_x, ld_y, N, M, d, Kbuf,
                              ldk, s);
}

// ---- K = exp(Phi / 2 sigma - c_x) -------------------------------------------

// One workgroup per row: c_x = max_y Phi_xy / 2 sigma, then the shifted
// exponentials. Src and dst may alias (Phi computed into K's buffer).
template <typename TP, typename TK>
__global__ void __launch_bounds__(256)
    k_materialize(const TP* Phi, int64_t ldp, TK* K, int64_t ldk, int64_t M,
                  double inv2s, double* cshift, Ctl* ctl) {
  __shared__ double red[4];
  const int64_t x = blockIdx.x;
  const TP* row = Phi + x * ldp;
  double mx = -INFINITY;
  bool finite = true;
  for (int64_t y = threadIdx.x; y < M; y += 256) {
    double p = (double)row[y];
    finite &= __builtin_isfinite(p);
    mx = p > mx ? p : mx;
  }
  if (!finite) atomicOr(&ctl->nonfinite, 1);
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  const double c = mx * inv2s;
  if (threadIdx.x == 0) cshift[x] = c;
  TK* krow = K + x * ldk;
  for (int64_t y = threadIdx.x; y < M; y += 256) {
    double p = (double)row[y];
    krow[y] = (TK)exp(fma(p, inv2s, -c));
  }
}

hipError_t launch_materialize(const void* Phi, ipfp_dtype pdt, int64_t ldp,
                              void* Kbuf, ipfp_dtype kdt, int64_t ldk,
                              int64_t N, int64_t M, double sigma,
                              double* cshift, Ctl* ctl, hipStream_t s) {
  const double inv2s = 1.0 / (2.0 * sigma);
  dim3 grid((unsigned)N);
  if (pdt == IPFP_F64 && kdt == IPFP_F64)
    hipLaunchKernelGGL((k_materialize<double, double>), grid, dim3(256), 0, s,
                       (const double*)Phi, ldp, (double*)Kbuf, ldk, M, inv2s, cshift, ctl);
  else if (pdt == IPFP_F64 && kdt == IPFP_F32)
    hipLaunchKernelGGL((k_materialize<double, float>), grid, dim3(256), 0, s,
                       (const double*)Phi, ldp, (float*)Kbuf, ldk, M, inv2s, cshift, ctl);
  else if (pdt == IPFP_F32 && kdt == IPFP_F64)
    hipLaunchKernelGGL((k_materialize<float, double>), grid, dim3(256), 0, s,
                       (const float*)Phi, ldp, (double*)Kbuf, ldk, M, inv2s, cshift, ctl);
  else
    hipLaunchKernelGGL((k_materialize<float, float>), grid, dim3(256), 0, s,
                       (const float*)Phi, ldp, (float*)Kbuf, ldk, M, inv2s, cshift, ctl);
  return hipGetLastError();
}

// ---- row pass: s_x = (1/2) e^{c_x} sum_y K'_xy v_y, then u_x ----------------

template <typename TK>
struct Vec16;  // 16-byte vector of TK
template <>
struct Vec16<float> {
  typedef float4 T;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  typedef double2 T;
  static constexpr int n = 2;
};

// 16 bytes of K. K is read once per pass and is larger than the caches, so
// the load is marked nontemporal (streaming).
template <typename TK>
__device__ __forceinline__ typename Vec16<TK>::T load_k(const TK* p) {
  typedef TK v16 __attribute__((ext_vector_type(16 / sizeof(TK))));
  const v16 r = __builtin_nontemporal_load(reinterpret_cast<const v16*>(p));
  typename Vec16<TK>::T o;
  __builtin_memcpy(&o, &r, 16);
  return o;
}

template <typename TK>
__device__ __forceinline__ void vec_get(const typename Vec16<TK>::T& v, double* o);
template <>
__device__ __forceinline__ void vec_get<float>(const float4& v, double* o) {
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <>
__device__ __forceinline__ void vec_get<double>(const double2& v, double* o) {
  o[0] = v.x; o[1] = v.y;
}

constexpr int kRowsPerWave = 4;

// Four waves per workgroup, four rows per wave: each lane streams 16-byte
// chunks of the four rows and reuses the matching chunk of v from registers.
// The lane-strided FP64 partial sums are combined by a fixed butterfly, so the
// result is bitwise reproducible. Row residual of the state being replaced:
// |u_old^2 + 2 u_old s - n| / n (eq. 5).
template <typename TK>
__global__ void __launch_bounds__(256)
    k_plain_row(const TK* __restrict__ K, int64_t ldk, int64_t N, int64_t M,
                const double* __restrict__ cshift, const double* __restrict__ v,
                const double* __restrict__ n, double* u2, double* ut,
                double* res_block, Ctl* ctl) {
  __shared__ double red[4];
  if (ctl->done) return;
  constexpr int VN = Vec16<TK>::n;
  typedef typename Vec16<TK>::T VT;
  const int i = ctl->sweep;
  const double* u_old = u2 + (int64_t)(i & 1) * N;
  double* u_new = u2 + (int64_t)((i + 1) & 1) * N;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * kRowsPerWave;
  const TK* rp[kRowsPerWave];
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    int64_t x = row0 + r < N ? row0 + r : N - 1;
    rp[r] = K + x * ldk;
  }
  double acc[kRowsPerWave] = {};
  const int64_t Mv = (M / VN) * VN;
  for (int64_t j = (int64_t)lane * VN; j < Mv; j += 64 * VN) {
    double vv[VN];
#pragma unroll
    for (int e = 0; e < VN; ++e) vv[e] = v[j + e];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      VT kv = load_k<TK>(rp[r] + j);
      double kd[VN];
      vec_get<TK>(kv, kd);
#pragma unroll
      for (int e = 0; e < VN; ++e) acc[r] = fma(kd[e], vv[e], acc[r]);
    }
  }
  for (int64_t j = Mv + lane; j < M; j += 64) {
    double vj = v[j];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) acc[r] = fma((double)rp[r][j], vj, acc[r]);
  }
  double res = 0.0;
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    double S = wave_sum(acc[r]);
    const int64_t x = row0 + r;
    if (lane == r && x < N) {
      const double ec = exp(cshift[x]);
      const double s = 0.5 * ec * S;
      const double uo = u_old[x], nx = n[x];
      res = fabs(fma(uo, uo, -nx) + 2.0 * uo * s) / nx;
      const double un = quad_root(nx, s);
      if (!__builtin_isfinite(un)) atomicOr(&ctl->nonfinite, 1);
      u_new[x] = un;
      ut[x] = ec * un;
    }
  }
  res = wave_max(res);
  if (lane == 0) red[wave] = res;
  __syncthreads();
  if (threadIdx.x == 0)
    res_block[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

hipError_t launch_plain_row(const void* K, ipfp_dtype kdt, int64_t ldk,
                            int64_t N, int64_t M, const double* cshift,
                            const double* v, const double* n, double* u2,
                            double* ut, double* res_block, int* nblocks,
                            Ctl* ctl, hipStream_t s) {
  const int64_t blocks = (N + 4 * kRowsPerWave - 1) / (4 * kRowsPerWave);
  *nblocks = (int)blocks;
  if (kdt == IPFP_F64)
    hipLaunchKernelGGL(k_plain_row<double>, dim3((unsigned)blocks), dim3(256), 0,
                       s, (const double*)K, ldk, N, M, cshift, v, n, u2, ut,
                       res_block, ctl);
  else
    hipLaunchKernelGGL(k_plain_row<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float*)K, ldk, N, M, cshift, v, n, u2, ut,
                       res_block, ctl);
  return hipGetLastError();
}

// ---- column pass: s_y = (1/2) sum_x K'_xy ut_x, split over row ranges ------

constexpr int kColRowUnroll = 4;

// Each thread owns one 16-byte column chunk and walks the rows of its split:
// a wave reads 1 KiB of one row per step (coalesced), ut_x is uniform across
// the workgroup. Partials go to part[split][y] and are summed in split order.
template <typename TK>
__global__ void __launch_bounds__(256)
    k_plain_col(const TK* __restrict__ K, int64_t ldk, int64_t N, int64_t M,
                const double* __restrict__ ut, int rows_per_split,
                double* __restrict__ part, Ctl* ctl) {
  if (ctl->done) return;
  constexpr int VN = Vec16<TK>::n;
  typedef typename Vec16<TK>::T VT;
  const int64_t y0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * VN;
  const int split = blockIdx.y;
  const int64_t x0 = (int64_t)split * rows_per_split;
  const int64_t x1 = x0 + rows_per_split < N ? x0 + rows_per_split : N;
  if (y0 >= M) return;
  double acc[VN] = {};
  const bool full = y0 + VN <= M;
  if (full) {
    int64_t x = x0;
    for (; x + kColRowUnroll <= x1; x += kColRowUnroll) {
      VT kv[kColRowUnroll];
#pragma unroll
      for (int q = 0; q < kColRowUnroll; ++q)
        kv[q] = load_k<TK>(K + (x + q) * ldk + y0);
#pragma unroll
      for (int q = 0; q < kColRowUnroll; ++q) {
        double kd[VN];
        vec_get<TK>(kv[q], kd);
        const double w = ut[x + q];
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[e] = fma(kd[e], w, acc[e]);
      }
    }
    for (; x < x1; ++x) {
      VT kv = load_k<TK>(K + x * ldk + y0);
      double kd[VN];
      vec_get<TK>(kv, kd);
      const double w = ut[x];
#pragma unroll
      for (int e = 0; e < VN; ++e) acc[e] = fma(kd[e], w, acc[e]);
    }
  } else {
    for (int64_t x = x0; x < x1; ++x) {
      const double w = ut[x];
      for (int e = 0; e < VN; ++e)
        if (y0 + e < M) acc[e] = fma((double)K[x * ldk + y0 + e], w, acc[e]);
    }
  }
  double* out = part + (int64_t)split * M;
#pragma unroll
  for (int e = 0; e < VN; ++e)
    if (y0 + e < M) out[y0 + e] = acc[e];
}

__global__ void __launch_bounds__(256)
    k_col_combine(const double* __restrict__ part, int splits, int64_t M,
                  const double* __restrict__ m, double* v, Ctl* ctl) {
  if (ctl->done) return;
  const int64_t y = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (y >= M) return;
  double S = 0.0;
  for (int k = 0; k < splits; ++k) S += part[(int64_t)k * M + y];
  const double vn = quad_root(m[y], 0.5 * S);
  if (!__builtin_isfinite(vn)) atomicOr(&ctl->nonfinite, 1);
  v[y] = vn;
}

int plain_splits(int64_t N, int64_t M, ipfp_dtype kdt) {
  const int VN = kdt == IPFP_F64 ? 2 : 4;
  const int64_t colblocks = (M + 256 * VN - 1) / (256 * VN);
  int64_t S = (2048 + colblocks - 1) / colblocks;
  const int64_t maxS = (N + 63) / 64;  // keep >= 64 rows per split
  if (S > maxS) S = maxS;
  if (S < 1) S = 1;
  if (S > 256) S = 256;
  return (int)S;
}

hipError_t launch_plain_col(const void* K, ipfp_dtype kdt, int64_t ldk,
                            int64_t N, int64_t M, const double* ut, int splits,
                            double* part, const double* m, double* v, Ctl* ctl,
                            hipStream_t s) {
  const int VN = kdt == IPFP_F64 ? 2 : 4;
  const int64_t colblocks = (M + 256 * VN - 1) / (256 * VN);
  const int rps = (int)((N + splits - 1) / splits);
  dim3 grid((unsigned)colblocks, (unsigned)splits);
  if (kdt == IPFP_F64)
    hipLaunchKernelGGL(k_plain_col<double>, grid, dim3(256), 0, s,
                       (const double*)K, ldk, N, M, ut, rps, part, ctl);
  else
    hipLaunchKernelGGL(k_plain_col<float>, grid, dim3(256), 0, s,
                       (const float*)K, ldk, N, M, ut, rps, part, ctl);
  hipLaunchKernelGGL(k_col_combine, dim3((unsigned)((M + 255) / 256)), dim3(256),
                     0, s, part, splits, M, m, v, ctl);
  return hipGetLastError();
}

}  // namespace ipfp
