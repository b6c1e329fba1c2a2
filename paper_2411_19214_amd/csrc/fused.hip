// Fused (mini-batch) IPFP path for gfx950: the surplus Phi = [U|Q][V|P]^T is
// formed tile by tile on the matrix cores and consumed in registers, so the
// kernel K = exp(Phi / 2 sigma) is never stored (Sec. 3.3, eq. 9-10).
//
// One reduction pass computes, for every "output" row o (a candidate x in the
// row half-sweep, an employer y in the column half-sweep), the sum over the
// "reduced" side r of
//      2^( c (Phi_or + h_o) + beta_r ),   c = log2(e) / (2 sigma),
// where beta_r = log2 of the reduced side's current scaling and h_o is a
// per-row additive shift (in surplus units) chosen so the terms stay in FP32
// range. The matching row sum of eq. 6 is then (K w)_o = 2^(-c h_o) * sum.
//
// Work decomposition: a workgroup owns WAVES * XT * 32 output rows and one
// contiguous range ("split") of reduced-side tiles. Each wave keeps its
// output rows' operand fragments in registers for the whole pass; tiles of the
// reduced side (TY rows each) are staged through LDS (double-buffered) and
// shared by all waves. MFMA layout (32x32 outputs): the reduced rows are the
// A operand (M index), the output rows the B operand (N index), so a lane
// holds one output row (lane % 32) and 16 reduced rows; the shift enters as
// the accumulator's initial value, and a lane's 16 terms are summed in FP32
// and then added to an FP64 running sum. Partial sums per (split, row) are
// combined in fixed split order in FP64, so results are bitwise reproducible
// for a fixed split count.
#include <math.h>

#include <type_traits>

#include "common.h"

namespace ipfp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));

// ---- packing: [A|B] -> padded BF16 / FP8 rows ------------------------------

int64_t fused_kpad(int64_t d, ipfp_dtype compute) {
  const int64_t k2 = 2 * d;
  if (compute == IPFP_FP8E4M3) return ((k2 + 63) / 64) * 64;
  // BF16: multiples of 32 (two 16-wide MFMA k-steps) keep rows 64-byte aligned
  return ((k2 + 31) / 32) * 32;
}

__device__ __forceinline__ float in_as_float(const void* p, int64_t i,
                                             ipfp_dtype dt) {
  if (dt == IPFP_F64) return (float)static_cast<const double*>(p)[i];
  if (dt == IPFP_F32) return static_cast<const float*>(p)[i];
  return __uint_as_float((uint32_t)static_cast<const uint16_t*>(p)[i] << 16);
}

// BF16 round-to-nearest-even of an FP32 value.
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x7FFFFFu)) return 0x7FC0;
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// OCP e4m3fn code of a finite value with |f| <= 448 (round to nearest even).
__device__ __forceinline__ uint8_t e4m3_rne(float f) {
  uint8_t sign = f < 0.f ? 0x80 : 0;
  float a = fabsf(f);
  uint32_t code;
  if (a < 0.015625f) {                      // below 2^-6: steps of 2^-9
    code = (uint32_t)rintf(a * 512.f);      // 8 rounds up to the smallest normal
  } else {
    int e;
    frexpf(a, &e);                          // a = m 2^e, m in [0.5, 1)
    e -= 1;                                 // a in [2^e, 2^(e+1))
    int q = (int)rintf(ldexpf(a, 3 - e));   // in [8, 16]
    if (q == 16) { q = 8; e += 1; }
    code = (uint32_t)(((e + 7) << 3) | (q - 8));
  }
  if (code > 0x7E) code = 0x7E;             // saturate at 448
  return sign | (uint8_t)code;
}

__device__ __forceinline__ float e4m3_val(uint8_t c) {
  const int e = (c >> 3) & 0xF, f = c & 7;
  float v = e == 0 ? ldexpf((float)f, -9) : ldexpf((float)(8 + f), e - 10);
  return (c & 0x80) ? -v : v;
}

// One wave per row. BF16: codes of RNE(fp32(x)). FP8: power-of-two scale
// s = 2^e with the smallest e such that amax <= 448 s, codes e4m3(x / s).
// Also writes the 2-norm of the packed (dequantised) row.
__global__ void __launch_bounds__(256)
    k_pack(const void* A, const void* B, ipfp_dtype in_dt, int64_t ld,
           int64_t rows, int64_t d, ipfp_dtype compute, int64_t kpad, void* out,
           float* scale, float* norm, Ctl* ctl) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int64_t k2 = 2 * d;
  bool finite = true;
  float amax = 0.f;
  for (int64_t k = lane; k < k2; k += 64) {
    float x = k < d ? in_as_float(A, row * ld + k, in_dt)
                    : in_as_float(B, row * ld + k - d, in_dt);
    finite &= (x - x == 0.f);
    amax = fmaxf(amax, fabsf(x));
  }
  if (!finite) atomicOr(&ctl->nonfinite, 1);
  float ss = 0.f;
  if (compute == IPFP_FP8E4M3) {
    amax = wave_max(amax);
    int e = 0;
    if (amax > 0.f) {
      int ex;
      float mant = frexpf(amax, &ex);
      e = mant <= 0.875f ? ex - 9 : ex - 8;
    }
    uint8_t* o = static_cast<uint8_t*>(out) + row * kpad;
    for (int64_t k = lane; k < kpad; k += 64) {
      uint8_t code = 0;
      if (k < k2) {
        float x = k < d ? in_as_float(A, row * ld + k, in_dt)
                        : in_as_float(B, row * ld + k - d, in_dt);
        code = e4m3_rne(ldexpf(x, -e));
        float q = ldexpf(e4m3_val(code), e);
        ss = fmaf(q, q, ss);
      }
      o[k] = code;
    }
    if (lane == 0) scale[row] = ldexpf(1.f, e);
  } else {
    uint16_t* o = static_cast<uint16_t*>(out) + row * kpad;
    for (int64_t k = lane; k < kpad; k += 64) {
      uint16_t code = 0;
      if (k < k2) {
        if (in_dt == IPFP_BF16)
          code = k < d ? static_cast<const uint16_t*>(A)[row * ld + k]
                       : static_cast<const uint16_t*>(B)[row * ld + k - d];
        else
          code = bf16_rne(k < d ? in_as_float(A, row * ld + k, in_dt)
                                : in_as_float(B, row * ld + k - d, in_dt));
        float q = __uint_as_float((uint32_t)code << 16);
        ss = fmaf(q, q, ss);
      }
      o[k] = code;
    }
  }
  ss = wave_sum(ss);
  if (lane == 0) norm[row] = sqrtf(ss);
}

hipError_t launch_pack(const void* A, const void* B, ipfp_dtype in_dt,
                       int64_t ld, int64_t rows, int64_t d, ipfp_dtype compute,
                       int64_t kpad, void* out, float* scale, float* norm,
                       Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, A,
                     B, in_dt, ld, rows, d, compute, kpad, out, scale, norm, ctl);
  return hipGetLastError();
}

// ---- the reduction pass ------------------------------------------------------

// Operand traits: bytes per element, bytes a lane feeds one MFMA (SB) and the
// K extent of one MFMA (KS).
template <bool FP8>
struct Op;
template <>
struct Op<false> {  // BF16, v_mfma_f32_32x32x16_bf16
  static constexpr int ES = 2, SB = 16, KS = 16;
};
template <>
struct Op<true> {  // FP8 e4m3, v_mfma_scale_f32_32x32x64_f8f6f4
  static constexpr int ES = 1, SB = 32, KS = 64;
};

// Reduced rows staged per LDS buffer (a multiple of 32) and whether the
// epilogue is explicitly interleaved with the next accumulator's MFMAs; both
// are build-time tuning knobs.
#ifndef IPFP_TY
#define IPFP_TY 64
#endif
#ifndef IPFP_SCHED
#define IPFP_SCHED 1
#endif
constexpr int kTY = IPFP_TY;

template <int KP, int XT, int WAVES, bool FP8>
__global__ void __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(2)))
    k_fused_pass(const uint8_t* __restrict__ Xo, const float* __restrict__ xscale,
                 const uint8_t* __restrict__ Yr, const float* __restrict__ yscale,
                 const float* __restrict__ bias, const float* __restrict__ shift,
                 float c, int R, int L, int tiles_per_split, int nsplit,
                 double* __restrict__ part, Ctl* ctl) {
  typedef Op<FP8> O;
  constexpr int RB = KP * O::ES;           // bytes per packed row
  constexpr int NS = KP / O::KS;           // MFMAs per 32x32 output tile
  constexpr int LS = RB + 16;              // LDS row stride (bank-conflict pad)
  constexpr int NT = WAVES * 64;
  constexpr int CH = kTY * RB / 16;        // 16-byte chunks per stage
  constexpr int CPT = (CH + NT - 1) / NT;  // chunks per thread
  constexpr int SUB = kTY / 32;

  __shared__ __attribute__((aligned(16))) uint8_t ys[2][kTY * LS];
  __shared__ __attribute__((aligned(16))) float bs[2][kTY];
  __shared__ int32_t ysc[2][kTY];          // FP8: E8M0 scale byte per row

  if (ctl->done) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->fix_rows = 0;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int split = blockIdx.x % nsplit;
  const int rb = blockIdx.x / nsplit;
  const int T = (L + kTY - 1) / kTY;
  const int t0 = split * tiles_per_split;
  const int t1 = min(T, t0 + tiles_per_split);
  const int row_base = (rb * WAVES + wave) * (XT * 32);

  // output-side operand fragments, shift accumulators and scales (registers)
  typedef typename std::conditional<FP8, intx8, bf16x8>::type Frag;
  Frag bfrag[XT][NS];
  floatx16 shv[XT];
  int xsc[XT];
#pragma unroll
  for (int t = 0; t < XT; ++t) {
    const int x = row_base + t * 32 + l32;
    const bool ok = x < R;
    const uint8_t* src = Xo + (int64_t)(ok ? x : 0) * RB + h * O::SB;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (FP8) {
        intx4 lo = ok ? *reinterpret_cast<const intx4*>(src + s * 2 * O::SB) : intx4{0, 0, 0, 0};
        intx4 hi = ok ? *reinterpret_cast<const intx4*>(src + s * 2 * O::SB + 16) : intx4{0, 0, 0, 0};
        intx8 v;
        v[0] = lo[0]; v[1] = lo[1]; v[2] = lo[2]; v[3] = lo[3];
        v[4] = hi[0]; v[5] = hi[1]; v[6] = hi[2]; v[7] = hi[3];
        *reinterpret_cast<intx8*>(&bfrag[t][s]) = v;
      } else {
        intx4 v = ok ? *reinterpret_cast<const intx4*>(src + s * 2 * O::SB) : intx4{0, 0, 0, 0};
        *reinterpret_cast<intx4*>(&bfrag[t][s]) = v;
      }
    }
    const float hv = ok ? shift[x] : 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) shv[t][r] = hv;
    xsc[t] = FP8 && ok ? (int)((__float_as_uint(xscale[x]) >> 23) & 0xFF) : 127;
  }

  double run[XT];
#pragma unroll
  for (int t = 0; t < XT; ++t) run[t] = 0.0;

  // stage loader: global -> registers -> LDS
  intx4 pre[CPT];
  float pb = 0.f;
  int psc = 127;
  auto gload = [&](int tile) {
    // Branch-free, so that a whole tile is one scheduling region: rows past
    // the end are clamped to the last row (a valid read) and masked by a -inf
    // bias; surplus threads repeat the last chunk, and every thread loads the
    // bias of row tid % kTY (duplicates store identical values).
    const int64_t y0 = (int64_t)tile * kTY;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int chunk = min(tid + q * NT, CH - 1);
      const int r = chunk / (RB / 16), cb = chunk % (RB / 16);
      const int64_t y = min(y0 + r, (int64_t)L - 1);
      pre[q] = *reinterpret_cast<const intx4*>(Yr + y * RB + cb * 16);
    }
    const int64_t y = y0 + (tid % kTY);
    const int64_t yc = min(y, (int64_t)L - 1);
    const float bb = bias[yc];
    pb = y < L ? bb : -INFINITY;
    if (FP8) psc = (int)((__float_as_uint(yscale[yc]) >> 23) & 0xFF);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int chunk = min(tid + q * NT, CH - 1);
      const int r = chunk / (RB / 16), cb = chunk % (RB / 16);
      *reinterpret_cast<intx4*>(&ys[buf][r * LS + cb * 16]) = pre[q];
    }
    bs[buf][tid % kTY] = pb;
    if (FP8) ysc[buf][tid % kTY] = psc;
  };

  // The epilogue (exp2 and sums) of each 32x32 accumulator runs while the
  // matrix cores compute the next one: `accp` holds the accumulator whose
  // epilogue is pending, `bvp` its biases; its output tile is always the one
  // computed just before the current one, so its running-sum index is static.
  // The first pending epilogue is a dummy with -inf biases (adds zero).
  floatx16 accp;
  float bvp[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    accp[r] = 0.f;
    bvp[r] = -INFINITY;
  }
  auto epilogue = [&](const floatx16& a, const float* b, double& acc_run) {
    float e[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) e[r] = __builtin_amdgcn_exp2f(fmaf(a[r], c, b[r]));
#pragma unroll
    for (int w = 8; w > 0; w >>= 1)
#pragma unroll
      for (int r = 0; r < w; ++r) e[r] += e[r + w];
    acc_run += (double)e[0];
  };
  // VALU instructions of one epilogue (16 fma, 16 exp, 15 add, cvt, add_f64)
  // spread over the NS matrix instructions of the next accumulator
  constexpr int kEpiValu = 49;
  constexpr int kValuPerMfma = (kEpiValu + NS - 1) / NS;

  if (t0 < t1) {
    gload(t0);
    lstore(0);
  }
  __syncthreads();

  for (int tile = t0; tile < t1; ++tile) {
    const int buf = (tile - t0) & 1;
    gload(min(tile + 1, t1 - 1));   // prefetch (the last iteration reloads harmlessly)
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub) {
      const uint8_t* arow = &ys[buf][(sub * 32 + l32) * LS + h * O::SB];
      Frag afrag[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (FP8) {
          intx4 lo = *reinterpret_cast<const intx4*>(arow + s * 2 * O::SB);
          intx4 hi = *reinterpret_cast<const intx4*>(arow + s * 2 * O::SB + 16);
          intx8 v;
          v[0] = lo[0]; v[1] = lo[1]; v[2] = lo[2]; v[3] = lo[3];
          v[4] = hi[0]; v[5] = hi[1]; v[6] = hi[2]; v[7] = hi[3];
          *reinterpret_cast<intx8*>(&afrag[s]) = v;
        } else {
          *reinterpret_cast<intx4*>(&afrag[s]) =
              *reinterpret_cast<const intx4*>(arow + s * 2 * O::SB);
        }
      }
      const int asc = FP8 ? ysc[buf][sub * 32 + l32] : 127;
      // bias of the 16 reduced rows this lane holds: 8 g + 4 h + (0..3)
      float bv[16];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float4 b4 = *reinterpret_cast<const float4*>(&bs[buf][sub * 32 + 8 * g + 4 * h]);
        bv[4 * g + 0] = b4.x;
        bv[4 * g + 1] = b4.y;
        bv[4 * g + 2] = b4.z;
        bv[4 * g + 3] = b4.w;
      }
#pragma unroll
      for (int t = 0; t < XT; ++t) {
        floatx16 acc = shv[t];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if constexpr (FP8) {
            acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                *reinterpret_cast<intx8*>(&afrag[s]), *reinterpret_cast<intx8*>(&bfrag[t][s]),
                acc, 0, 0, 0, asc, 0, xsc[t]);
          } else {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(afrag[s], bfrag[t][s], acc, 0, 0, 0);
          }
        }
        epilogue(accp, bvp, run[t == 0 ? XT - 1 : t - 1]);
#if IPFP_SCHED
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);             // MFMA
          __builtin_amdgcn_sched_group_barrier(0x002, kValuPerMfma, 0);  // VALU
        }
#endif
        accp = acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) bvp[r] = bv[r];
      }
    }
    lstore(buf ^ 1);
    __syncthreads();
  }
  epilogue(accp, bvp, run[XT - 1]);

#pragma unroll
  for (int t = 0; t < XT; ++t) {
    const double tot = run[t] + __shfl_xor(run[t], 32, 64);
    const int x = row_base + t * 32 + l32;
    if (h == 0 && x < R) part[(int64_t)split * R + x] = tot;
  }
}

// ---- combine partial sums, update scalings -----------------------------------

// Finishes output row o given lS = log2((K w)_o): the residual of the current
// scaling (eq. 5), the quadratic root of eq. 6, the FP32 log2 of the new
// scaling (bias of the other half-sweep) and the next shift.
__device__ __forceinline__ double finish_row(int64_t o, double lS, float c,
                                             const double* marg,
                                             const double* w_old, double* w_new,
                                             float* lw_new, float* shift,
                                             bool residual, Ctl* ctl) {
  const double nx = marg[o];
  double res = 0.0;
  if (residual) {
    const double wo = w_old[o];
    const double two_s_wo = wo > 0.0 ? exp2(log2(wo) + lS) : 0.0;
    res = fabs(fma(wo, wo, -nx) + two_s_wo) / nx;
  }
  const double w = lS < 1000.0 ? quad_root(nx, exp2(lS - 1.0)) : nx * exp2(-lS);
  if (!(w - w == 0.0)) atomicOr(&ctl->nonfinite, 1);
  w_new[o] = w;
  lw_new[o] = (float)log2(w);
  const double hn = -lS / (double)c;
  shift[o] = (hn - hn == 0.0) ? (float)hn : 0.f;
  return res;
}

__global__ void __launch_bounds__(256)
    k_fused_combine(const double* __restrict__ part, int splits, int64_t R,
                    float* shift, float c, const double* __restrict__ marg,
                    double* w2, int dbuf, float* lw_new, double* res_block,
                    int32_t* fix_list, int residual, Ctl* ctl) {
  __shared__ double red[4];
  if (ctl->done) return;
  const int i = ctl->sweep;
  const double* w_old = dbuf ? w2 + (int64_t)(i & 1) * R : w2;
  double* w_new = dbuf ? w2 + (int64_t)((i + 1) & 1) * R : w2;
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double res = 0.0;
  if (o < R) {
    double l = 0.0;
    for (int k = 0; k < splits; ++k) l += part[(int64_t)k * R + o];
    if (!(l >= 0x1p-60) || l == INFINITY) {  // out of safe range (or NaN)
      const int slot = atomicAdd(&ctl->fix_rows, 1);
      fix_list[slot] = (int32_t)o;
    } else {
      const double lS = log2(l) - (double)c * (double)shift[o];
      res = finish_row(o, lS, c, marg, w_old, w_new, lw_new, shift,
                       residual != 0, ctl);
    }
  }
  res = wave_max(res);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = res;
  __syncthreads();
  if (threadIdx.x == 0)
    res_block[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Exact-shift fallback for rows whose shifted sum left the safe range: two
// passes over the reduced side with FP32 dot products of the same packed
// operands, the first for the maximum exponent, the second for the sum.
template <bool FP8>
__device__ __forceinline__ float dot_packed(const uint8_t* a, const uint8_t* b,
                                            int kpad) {
  float acc = 0.f;
  if (FP8) {
    for (int k = 0; k < kpad; ++k) acc = fmaf(e4m3_val(a[k]), e4m3_val(b[k]), acc);
  } else {
    const uint16_t* a16 = reinterpret_cast<const uint16_t*>(a);
    const uint16_t* b16 = reinterpret_cast<const uint16_t*>(b);
    for (int k = 0; k < kpad; ++k)
      acc = fmaf(__uint_as_float((uint32_t)a16[k] << 16),
                 __uint_as_float((uint32_t)b16[k] << 16), acc);
  }
  return acc;
}

template <bool FP8>
__global__ void __launch_bounds__(256)
    k_fused_fixup(const uint8_t* Xo, const float* xscale, const uint8_t* Yr,
                  const float* yscale, int kpad, const float* bias, float* shift,
                  float c, int64_t L, int64_t R, const double* marg, double* w2,
                  int dbuf, float* lw_new, double* res_slot,
                  const int32_t* fix_list, int residual, Ctl* ctl) {
  __shared__ float fred[4];
  __shared__ double dred[4];
  if (ctl->done) return;
  const int count = ctl->fix_rows;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->fix_total += count;
  const int i = ctl->sweep;
  const double* w_old = dbuf ? w2 + (int64_t)(i & 1) * R : w2;
  double* w_new = dbuf ? w2 + (int64_t)((i + 1) & 1) * R : w2;
  const int ES = FP8 ? 1 : 2;
  double res = 0.0;
  for (int k = blockIdx.x; k < count; k += gridDim.x) {
    const int64_t o = fix_list[k];
    const uint8_t* xr = Xo + o * kpad * ES;
    const float sx = FP8 ? xscale[o] : 1.f;
    float tmax = -INFINITY;
    for (int64_t y = threadIdx.x; y < L; y += 256) {
      const float sc = FP8 ? sx * yscale[y] : 1.f;
      const float t = fmaf(dot_packed<FP8>(xr, Yr + y * kpad * ES, kpad) * sc, c, bias[y]);
      tmax = fmaxf(tmax, t);
    }
    tmax = wave_max(tmax);
    if ((threadIdx.x & 63) == 0) fred[threadIdx.x >> 6] = tmax;
    __syncthreads();
    tmax = fmaxf(fmaxf(fred[0], fred[1]), fmaxf(fred[2], fred[3]));
    double sum = 0.0;
    if (tmax > -INFINITY) {
      for (int64_t y = threadIdx.x; y < L; y += 256) {
        const float sc = FP8 ? sx * yscale[y] : 1.f;
        const float t = fmaf(dot_packed<FP8>(xr, Yr + y * kpad * ES, kpad) * sc, c, bias[y]);
        sum += exp2((double)t - (double)tmax);
      }
    }
    sum = wave_sum(sum);
    if ((threadIdx.x & 63) == 0) dred[threadIdx.x >> 6] = sum;
    __syncthreads();
    sum = (dred[0] + dred[1]) + (dred[2] + dred[3]);
    const double lS = sum > 0.0 ? (double)tmax + log2(sum) : -INFINITY;
    if (threadIdx.x == 0) {
      double r = finish_row(o, lS, c, marg, w_old, w_new, lw_new, shift,
                            residual != 0, ctl);
      res = fmax(res, r);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) res_slot[blockIdx.x] = res;
}

// ---- shifts for the first pass, small vector kernels -------------------------

// out[0] = max_k f[k] (f may be null), out[1] = log2(max_k w[k]) (w may be
// null: 0). One workgroup.
__global__ void __launch_bounds__(256)
    k_max_pair(const float* f, int64_t nf, const double* w, int64_t nw,
               float* out) {
  __shared__ float a[256];
  __shared__ double b[256];
  float fm = 0.f;
  double wm = 0.0;
  for (int64_t k = threadIdx.x; f && k < nf; k += 256) fm = fmaxf(fm, f[k]);
  for (int64_t k = threadIdx.x; w && k < nw; k += 256) wm = fmax(wm, w[k]);
  a[threadIdx.x] = fm;
  b[threadIdx.x] = wm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      a[threadIdx.x] = fmaxf(a[threadIdx.x], a[threadIdx.x + o]);
      b[threadIdx.x] = fmax(b[threadIdx.x], b[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = a[0];
    out[1] = w ? (float)log2(b[0]) : 0.f;
  }
}

// Shift from the Cauchy-Schwarz bound c Phi_or <= c |x_o| max_r |y_r| plus
// the largest bias: every first-pass term is then <= 1.
__global__ void k_shift_init(const float* onorm, int64_t R, const float* mx,
                             float lscale, float c, float* shift) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= R) return;
  const double g = (double)c * (double)onorm[o] * (double)mx[0] * 1.0001 +
                   (double)lscale * (double)mx[1];
  shift[o] = (float)(-g / (double)c);
}

hipError_t launch_initial_shift(const FusedSide& out, const FusedSide& red,
                                float c, double lscale, const double* wmax_src,
                                int64_t wmax_len, float* shift, float* tmp,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_max_pair, dim3(1), dim3(256), 0, s, red.norm, red.rows,
                     wmax_src, wmax_len, tmp);
  hipLaunchKernelGGL(k_shift_init, dim3((unsigned)((out.rows + 255) / 256)),
                     dim3(256), 0, s, out.norm, out.rows, tmp, (float)lscale, c,
                     shift);
  return hipGetLastError();
}

__global__ void k_log2_vec(const double* w, float* lw, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < len) lw[i] = (float)log2(w[i]);
}

hipError_t launch_log2_vec(const double* w, float* lw, int64_t len,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_log2_vec, dim3((unsigned)((len + 255) / 256)), dim3(256), 0,
                     s, w, lw, len);
  return hipGetLastError();
}

// ---- dispatch ---------------------------------------------------------------

template <int KP, int XT, int WAVES, bool FP8>
static hipError_t pass_t(const FusedPass& fp, Ctl* ctl, hipStream_t s) {
  const int rows_per_wg = WAVES * XT * 32;
  const int64_t rblocks = (fp.out.rows + rows_per_wg - 1) / rows_per_wg;
  const int T = (int)((fp.red.rows + kTY - 1) / kTY);
  const int tps = (T + fp.splits - 1) / fp.splits;
  const int64_t grid = rblocks * fp.splits;
  hipLaunchKernelGGL((k_fused_pass<KP, XT, WAVES, FP8>), dim3((unsigned)grid),
                     dim3(WAVES * 64), 0, s, (const uint8_t*)fp.out.ops,
                     fp.out.scale, (const uint8_t*)fp.red.ops, fp.red.scale,
                     fp.bias, fp.shift, fp.c, (int)fp.out.rows, (int)fp.red.rows,
                     tps, fp.splits, fp.part, ctl);
  return hipGetLastError();
}

template <int KP, bool FP8>
static hipError_t pass_kp(const FusedPass& fp, Ctl* ctl, hipStream_t s) {
  // register budget: two 32-row output tiles per wave while the operand
  // fragments of both fit in 64 VGPRs per lane
  constexpr int XT = (KP * Op<FP8>::ES <= (FP8 ? 128 : 256)) ? 2 : 1;
  if (fp.tile_rows >= 512 / (2 / XT)) return pass_t<KP, XT, 8, FP8>(fp, ctl, s);
  return pass_t<KP, XT, 4, FP8>(fp, ctl, s);
}

hipError_t launch_fused_pass(const FusedPass& fp, Ctl* ctl, hipStream_t s) {
  if (fp.compute == IPFP_FP8E4M3) {
    switch (fp.kpad) {
      case 64: return pass_kp<64, true>(fp, ctl, s);
      case 128: return pass_kp<128, true>(fp, ctl, s);
      case 192: return pass_kp<192, true>(fp, ctl, s);
      case 256: return pass_kp<256, true>(fp, ctl, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (fp.kpad) {
    case 32: return pass_kp<32, false>(fp, ctl, s);
    case 64: return pass_kp<64, false>(fp, ctl, s);
    case 96: return pass_kp<96, false>(fp, ctl, s);
    case 128: return pass_kp<128, false>(fp, ctl, s);
    case 160: return pass_kp<160, false>(fp, ctl, s);
    case 192: return pass_kp<192, false>(fp, ctl, s);
    case 224: return pass_kp<224, false>(fp, ctl, s);
    case 256: return pass_kp<256, false>(fp, ctl, s);
    default: return hipErrorInvalidValue;
  }
}

int fused_rows_per_wg(int64_t kpad, ipfp_dtype compute, int tile_rows) {
  const bool fp8 = compute == IPFP_FP8E4M3;
  const int es = fp8 ? 1 : 2;
  const int xt = (kpad * es <= (fp8 ? 128 : 256)) ? 2 : 1;
  const int waves = tile_rows >= 512 / (2 / xt) ? 8 : 4;
  return waves * xt * 32;
}

hipError_t launch_fused_combine(const FusedPass& fp, double* w2, int dbuf,
                                Ctl* ctl, int* nblocks, hipStream_t s) {
  const int64_t blocks = (fp.out.rows + 255) / 256;
  *nblocks = (int)blocks;
  hipLaunchKernelGGL(k_fused_combine, dim3((unsigned)blocks), dim3(256), 0, s,
                     fp.part, fp.splits, fp.out.rows, fp.shift, fp.c, fp.marg, w2,
                     dbuf, fp.lw_new, fp.res_block, fp.fix_list,
                     fp.residual ? 1 : 0, ctl);
  return hipGetLastError();
}

constexpr int kFixupBlocks = 64;
int fused_fixup_blocks() { return kFixupBlocks; }

hipError_t launch_fused_fixup(const FusedPass& fp, double* w2, int dbuf,
                              double* res_slot, Ctl* ctl, hipStream_t s) {
  if (fp.compute == IPFP_FP8E4M3)
    hipLaunchKernelGGL(k_fused_fixup<true>, dim3(kFixupBlocks), dim3(256), 0, s,
                       (const uint8_t*)fp.out.ops, fp.out.scale,
                       (const uint8_t*)fp.red.ops, fp.red.scale, (int)fp.kpad,
                       fp.bias, fp.shift, fp.c, fp.red.rows, fp.out.rows, fp.marg,
                       w2, dbuf, fp.lw_new, res_slot, fp.fix_list,
                       fp.residual ? 1 : 0, ctl);
  else
    hipLaunchKernelGGL(k_fused_fixup<false>, dim3(kFixupBlocks), dim3(256), 0, s,
                       (const uint8_t*)fp.out.ops, fp.out.scale,
                       (const uint8_t*)fp.red.ops, fp.red.scale, (int)fp.kpad,
                       fp.bias, fp.shift, fp.c, fp.red.rows, fp.out.rows, fp.marg,
                       w2, dbuf, fp.lw_new, res_slot, fp.fix_list,
                       fp.residual ? 1 : 0, ctl);
  return hipGetLastError();
}

int fused_auto_splits(int64_t R, int64_t L, int rows_per_wg) {
  // Enough workgroups to fill 256 CUs several times over, and at most ~4096
  // reduced rows per... keep every split at least 8 tiles long.
  const int64_t rblocks = (R + rows_per_wg - 1) / rows_per_wg;
  const int64_t T = (L + kTY - 1) / kTY;
  int64_t S = 1;
  while (rblocks * S < 2048 && S * 2 <= 64 && T / (S * 2) >= 8) S *= 2;
  return (int)S;
}

}  // namespace ipfp
