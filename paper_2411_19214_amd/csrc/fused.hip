// Fused (mini-batch) IPFP path for gfx950: the surplus Phi = [U|Q][V|P]^T is
// formed tile by tile on the matrix cores and consumed in registers, so the
// kernel K = exp(Phi / 2 sigma) is never stored (Sec. 3.3, eq. 9-10).
//
// Scaling. Both packed operands are multiplied by sqrt(c), c = log2(e) /
// (2 sigma), before rounding to BF16 / FP8, so one matrix product yields the
// surplus already in log2 units: T_xy = <sqrt(c) x_x, sqrt(c) y_y> = c Phi_xy
// and K_xy = 2^T_xy. Every output row o gets a fixed shift h_o = -max_r T_or,
// found once by a max pass at set-up (the surplus never changes between
// sweeps), so every term 2^(T + h) lies in (0, 1].
//
// One reduction pass then computes, for every output row o (a candidate x in
// the row half-sweep, an employer y in the column half-sweep),
//      S_o = sum_r 2^(T_or + h_o) w~_r,   w~_r = w_r 2^-E,
// where w is the reduced side's current scaling (v for the row pass, u for the
// column pass) and E its largest binary exponent, so (K w)_o = 2^(E - h_o) S_o
// (eq. 6, eq. 9). Per pair that is one exp2 and one FMA on the VALU.
//
// Work decomposition: a workgroup owns WAVES * XT * 32 output rows and one
// contiguous range ("split") of reduced-side tiles. Each wave keeps its
// output rows' operand fragments in registers for the whole pass; tiles of the
// reduced side (kTY rows each) are staged through LDS (double-buffered) and
// shared by all waves. MFMA layout (32x32 outputs): the reduced rows are the
// A operand (M index), the output rows the B operand (N index), so a lane
// holds one output row (lane % 32) and 16 reduced rows; the shift enters as
// the accumulator's initial value; a lane's 16 weighted terms are summed in
// FP32 and added to an FP64 running sum. Partial sums per (split, row) are
// combined in fixed split order in FP64, so results are bitwise reproducible
// for a fixed split count.
//
// The same tile machinery serves the grouped (many-market) launches of the
// serving layer, the recommendation lists (top-k epilogue instead of the sum)
// and the welfare gradient (a second matrix-core product of the exp'd tile
// with the value rows).
#include <limits.h>
#include <math.h>

#include <atomic>
#include <type_traits>

#include "common.h"

namespace ipfp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef int intx4 __attribute__((ext_vector_type(4)));

// ---- packing: sqrt(c) [A|B] -> padded BF16 / FP8 rows ----------------------

int64_t fused_kpad(int64_t d, ipfp_dtype compute) {
  const int64_t k2 = 2 * d;
  if (compute == IPFP_FP8E4M3) return ((k2 + 63) / 64) * 64;
  // BF16 and FP32: multiples of 32 (two 16-wide BF16 MFMA k-steps, four
  // 8-wide FP32 k-steps) keep rows 64-byte aligned
  return ((k2 + 31) / 32) * 32;
}

float fused_prescale(double sigma) {
  return sigma > 0.0 ? (float)sqrt(1.4426950408889634 / (2.0 * sigma)) : 1.0f;
}

__device__ __forceinline__ float in_as_float(const void* p, int64_t i,
                                             ipfp_dtype dt) {
  if (dt == IPFP_F64) return (float)static_cast<const double*>(p)[i];
  if (dt == IPFP_F32) return static_cast<const float*>(p)[i];
  if (dt == IPFP_FP8E4M3) return e4m3_val(static_cast<const uint8_t*>(p)[i]);
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

// One wave per row; every value is first rounded to FP32 (FP8 input: the
// code's value times the row's power-of-two scale, exact) and multiplied by
// the prescale p in FP32. BF16: codes of RNE(p x). FP8: power-of-two scale
// s = 2^e with the smallest e such that amax(p x) <= 448 s, codes
// e4m3(p x / s). FP32: the FP32 products p x themselves.
__global__ void __launch_bounds__(256)
    k_pack(const void* A, const void* B, ipfp_dtype in_dt, const float* in_scale, int64_t ld,
           int64_t rows, int64_t d, ipfp_dtype compute, int64_t kpad, float p,
           void* out, float* scale, Ctl* ctl) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int64_t k2 = 2 * d;
  const float rs = in_dt == IPFP_FP8E4M3 ? in_scale[row] : 1.f;
  if (in_dt == IPFP_FP8E4M3 && lane == 0 && !pow2_scale_ok(rs)) atomicOr(&ctl->bad_margin, 1);
  auto val = [&](int64_t k) {
    const float x = k < d ? in_as_float(A, row * ld + k, in_dt)
                          : in_as_float(B, row * ld + k - d, in_dt);
    return (x * rs) * p;
  };
  bool finite = true;
  float amax = 0.f;
  for (int64_t k = lane; k < k2; k += 64) {
    const float x = val(k);
    finite &= __builtin_isfinite(x);
    amax = fmaxf(amax, fabsf(x));
  }
  if (!finite) atomicOr(&ctl->nonfinite, 1);
  if (compute == IPFP_FP8E4M3) {
    amax = wave_max(amax);
    int e = 0;
    if (amax > 0.f) {
      int ex;
      float mant = frexpf(amax, &ex);
      e = mant <= 0.875f ? ex - 9 : ex - 8;
    }
    uint8_t* o = static_cast<uint8_t*>(out) + row * kpad;
    for (int64_t k = lane; k < kpad; k += 64)
      o[k] = k < k2 ? e4m3_rne(ldexpf(val(k), -e)) : 0;
    if (lane == 0) scale[row] = ldexpf(1.f, e);
  } else if (compute == IPFP_F32) {
    float* o = static_cast<float*>(out) + row * kpad;
    for (int64_t k = lane; k < kpad; k += 64) o[k] = k < k2 ? val(k) : 0.f;
  } else {
    uint16_t* o = static_cast<uint16_t*>(out) + row * kpad;
    for (int64_t k = lane; k < kpad; k += 64)
      o[k] = k < k2 ? bf16_rne(val(k)) : 0;
  }
}

hipError_t launch_pack(const void* A, const void* B, ipfp_dtype in_dt,
                       const float* in_scale, int64_t ld, int64_t rows, int64_t d,
                       ipfp_dtype compute, int64_t kpad, float prescale, void* out,
                       float* scale, Ctl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, A,
                     B, in_dt, in_scale, ld, rows, d, compute, kpad, prescale, out, scale,
                     ctl);
  return hipGetLastError();
}

// ---- the reduction pass ------------------------------------------------------

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Operand kinds of the fused passes.
enum OpKind { kBF16 = 0, kFP8 = 1, kF32 = 2 };

// Operand traits: bytes per element (ES), bytes a lane reads per k-step (SB),
// the K extent of one k-step (KS) and the lane's fragment of a k-step. A
// k-step is one MFMA for BF16 and FP8 and four for FP32 (a lane's 16 bytes
// are four consecutive K slots, fed one per 32x32x2 MFMA): both operands read
// the same packed positions in the same order, so any assignment of K slots
// to lanes and steps sums the same products.
template <int OK>
struct Op;
template <>
struct Op<kBF16> {  // BF16, v_mfma_f32_32x32x16_bf16
  static constexpr int ES = 2, SB = 16, KS = 16;
  typedef bf16x8 Frag;
};
template <>
struct Op<kFP8> {  // FP8 e4m3, v_mfma_scale_f32_32x32x64_f8f6f4
  static constexpr int ES = 1, SB = 32, KS = 64;
  typedef intx8 Frag;
};
template <>
struct Op<kF32> {  // FP32, four v_mfma_f32_32x32x2_f32 per k-step
  static constexpr int ES = 4, SB = 16, KS = 8;
  typedef floatx4 Frag;
};

// Reduced rows staged per LDS buffer (a multiple of 64): IPFP_TY (a build-time
// knob) for packed rows up to 256 bytes, half of it for longer rows so that
// the double buffer stays near 70 KiB of LDS (FP32 rows of 2d > 128: 130 KiB).
#ifndef IPFP_TY
#define IPFP_TY 128
#endif

// Upper bound on waves per SIMD the compiler schedules the reduction pass for.
// BF16 rows of 2d >= 192 fit three waves per SIMD when scheduled for it, but
// an 8-wave workgroup uses only two of them, and the kernel compiled for two
// (more registers per wave) is 15-60 % faster there (MI355X, N = M = 1e6);
// elsewhere the default scheduling is as fast or faster. FP32 passes keep
// the whole register file (their operand fragments are twice the BF16 ones):
// one wave per SIMD, four-wave workgroups.
constexpr int pass_max_waves(int kp, int ok) {
  return ok == kF32 ? 1 : ((ok == kBF16 && kp >= 192) ? 2 : 8);
}
constexpr int pass_min_waves(int ok) { return ok == kF32 ? 1 : 2; }

constexpr int ty_for(int row_bytes) { return row_bytes <= 256 ? IPFP_TY : IPFP_TY / 2; }

// Register budget: two 32-row output tiles per wave while the operand
// fragments of both fit in 64 VGPRs per lane (one tile for FP32): BF16 rows
// up to 2d = 128, FP8 rows up to 2d = 256. Two tiles per wave halve the LDS
// fragment reads per MFMA; with one tile the fragment reads of a compute
// unit's four SIMDs alone take the LDS bandwidth (MI355X: C5 FP8, kpad 256,
// 91.7 ms per pass with one tile, 81.5 ms with two).
constexpr int xt_for(int kp, int ok) {
  return ok == kF32 ? 1 : ((ok == kFP8 ? kp <= 256 : (kp <= 128 && kp != 96)) ? 2 : 1);
}

static int op_kind(ipfp_dtype compute) {
  return compute == IPFP_FP8E4M3 ? kFP8 : (compute == IPFP_F32 ? kF32 : kBF16);
}

// Waves per workgroup of a sum or max pass: 8 when the requested height
// covers them, else 4; FP32 passes always use 4 (one wave per SIMD).
static int pass_waves(int ok, int xt, int tile_rows) {
  return ok != kF32 && tile_rows >= xt * 256 ? 8 : 4;
}

static int elem_bytes(int ok) { return ok == kFP8 ? 1 : (ok == kF32 ? 4 : 2); }

// The kpads every operand kind is built for (BF16 and FP32 rows are padded to
// multiples of 32 values, FP8 rows to multiples of 64).
#define IPFP_KP16(X, OKV) X(32, OKV) X(64, OKV) X(96, OKV) X(128, OKV) X(160, OKV) \
  X(192, OKV) X(224, OKV) X(256, OKV)
#define IPFP_KP8(X, OKV) X(64, OKV) X(128, OKV) X(192, OKV) X(256, OKV)

// Binary exponent e with w = m 2^e, m in [0.5, 1) (INT_MIN for w = 0).
__device__ __forceinline__ int exponent_of(double w) {
  if (!(w > 0.0)) return INT_MIN;
  int e;
  frexp(w, &e);
  return e;
}

// Everything a reduction pass keeps per wave, plus the staging of the reduced
// side through LDS; shared by the max pass and the sum pass.
template <int KP, int XT, int WAVES, int OK>
struct PassCore {
  typedef Op<OK> O;
  static constexpr int RB = KP * O::ES;           // bytes per packed row
  static constexpr int kTY = ty_for(RB);          // reduced rows per stage
  static constexpr int NS = KP / O::KS;           // k-steps per 32x32 tile
  static constexpr int LS = RB + 16;              // LDS row stride (pad)
  static constexpr int NT = WAVES * 64;
  static constexpr int CH = kTY * RB / 16;        // 16-byte chunks per stage
  static constexpr int CPT = (CH + NT - 1) / NT;  // chunks per thread
  static constexpr int SUB = kTY / 32;
  typedef typename O::Frag Frag;
};

// Reads the fragment of k-step s for the packed row at `arow` (which already
// points at the lane's half: + h * SB).
template <int OK>
__device__ __forceinline__ typename Op<OK>::Frag lds_frag(const uint8_t* arow, int s) {
  typedef Op<OK> O;
  typename O::Frag f;
  if constexpr (OK == kFP8) {
    intx4 lo = *reinterpret_cast<const intx4*>(arow + s * 2 * O::SB);
    intx4 hi = *reinterpret_cast<const intx4*>(arow + s * 2 * O::SB + 16);
    intx8 v;
    v[0] = lo[0]; v[1] = lo[1]; v[2] = lo[2]; v[3] = lo[3];
    v[4] = hi[0]; v[5] = hi[1]; v[6] = hi[2]; v[7] = hi[3];
    *reinterpret_cast<intx8*>(&f) = v;
  } else {
    *reinterpret_cast<intx4*>(&f) = *reinterpret_cast<const intx4*>(arow + s * 2 * O::SB);
  }
  return f;
}

template <int OK>
__device__ __forceinline__ floatx16 mfma_step(const typename Op<OK>::Frag& a,
                                              const typename Op<OK>::Frag& b, floatx16 c,
                                              int asc, int bsc) {
  if constexpr (OK == kFP8) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
        *reinterpret_cast<const intx8*>(&a), *reinterpret_cast<const intx8*>(&b), c, 0, 0,
        0, asc, 0, bsc);
  } else if constexpr (OK == kF32) {
#pragma unroll
    for (int j = 0; j < 4; ++j) c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j], b[j], c, 0, 0, 0);
    return c;
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
}

// Two independent accumulator chains advanced by one k-step each. For FP32
// the chains' four MFMAs alternate, so no MFMA waits on the one before it.
template <int OK>
__device__ __forceinline__ void mfma_pair(const typename Op<OK>::Frag& a0,
                                          const typename Op<OK>::Frag& b0, floatx16& c0,
                                          int asc0, int bsc0,
                                          const typename Op<OK>::Frag& a1,
                                          const typename Op<OK>::Frag& b1, floatx16& c1,
                                          int asc1, int bsc1) {
  if constexpr (OK == kF32) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[j], b0[j], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[j], b1[j], c1, 0, 0, 0);
    }
  } else {
    c0 = mfma_step<OK>(a0, b0, c0, asc0, bsc0);
    c1 = mfma_step<OK>(a1, b1, c1, asc1, bsc1);
  }
}

// Work item of block `bid` in a list of W items ordered split-major (all row
// blocks of split 0, then split 1, ...). Workgroups are dispatched to the 8
// XCDs round robin (bid % 8); each XCD takes a contiguous run of the list, so
// the workgroups it holds at once mostly share a split and stream the same
// reduced tiles through its own L2. A bijection of [0, W) for every W.
__device__ __forceinline__ int xcd_item(int bid, int W) {
  const int per = (W + 7) / 8, rem = W - 8 * (per - 1);   // XCDs g < rem take per
  const int g = bid & 7, i = bid >> 3;
  return g <= rem ? g * per + i : rem * per + (g - rem) * (per - 1) + i;
}

// The reduction pass. MAXMODE: per (split, row) maximum of T over the split
// (set-up). Otherwise the weighted sum S described at the top of this file.
//
// Where the MFMAs dominate a step (FP8 operands, BF16 with 2d = 128 or
// 2d >= 192) sum mode runs two independent accumulators ("chains") at a time
// -- the two output tiles of a wave (XT = 2) or two consecutive reduced
// subtiles (XT = 1) -- so consecutive MFMAs never wait on each other, and the
// exp2/FMA epilogue of the previous pair is spread between this pair's MFMAs:
// the matrix cores and the transcendental/FMA pipe then work at the same time.
// Elsewhere it finishes one accumulator (MFMAs, then its epilogue) before the
// next.
//
// `bid` is the workgroup's index within this market's grid (blockIdx.x for a
// single-market launch, the offset within the market's range of a grouped
// launch).
template <int KP, int XT, int WAVES, int OK, bool MAXMODE>
__device__ __forceinline__ void fused_pass_body(
    const uint8_t* __restrict__ Xo, const float* __restrict__ xscale,
    const uint8_t* __restrict__ Yr, const float* __restrict__ yscale,
    const double* __restrict__ wred, int red_dbuf, int exp_red, int exp_out,
    const float* __restrict__ shift, int R, int L, int tiles_per_split, int nsplit,
    double* __restrict__ part, Ctl* ctl, const int bid) {
  typedef PassCore<KP, XT, WAVES, OK> C;
  typedef typename C::Frag Frag;
  typedef Op<OK> O;
  constexpr bool FP8 = OK == kFP8;
  constexpr int RB = C::RB, kTY = C::kTY, NS = C::NS, LS = C::LS, NT = C::NT;
  constexpr int CH = C::CH, CPT = C::CPT, SUB = C::SUB;

  __shared__ __attribute__((aligned(16))) uint8_t ys[2][kTY * LS];
  // weights are triple-buffered: the pending epilogue reads a tile's weights
  // during the following tile, while other waves may already be staging the
  // tile after that
  __shared__ __attribute__((aligned(16))) float ws[3][kTY];
  __shared__ __attribute__((aligned(16))) float wzero[32];
  __shared__ int32_t ysc[2][kTY];          // FP8: E8M0 scale byte per row

  if (ctl->done) return;
  if (!MAXMODE && bid == 0 && threadIdx.x == 0)
    ctl->wexp[exp_out] = INT_MIN;          // the combine of this pass sets it
  int E = MAXMODE ? 0 : ctl->wexp[exp_red];
  if (E == INT_MIN) E = 0;
  // a double-buffered reduced side (u) holds the current state in the half
  // selected by the sweep counter
  if (red_dbuf) wred += (int64_t)(ctl->sweep & 1) * L;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int rblocks = (R + WAVES * XT * 32 - 1) / (WAVES * XT * 32);
  const int item = xcd_item(bid, rblocks * nsplit);
  const int split = item / rblocks;
  const int rb = item - split * rblocks;
  const int T = (L + kTY - 1) / kTY;
  const int t0 = split * tiles_per_split;
  const int t1 = min(T, t0 + tiles_per_split);
  const int row_base = (rb * WAVES + wave) * (XT * 32);
  if (tid < 32) wzero[tid] = 0.f;

  // output-side operand fragments, shift accumulators and scales (registers)
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
      Frag f = lds_frag<OK>(src, s);   // same layout as a staged row
      if (!ok) *reinterpret_cast<intx4*>(&f) = intx4{0, 0, 0, 0};
      if constexpr (FP8) {
        if (!ok) reinterpret_cast<intx4*>(&f)[1] = intx4{0, 0, 0, 0};
      }
      bfrag[t][s] = f;
    }
    const float hv = (!MAXMODE && ok) ? shift[x] : 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) shv[t][r] = hv;
    xsc[t] = FP8 && ok ? (int)((__float_as_uint(xscale[x]) >> 23) & 0xFF) : 127;
  }

  double run[XT];
  float mx[XT];
#pragma unroll
  for (int t = 0; t < XT; ++t) {
    run[t] = 0.0;
    mx[t] = -INFINITY;
  }

  // stage loader: global -> registers -> LDS. Branch-free: rows past the end
  // are clamped to the last row (a valid read) and get weight 0 (the max pass
  // only ever sees duplicates of real rows); surplus threads repeat the last
  // chunk, and every thread loads the weight of row tid % kTY (duplicates
  // store identical values).
  intx4 pre[CPT];
  float pw = 0.f;
  int psc = 127;
  // Row arithmetic is 32-bit (L < 2^31): one 32x32->64 multiply-add per load.
  auto gload = [&](int tile) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int chunk = min(tid + q * NT, CH - 1);
      const int r = chunk / (RB / 16), cb = chunk % (RB / 16);
      const uint32_t y = (uint32_t)min(tile * kTY + r, L - 1);
      pre[q] = *reinterpret_cast<const intx4*>(Yr + cb * 16 + (uint64_t)y * RB);
    }
    const int y = tile * kTY + (tid % kTY);
    const int yc = min(y, L - 1);
    if (!MAXMODE) {
      const float wv = (float)ldexp(wred[yc], -E);
      pw = y < L ? wv : 0.f;
    }
    if (FP8) psc = (int)((__float_as_uint(yscale[yc]) >> 23) & 0xFF);
  };
  auto lstore = [&](int buf, int wbuf) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int chunk = min(tid + q * NT, CH - 1);
      const int r = chunk / (RB / 16), cb = chunk % (RB / 16);
      *reinterpret_cast<intx4*>(&ys[buf][r * LS + cb * 16]) = pre[q];
    }
    if (!MAXMODE) ws[wbuf][tid % kTY] = pw;
    if (FP8) ysc[buf][tid % kTY] = psc;
  };

  // sum mode: the pending pair of accumulators, their weights (LDS; a buffer
  // is overwritten only after the following tile, so they are still there)
  // and their running-sum slots; a zero-weight dummy before the first tile
  constexpr int NPAIR = XT == 2 ? SUB : SUB / 2;
  // the paired, pipelined schedule pays off where the MFMAs dominate a step
  // (FP8 and FP32 operands, BF16 with 2d = 128 or 2d >= 192); elsewhere one
  // chain at a time
  constexpr bool kPaired = OK != kBF16 || KP == 128 || KP >= 192;
  // BF16 with 2d = 128: explicit scheduling groups (below) interleave each
  // MFMA with its share of the pending epilogue
  constexpr bool kGrouped = OK == kBF16 && KP == 128;
  floatx16 pc0, pc1;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    pc0[r] = 0.f;
    pc1[r] = 0.f;
  }
  const float* pw0 = &wzero[4 * h];
  const float* pw1 = pw0;
  // exp2/FMA of pending entry r of both chains into four partial sums
  auto epi1 = [&](const int r, const float* w0, const float* w1, float* s4) {
    const float e0 = __builtin_amdgcn_exp2f(pc0[r]);
    const float e1 = __builtin_amdgcn_exp2f(pc1[r]);
    s4[r & 1] = fmaf(e0, w0[r], s4[r & 1]);
    s4[2 + (r & 1)] = fmaf(e1, w1[r], s4[2 + (r & 1)]);
  };
  constexpr int PER = (16 + NS - 1) / NS;   // pending entries per k-step
  auto load_w = [&](const float* p, float* w) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const floatx4 w4 = *reinterpret_cast<const floatx4*>(p + 8 * g);
      w[4 * g + 0] = w4[0];
      w[4 * g + 1] = w4[1];
      w[4 * g + 2] = w4[2];
      w[4 * g + 3] = w4[3];
    }
  };
  auto flush = [&](const float* s4) {
    // the pending pair's tiles: (t = 0, 1) for XT = 2, both tile 0 for XT = 1
    run[0] += (double)(s4[0] + s4[1]);
    run[XT - 1] += (double)(s4[2] + s4[3]);
  };

  if (t0 < t1) {
    gload(t0);
    lstore(0, 0);
  }
  __syncthreads();

  int wbuf = 0;
  for (int tile = t0; tile < t1; ++tile) {
    const int buf = (tile - t0) & 1;
    const int wnext = wbuf == 2 ? 0 : wbuf + 1;
    gload(min(tile + 1, t1 - 1));   // prefetch (the last iteration reloads harmlessly)
    // the next stage's global loads go out before any of this stage's work
    if constexpr (!MAXMODE && kGrouped) __builtin_amdgcn_sched_barrier(0);
    if constexpr (MAXMODE) {
      // the XT accumulators of MS subtiles advance together: independent
      // MFMA chains, interleaved k-step by k-step. Two subtiles for BF16
      // (MI355X, N = M = 1e6: 2d = 128 189 -> 182 ms, 2d = 64 99 -> 97 ms
      // per pass), one otherwise (with FP8 rows of 2d = 256 two would spill)
      constexpr int MS = OK == kBF16 && SUB % 2 == 0 ? 2 : 1;
#pragma unroll
      for (int sub = 0; sub < SUB; sub += MS) {
        const uint8_t* arow[MS];
        int asc[MS];
        floatx16 acc[MS][XT];
#pragma unroll
        for (int u = 0; u < MS; ++u) {
          arow[u] = &ys[buf][((sub + u) * 32 + l32) * LS + h * O::SB];
          asc[u] = FP8 ? ysc[buf][(sub + u) * 32 + l32] : 127;
#pragma unroll
          for (int t = 0; t < XT; ++t) acc[u][t] = shv[t];
        }
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int u = 0; u < MS; ++u) {
            const Frag f = lds_frag<OK>(arow[u], s);
#pragma unroll
            for (int t = 0; t < XT; ++t)
              acc[u][t] = mfma_step<OK>(f, bfrag[t][s], acc[u][t], asc[u], xsc[t]);
          }
#pragma unroll
        for (int u = 0; u < MS; ++u)
#pragma unroll
          for (int t = 0; t < XT; ++t) {
            float m0 = fmaxf(acc[u][t][0], acc[u][t][1]), m1 = fmaxf(acc[u][t][2], acc[u][t][3]);
#pragma unroll
            for (int r = 4; r < 16; r += 2) {
              m0 = fmaxf(m0, acc[u][t][r]);
              m1 = fmaxf(m1, acc[u][t][r + 1]);
            }
            mx[t] = fmaxf(mx[t], fmaxf(m0, m1));
          }
      }
    } else if constexpr (!kPaired && KP == 64) {
      // two accumulators at a time (the wave's two output tiles, or two
      // consecutive subtiles of its one tile), their MFMA chains interleaved
      // k-step by k-step so that consecutive MFMAs are independent; then
      // each one's epilogue, in tile and subtile order (the same sums bit
      // for bit as one accumulator at a time). MI355X, N = M = 1e6, BF16:
      // 2d = 64 1.4 % faster per sweep, with fewer registers. 2d = 32 is
      // unchanged and 2d = 160 0.3 % slower (one wave fewer per SIMD); at
      // 2d = 96 the single-market pass gains 1.3 % but the grouped one
      // would drop from four waves per SIMD to two: those keep the schedule
      // below.
      auto epi_seq = [&](const floatx16& acc, const float* w) {
        float s0 = __builtin_amdgcn_exp2f(acc[0]) * w[0];
        float s1 = __builtin_amdgcn_exp2f(acc[1]) * w[1];
#pragma unroll
        for (int r = 2; r < 16; r += 2) {
          s0 = fmaf(__builtin_amdgcn_exp2f(acc[r]), w[r], s0);
          s1 = fmaf(__builtin_amdgcn_exp2f(acc[r + 1]), w[r + 1], s1);
        }
        return (double)(s0 + s1);
      };
#pragma unroll
      for (int q = 0; q < NPAIR; ++q) {
        const int sub0 = XT == 2 ? q : 2 * q, sub1 = XT == 2 ? q : 2 * q + 1;
        constexpr int ta = 0, tb = XT - 1;
        const uint8_t* arow0 = &ys[buf][(sub0 * 32 + l32) * LS + h * O::SB];
        const uint8_t* arow1 = &ys[buf][(sub1 * 32 + l32) * LS + h * O::SB];
        const int asc0 = FP8 ? ysc[buf][sub0 * 32 + l32] : 127;
        const int asc1 = FP8 ? ysc[buf][sub1 * 32 + l32] : 127;
        floatx16 a0 = shv[ta], a1 = shv[tb];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const Frag f0 = lds_frag<OK>(arow0, s);
          const Frag f1 = XT == 2 ? f0 : lds_frag<OK>(arow1, s);
          mfma_pair<OK>(f0, bfrag[ta][s], a0, asc0, xsc[ta], f1, bfrag[tb][s], a1, asc1,
                        xsc[tb]);
        }
        float w0[16];
        load_w(&ws[wbuf][sub0 * 32 + 4 * h], w0);
        run[ta] += epi_seq(a0, w0);
        if constexpr (XT == 2) {
          run[tb] += epi_seq(a1, w0);
        } else {
          float w1[16];
          load_w(&ws[wbuf][sub1 * 32 + 4 * h], w1);
          run[tb] += epi_seq(a1, w1);
        }
      }
    } else if constexpr (!kPaired) {
      // one accumulator at a time, its epilogue right after its MFMAs
#pragma unroll
      for (int sub = 0; sub < SUB; ++sub) {
        const uint8_t* arow = &ys[buf][(sub * 32 + l32) * LS + h * O::SB];
        const int asc = FP8 ? ysc[buf][sub * 32 + l32] : 127;
        float w[16];
        load_w(&ws[wbuf][sub * 32 + 4 * h], w);
#pragma unroll
        for (int t = 0; t < XT; ++t) {
          floatx16 acc = shv[t];
#pragma unroll
          for (int s = 0; s < NS; ++s)
            acc = mfma_step<OK>(lds_frag<OK>(arow, s), bfrag[t][s], acc, asc, xsc[t]);
          float s0 = __builtin_amdgcn_exp2f(acc[0]) * w[0];
          float s1 = __builtin_amdgcn_exp2f(acc[1]) * w[1];
#pragma unroll
          for (int r = 2; r < 16; r += 2) {
            s0 = fmaf(__builtin_amdgcn_exp2f(acc[r]), w[r], s0);
            s1 = fmaf(__builtin_amdgcn_exp2f(acc[r + 1]), w[r + 1], s1);
          }
          run[t] += (double)(s0 + s1);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < NPAIR; ++q) {
        const int sub0 = XT == 2 ? q : 2 * q, sub1 = XT == 2 ? q : 2 * q + 1;
        constexpr int ta = 0, tb = XT - 1;
        const uint8_t* arow0 = &ys[buf][(sub0 * 32 + l32) * LS + h * O::SB];
        const uint8_t* arow1 = &ys[buf][(sub1 * 32 + l32) * LS + h * O::SB];
        const int asc0 = FP8 ? ysc[buf][sub0 * 32 + l32] : 127;
        const int asc1 = FP8 ? ysc[buf][sub1 * 32 + l32] : 127;
        float w0[16], w1[16];
        load_w(pw0, w0);
        if constexpr (XT == 2) {
#pragma unroll
          for (int r = 0; r < 16; ++r) w1[r] = w0[r];
        } else {
          load_w(pw1, w1);
        }
        float s4[4] = {0.f, 0.f, 0.f, 0.f};
        floatx16 a0 = shv[ta], a1 = shv[tb];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const Frag f0 = lds_frag<OK>(arow0, s);
          const Frag f1 = XT == 2 ? f0 : lds_frag<OK>(arow1, s);
          mfma_pair<OK>(f0, bfrag[ta][s], a0, asc0, xsc[ta], f1, bfrag[tb][s], a1, asc1,
                        xsc[tb]);
#pragma unroll
          for (int u = 0; u < PER; ++u)
            if (s * PER + u < 16) epi1(s * PER + u, w0, w1, s4);
        }
        flush(s4);
        if constexpr (kGrouped) {
          // scheduling groups (masks: 0x008 MFMA, 0x400 transcendental,
          // 0x002 other VALU, 0x100 LDS read): the weight reads and two
          // k-steps of fragment reads first, then each MFMA followed by its
          // share of the pending epilogue (PER exp2, PER FMAs) and the next
          // fragment read. Without them the compiler clusters the epilogue
          // after the first MFMAs and leaves the rest back to back.
          __builtin_amdgcn_sched_group_barrier(0x100, 4 + 2, 0);
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x400, PER, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, PER, 0);
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x400, PER, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, PER, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        pc0 = a0;
        pc1 = a1;
        pw0 = &ws[wbuf][sub0 * 32 + 4 * h];
        pw1 = &ws[wbuf][sub1 * 32 + 4 * h];
      }
    }
    lstore(buf ^ 1, wnext);
    wbuf = wnext;
    __syncthreads();
  }
  if constexpr (!MAXMODE && kPaired) {
    float w0[16], w1[16];
    load_w(pw0, w0);
    load_w(pw1, w1);
    float s4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 16; ++r) epi1(r, w0, w1, s4);
    flush(s4);
  }

#pragma unroll
  for (int t = 0; t < XT; ++t) {
    const int x = row_base + t * 32 + l32;
    double tot;
    if (MAXMODE) {
      const float o = __shfl_xor(mx[t], 32, 64);
      tot = (double)fmaxf(mx[t], o);
    } else {
      tot = run[t] + __shfl_xor(run[t], 32, 64);
    }
    if (h == 0 && x < R) part[(int64_t)split * R + x] = tot;
  }
}

template <int KP, int XT, int WAVES, int OK, bool MAXMODE>
__global__ void __launch_bounds__(WAVES * 64)
    __attribute__((amdgpu_waves_per_eu(pass_min_waves(OK), pass_max_waves(KP, OK))))
    k_fused_pass(const uint8_t* __restrict__ Xo, const float* __restrict__ xscale,
                 const uint8_t* __restrict__ Yr, const float* __restrict__ yscale,
                 const double* __restrict__ wred, int red_dbuf, int exp_red,
                 int exp_out, const float* __restrict__ shift, int R, int L,
                 int tiles_per_split, int nsplit, double* __restrict__ part,
                 Ctl* ctl) {
  fused_pass_body<KP, XT, WAVES, OK, MAXMODE>(Xo, xscale, Yr, yscale, wred, red_dbuf,
                                               exp_red, exp_out, shift, R, L,
                                               tiles_per_split, nsplit, part, ctl,
                                               (int)blockIdx.x);
}

// Grouped launch: the grid is the concatenation of several markets' grids;
// market idx[j] owns blocks [first[j], first[j + 1]).
__device__ __forceinline__ int group_find(const int32_t* __restrict__ first, int count,
                                          int b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (__builtin_amdgcn_readfirstlane(first[mid]) <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int KP, int XT, int WAVES, int OK>
__global__ void __launch_bounds__(WAVES * 64)
    __attribute__((amdgpu_waves_per_eu(pass_min_waves(OK), pass_max_waves(KP, OK))))
    k_group_pass(const GroupHalf* __restrict__ g, const int32_t* __restrict__ idx,
                 const int32_t* __restrict__ first, int count) {
  const int j = group_find(first, count, (int)blockIdx.x);
  const GroupHalf& p = g[__builtin_amdgcn_readfirstlane(idx[j])];
  fused_pass_body<KP, XT, WAVES, OK, false>(
      p.Xo, p.xscale, p.Yr, p.yscale, p.wred, p.red_dbuf, p.exp_red, p.exp_out, p.shift,
      p.R, p.L, p.tiles_per_split, p.nsplit, p.part, p.ctl,
      (int)blockIdx.x - __builtin_amdgcn_readfirstlane(first[j]));
}

// ---- recommendation lists: top-k per output row -------------------------------
//
// After the solve, mu_or = 2^(T_or) a_o w_r (eq. 4 with K in log2 units), so
// for a fixed output row o the reduced rows ranked by mu are ranked by the
// score T_or + log2 w_r. This pass forms T on the matrix cores exactly as the
// reduction pass does and keeps, per lane, the KT best (score, row) pairs in
// registers, sorted descending (ties keep the earlier row of the lane's
// stream). The two lanes that share an output row merge at the end; one
// partial list per (split, row) goes to memory and k_topk_merge combines the
// splits in fixed order.

// Inserts (s, i) into the descending list (ts, ti), dropping its last entry.
template <int KT>
__device__ __forceinline__ void topk_insert(float (&ts)[KT], int (&ti)[KT], float s, int i) {
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    const bool sw = s > ts[j];
    const float t = ts[j];
    const int u = ti[j];
    ts[j] = sw ? s : t;
    ti[j] = sw ? i : u;
    s = sw ? t : s;
    i = sw ? u : i;
  }
}

// Subtiles whose score chains a top-k pass interleaves (consecutive MFMAs
// then never wait on each other): two for BF16 rows of 2d = 96 and 128 with
// lists of up to 16, which still fit the two waves per SIMD that one chain
// ran at; else one. MI355X, N = M = 1e6, k = 10, one chain -> two (with the
// weights in the chains): BF16 2d = 128 319 -> 300 ms, 2d = 96 271 -> 256
// ms, 2d = 64 187 -> 214 ms; FP8 2d = 128 and 192 3 % slower (their MFMA
// is half as long, and the check work dominates).
template <int KP, int OK, int KT>
constexpr int topk_tp() {
  return PassCore<KP, 1, 4, OK>::SUB >= 4 && OK == kBF16 && KP >= 96 && KT <= 16 ? 2 : 1;
}

template <int KP, int OK, int KT>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(topk_tp<KP, OK, KT>(), topk_tp<KP, OK, KT>() == 2 ? 2 : 8)))
    k_topk_pass(const uint8_t* __restrict__ Xo, const float* __restrict__ xscale,
                const uint8_t* __restrict__ Yr, const float* __restrict__ yscale,
                const double* __restrict__ wred, int R, int L, int tiles_per_split,
                int nsplit, float* __restrict__ pscore, int32_t* __restrict__ pidx) {
  constexpr int WAVES = 4;
  typedef PassCore<KP, 1, WAVES, OK> C;
  typedef typename C::Frag Frag;
  typedef Op<OK> O;
  constexpr bool FP8 = OK == kFP8;
  constexpr int RB = C::RB, kTY = C::kTY, NS = C::NS, LS = C::LS, NT = C::NT;
  constexpr int CH = C::CH, CPT = C::CPT, SUB = C::SUB;
  __shared__ __attribute__((aligned(16))) uint8_t ys[2][kTY * LS];
  __shared__ __attribute__((aligned(16))) float lws[2][kTY];
  __shared__ int32_t ysc[2][kTY];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int rblocks = (R + WAVES * 32 - 1) / (WAVES * 32);
  const int item = xcd_item(blockIdx.x, rblocks * nsplit);
  const int split = item / rblocks, rb = item - split * rblocks;
  const int T = (L + kTY - 1) / kTY;
  const int t0 = split * tiles_per_split, t1 = min(T, t0 + tiles_per_split);
  const int x = (rb * WAVES + wave) * 32 + l32;
  const bool ok = x < R;

  Frag bfrag[NS];
  {
    const uint8_t* src = Xo + (int64_t)(ok ? x : 0) * RB + h * O::SB;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Frag f = lds_frag<OK>(src, s);
      if (!ok) *reinterpret_cast<intx4*>(&f) = intx4{0, 0, 0, 0};
      if constexpr (FP8) {
        if (!ok) reinterpret_cast<intx4*>(&f)[1] = intx4{0, 0, 0, 0};
      }
      bfrag[s] = f;
    }
  }
  const int xsc = FP8 && ok ? (int)((__float_as_uint(xscale[x]) >> 23) & 0xFF) : 127;

  float ts[KT];
  int ti[KT];
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    ts[j] = -INFINITY;
    ti[j] = -1;
  }

  // stage loader (as in the reduction pass): rows past the end are clamped and
  // get score -inf through lw
  intx4 pre[CPT];
  float plw = -INFINITY;
  int psc = 127;
  auto gload = [&](int tile) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int chunk = min(tid + q * NT, CH - 1);
      const int r = chunk / (RB / 16), cb = chunk % (RB / 16);
      const uint32_t y = (uint32_t)min(tile * kTY + r, L - 1);
      pre[q] = *reinterpret_cast<const intx4*>(Yr + cb * 16 + (uint64_t)y * RB);
    }
    const int y = tile * kTY + (tid % kTY);
    const int yc = min(y, L - 1);
    plw = y < L ? (float)log2(wred[yc]) : -INFINITY;
    if (FP8) psc = (int)((__float_as_uint(yscale[yc]) >> 23) & 0xFF);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int chunk = min(tid + q * NT, CH - 1);
      const int r = chunk / (RB / 16), cb = chunk % (RB / 16);
      *reinterpret_cast<intx4*>(&ys[buf][r * LS + cb * 16]) = pre[q];
    }
    lws[buf][tid % kTY] = plw;
    if (FP8) ysc[buf][tid % kTY] = psc;
  };

  if (t0 < t1) {
    gload(t0);
    lstore(0);
  }
  __syncthreads();
  // T of TP subtiles (MFMA chains over the packed rows), interleaved k-step
  // by k-step so that consecutive MFMAs are independent
  constexpr int TP = topk_tp<KP, OK, KT>();
  // BF16 and FP32 chains start from the reduced rows' log2 weights, so the
  // score comes out of the MFMAs (their FP32 sums keep it well inside the
  // lists' tolerance); the FP8 MFMA adds its inputs at reduced precision, so
  // there the weights are added after the chain
  constexpr bool kLwIn = OK != kFP8;
  auto tgrp = [&](int buf, int sub, floatx16 (&out)[TP]) {
    int asc[TP];
#pragma unroll
    for (int u = 0; u < TP; ++u) {
      asc[u] = FP8 ? ysc[buf][(sub + u) * 32 + l32] : 127;
      if constexpr (kLwIn) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const floatx4 w4 =
              *reinterpret_cast<const floatx4*>(&lws[buf][(sub + u) * 32 + 8 * g + 4 * h]);
#pragma unroll
          for (int e = 0; e < 4; ++e) out[u][4 * g + e] = w4[e];
        }
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) out[u][r] = 0.f;
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int u = 0; u < TP; ++u) {
        const uint8_t* arow = &ys[buf][((sub + u) * 32 + l32) * LS + h * O::SB];
        out[u] = mfma_step<OK>(lds_frag<OK>(arow, s), bfrag[s], out[u], asc[u], xsc);
      }
  };
  for (int tile = t0; tile < t1; ++tile) {
    const int buf = (tile - t0) & 1;
    gload(min(tile + 1, t1 - 1));
    // the next group's MFMA chains are issued before this group's scores are
    // checked, and the common case (no score above any lane's k-th best)
    // takes a single branch per subtile, so the chains run under the checks
    floatx16 nxt[TP], cur[TP];
    tgrp(buf, 0, nxt);
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub) {
      if (sub % TP == 0) {
#pragma unroll
        for (int u = 0; u < TP; ++u) cur[u] = nxt[u];
        if (sub + TP < SUB) tgrp(buf, sub + TP, nxt);
      }
      const floatx16 acc = cur[sub % TP];
      float sc[16];
      float top = -INFINITY;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int yr = sub * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        sc[r] = kLwIn ? acc[r] : acc[r] + lws[buf][yr];
        top = fmaxf(top, sc[r]);
      }
      if (top > ts[KT - 1]) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int yr = sub * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
          if (sc[r] > ts[KT - 1]) topk_insert<KT>(ts, ti, sc[r], tile * kTY + yr);
        }
      }
    }
    lstore(buf ^ 1);
    __syncthreads();
  }
  // lanes l and l + 32 hold the same output row: merge into the lower one
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    const float s = __shfl_xor(ts[j], 32, 64);
    const int i = __shfl_xor(ti[j], 32, 64);
    if (h == 0 && s > ts[KT - 1]) topk_insert<KT>(ts, ti, s, i);
  }
  if (h == 0 && ok) {
    const int64_t base = ((int64_t)split * R + x) * KT;
#pragma unroll
    for (int j = 0; j < KT; ++j) {
      pscore[base + j] = ts[j];
      pidx[base + j] = ti[j];
    }
  }
}

// Merges the split lists of every row (fixed split order) and writes the k
// best as (row index, log mu): log mu_or = ln 2 (score + log2 a_o).
template <int KT>
__global__ void __launch_bounds__(256)
    k_topk_merge(const float* __restrict__ pscore, const int32_t* __restrict__ pidx,
                 int nsplit, int R, const double* __restrict__ a_out, int k,
                 int32_t* __restrict__ idx_out, float* __restrict__ score_out) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= R) return;
  float ts[KT];
  int ti[KT];
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    ts[j] = -INFINITY;
    ti[j] = -1;
  }
  for (int sp = 0; sp < nsplit; ++sp) {
    const int64_t base = ((int64_t)sp * R + o) * KT;
    for (int j = 0; j < KT; ++j) {
      const float s = pscore[base + j];
      if (!(s > ts[KT - 1])) break;   // lists are sorted: the rest is smaller
      topk_insert<KT>(ts, ti, s, pidx[base + j]);
    }
  }
  const double la = log2(a_out[o]);
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    if (j < k) {
      idx_out[(int64_t)o * k + j] = ti[j];
      score_out[(int64_t)o * k + j] =
          ti[j] >= 0 ? (float)(((double)ts[j] + la) * 0.6931471805599453) : -INFINITY;
    }
  }
}

template <int KP, int OK, int KT>
static hipError_t topk_t(const FusedPass& fp, const double* a_out, int k, int splits,
                         float* pscore, int32_t* pidx, int32_t* idx_out, float* score_out,
                         hipStream_t s) {
  constexpr int kTY = ty_for(KP * Op<OK>::ES);
  const int64_t rblocks = (fp.out.rows + 127) / 128;
  const int T = (int)((fp.red.rows + kTY - 1) / kTY);
  const int tps = (T + splits - 1) / splits;
  hipLaunchKernelGGL((k_topk_pass<KP, OK, KT>), dim3((unsigned)(rblocks * splits)),
                     dim3(256), 0, s, (const uint8_t*)fp.out.ops, fp.out.scale,
                     (const uint8_t*)fp.red.ops, fp.red.scale, fp.w_red, (int)fp.out.rows,
                     (int)fp.red.rows, tps, splits, pscore, pidx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_topk_merge<KT>), dim3((unsigned)((fp.out.rows + 255) / 256)),
                     dim3(256), 0, s, pscore, pidx, splits, (int)fp.out.rows, a_out, k,
                     idx_out, score_out);
  return hipGetLastError();
}

template <int KP, int OK>
static hipError_t topk_kp(const FusedPass& fp, const double* a_out, int k, int splits,
                          float* pscore, int32_t* pidx, int32_t* idx_out, float* score_out,
                          hipStream_t s) {
  const int kt = topk_width(k);
  if (kt == 8)
    return topk_t<KP, OK, 8>(fp, a_out, k, splits, pscore, pidx, idx_out, score_out, s);
  if (kt == 12)
    return topk_t<KP, OK, 12>(fp, a_out, k, splits, pscore, pidx, idx_out, score_out, s);
  if (kt == 16)
    return topk_t<KP, OK, 16>(fp, a_out, k, splits, pscore, pidx, idx_out, score_out, s);
  return topk_t<KP, OK, 32>(fp, a_out, k, splits, pscore, pidx, idx_out, score_out, s);
}

int topk_width(int k) { return k <= 8 ? 8 : (k <= 12 ? 12 : (k <= 16 ? 16 : 32)); }

int topk_splits(int64_t R, int64_t L) { return fused_auto_splits(R, L, 128); }

hipError_t launch_topk(const FusedPass& fp, const double* a_out, int k, int splits,
                       float* pscore, int32_t* pidx, int32_t* idx_out, float* score_out,
                       hipStream_t s) {
  if (k < 1 || k > 32) return hipErrorInvalidValue;
#define IPFP_TOPK_CASE(KPV, OKV)                                                      \
  case KPV:                                                                           \
    return topk_kp<KPV, OKV>(fp, a_out, k, splits, pscore, pidx, idx_out, score_out, s);
  switch (op_kind(fp.compute)) {
    case kFP8:
      switch (fp.kpad) {
        IPFP_KP8(IPFP_TOPK_CASE, kFP8)
        default: return hipErrorInvalidValue;
      }
    case kF32:
      switch (fp.kpad) {
        IPFP_KP16(IPFP_TOPK_CASE, kF32)
        default: return hipErrorInvalidValue;
      }
    default:
      switch (fp.kpad) {
        IPFP_KP16(IPFP_TOPK_CASE, kBF16)
        default: return hipErrorInvalidValue;
      }
  }
#undef IPFP_TOPK_CASE
}

// ---- welfare gradient with respect to the factors ------------------------------
//
// dW*/dPhi = mu at the optimum (envelope theorem on eq. 2-3), so with
// Phi = X Y^T (eq. 8) the gradient of the output side is G_o = sum_r mu_or Y_r
// = a_o 2^(E - h_o) / p * sum_r P_or Ypk_r with P_or = 2^(T_or + h_o) w~_r
// (the reduction pass's terms) and Ypk = p Y the packed value rows. The pass
// is the reduction pass followed by a second product on the matrix cores
// (flash-attention-forward shape): the 32 x 32 tile of P, split into BF16
// high and low parts (about 16 significant bits together), times the value
// tile. The product needs the value rows column-contiguous and the T product
// the packed rows; both are laid out once per call in a stage image: for
// every stage of kTY reduced rows, the exact bytes its LDS buffers hold, pads
// included (packed rows of LS bytes; then, per column, the stage's values in
// two halves by bit 2 of the row index, each in order of (row >> 3, row & 3),
// and a 16-byte pad against bank conflicts). A stage is then filled by plain
// global-to-LDS copies (no registers, no LDS store instructions), and a lane
// reads the eight K values of one product MFMA as one 16-byte load. The
// product's K order is a permutation of the 32 reduced rows of a subtile that
// lets every lane feed its own P values as the B operand. A workgroup (4
// waves, one per SIMD: the FP64 sums take the registers of a second) covers
// 128 output rows and up to four 32-column blocks of G; wider rows take a
// second column group, recomputing T. FP32 accumulators are folded into FP64
// registers every IPFP_GRAD_FOLD stages; one FP64 partial per (split, row,
// column) results.

template <int KP>
struct GradImage {
  static constexpr int RB = KP * 2;               // bytes per packed row
  static constexpr int kTY = ty_for(RB);          // reduced rows per stage
  static constexpr int LS = RB + 16;              // packed row stride
  static constexpr int TS = kTY * 2 + 16;         // bytes per column per stage
  static constexpr int64_t YS = (int64_t)kTY * LS;      // packed rows of a stage
  static constexpr int64_t SS = YS + (int64_t)KP * TS;  // bytes per stage
};

// Packed rows of the stage image: stage y / kTY, row y % kTY, LS bytes (the
// row of Yr, the last row repeated past the end, then a zero pad). One thread
// per 16-byte chunk, n = T kTY LS / 16 threads.
template <int KP>
__global__ void __launch_bounds__(256)
    k_grad_image_rows(const uint8_t* __restrict__ Yr, int L, int64_t n,
                      uint8_t* __restrict__ img) {
  typedef GradImage<KP> G;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / (G::LS / 16)), cb = (int)(i % (G::LS / 16));
  const int tile = y / G::kTY, r = y % G::kTY;
  intx4 v = intx4{0, 0, 0, 0};
  if (cb < G::RB / 16)
    v = *reinterpret_cast<const intx4*>(Yr + (int64_t)min(y, L - 1) * G::RB + cb * 16);
  *reinterpret_cast<intx4*>(img + tile * G::SS + (int64_t)r * G::LS + cb * 16) = v;
}

// Value columns of the stage image: element e of half h of column c holds
// Yr[stage row 8 (e / 4) + 4 h + e % 4][c] (0 past the last row). Grid
// (Lp / 64, KP / 32), 256 threads: a block transposes 64 rows x 32 columns
// through LDS, then each thread writes 8 values (16 bytes) of one column half.
template <int KP>
__global__ void __launch_bounds__(256)
    k_grad_image_cols(const uint8_t* __restrict__ Yr, int L, uint8_t* __restrict__ img) {
  typedef GradImage<KP> G;
  __shared__ __attribute__((aligned(16))) uint16_t tile[32][72];   // [column][row]
  const int t = threadIdx.x;
  const int y0 = blockIdx.x * 64, c0 = blockIdx.y * 32;
  {
    const int r = t >> 2, j = t & 3;          // 64 rows x 4 chunks of 8 columns
    const int y = y0 + r;
    intx4 v = intx4{0, 0, 0, 0};
    if (y < L) v = *reinterpret_cast<const intx4*>(Yr + (int64_t)y * G::RB + (c0 + 8 * j) * 2);
#pragma unroll
    for (int i = 0; i < 8; ++i)
      tile[8 * j + i][r] = (uint16_t)((uint32_t)v[i >> 1] >> (16 * (i & 1)));
  }
  __syncthreads();
  const int c = t >> 3, h = (t >> 2) & 1, k = t & 3;
  const int stage = y0 / G::kTY, lr0 = y0 % G::kTY;   // lr0 is 0 or 64
  const int e0 = lr0 / 2 + 8 * k;
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 8; i += 2) {
    const int ea = e0 + i, eb = ea + 1;
    const int ra = 8 * (ea >> 2) + 4 * h + (ea & 3) - lr0;
    const int rb = 8 * (eb >> 2) + 4 * h + (eb & 3) - lr0;
    w[i / 2] = (uint32_t)tile[c][ra] | ((uint32_t)tile[c][rb] << 16);
  }
  uint8_t* col = img + stage * G::SS + G::YS + (int64_t)(c0 + c) * G::TS;
  *reinterpret_cast<intx4*>(col + h * G::kTY + e0 * 2) =
      intx4{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
  if (lr0 == 0 && h == 0 && k == 0)
    *reinterpret_cast<intx4*>(col + 2 * G::kTY) = intx4{0, 0, 0, 0};
}

// Stages of FP32 product accumulation between folds into the FP64 sums: each
// FP32 accumulator takes kTY / 8 MFMA additions per stage (16 at kTY = 128,
// high and low parts), so a fold every F stages bounds its rounding at about
// 16 F x 2^-24 of the folded terms' magnitudes.
#ifndef IPFP_GRAD_FOLD
#define IPFP_GRAD_FOLD 8
#endif

// 32-column blocks of G per workgroup (at most), and waves per workgroup
constexpr int grad_col_blocks(int kp) { return kp / 32 < 4 ? kp / 32 : 4; }
constexpr int kGradWaves = 4;

// Copies `bytes` (a multiple of 16) from global memory to LDS, the waves of
// the workgroup taking 1 KiB (64 lanes x 16 bytes) each in turn: lane l of a
// copy writes 16 bytes at the copy's LDS base + 16 l.
template <int WAVES, int BYTES>
__device__ __forceinline__ void stage_copy(const uint8_t* src, uint8_t* dst, int wave, int lane) {
  static_assert(BYTES % 16 == 0, "whole 16-byte chunks");
  constexpr int kCopies = (BYTES + 1023) / 1024;
#pragma unroll
  for (int i = 0; i < (kCopies + WAVES - 1) / WAVES; ++i) {
    const int c = wave + i * WAVES;
    if (c * 1024 + lane * 16 < BYTES)
      __builtin_amdgcn_global_load_lds(
          (const void*)(src + c * 1024 + lane * 16),
          (__attribute__((address_space(3))) void*)(dst + c * 1024), 16, 0, 0);
  }
}

// Waits until this wave's global-to-LDS copies (and every other vector memory
// load) have landed: vmcnt(0), expcnt and lgkmcnt left at their maxima.
__device__ __forceinline__ void wait_vector_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// NBL 32-column blocks per workgroup, a compile-time count: the product loop
// then has no branches, and its LDS reads and MFMAs schedule as one block.
// Groups g = 0 .. ngroups-1 cover column blocks nb_base + NBL g onwards; a
// row of 2d columns that is not a multiple of 4 blocks takes a second launch
// for its last, narrower group.
template <int KP, int NBL>
__global__ void __launch_bounds__(kGradWaves * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
    k_grad_pass(const uint8_t* __restrict__ Xo, const uint8_t* __restrict__ img,
                const double* __restrict__ wred, const int* __restrict__ Eptr,
                const float* __restrict__ shift, int R, int L, int tiles_per_split, int nsplit,
                int ngroups, int nb_base, double* __restrict__ gpart) {
  constexpr int WAVES = kGradWaves;
  typedef PassCore<KP, 1, WAVES, kBF16> C;
  typedef GradImage<KP> G;
  typedef typename C::Frag Frag;
  typedef Op<kBF16> O;
  constexpr int RB = C::RB, kTY = C::kTY, NS = C::NS, LS = C::LS, SUB = C::SUB;
  static_assert(LS == G::LS && kTY == G::kTY, "stage image layout");
  static_assert(NBL >= 1 && NBL <= 4 && NBL <= KP / 32, "column blocks per workgroup");
  constexpr int TS = G::TS;
  constexpr int YS = (int)G::YS;            // bytes of packed rows per stage
  constexpr int YT = NBL * 32 * TS;         // bytes of this group's columns per stage
  __shared__ __attribute__((aligned(16))) uint8_t ys[2][YS];
  __shared__ __attribute__((aligned(16))) uint8_t yt[2][YT];
  __shared__ __attribute__((aligned(16))) float ws[2][kTY];

  int E = *Eptr;
  if (E == INT_MIN) E = 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int rblocks = (R + WAVES * 32 - 1) / (WAVES * 32);
  const int item = xcd_item(blockIdx.x, rblocks * nsplit * ngroups);
  const int unit = item / rblocks, rb = item - unit * rblocks;
  const int split = unit / ngroups, grp = unit - split * ngroups;
  const int nb0 = nb_base + grp * NBL;
  const int T = (L + kTY - 1) / kTY;
  const int t0 = split * tiles_per_split, t1 = min(T, t0 + tiles_per_split);
  const int x = (rb * WAVES + wave) * 32 + l32;
  const bool ok = x < R;

  Frag bfrag[NS];
  {
    const uint8_t* src = Xo + (int64_t)(ok ? x : 0) * RB + h * O::SB;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Frag f = lds_frag<kBF16>(src, s);
      if (!ok) *reinterpret_cast<intx4*>(&f) = intx4{0, 0, 0, 0};
      bfrag[s] = f;
    }
  }
  const float hv = ok ? shift[x] : 0.f;
  floatx16 g32[NBL];
  double g64[NBL][16];
  {
    // The FP32 product sums start as the result of an MFMA (of zeros), like
    // every later value they take. Started from constant zeros, they were
    // kept in vector registers across the stage loop and copied to and from
    // the accumulator registers at every stage (128 moves per stage).
    const bf16x8 z = {};
    floatx16 c0;
#pragma unroll
    for (int j = 0; j < 16; ++j) c0[j] = 0.f;
#pragma unroll
    for (int nb = 0; nb < NBL; ++nb) g32[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(z, z, c0, 0, 0, 0);
  }
#pragma unroll
  for (int nb = 0; nb < NBL; ++nb)
#pragma unroll
    for (int j = 0; j < 16; ++j) g64[nb][j] = 0.0;

  // a stage's packed rows and this group's value columns, straight from the
  // image into LDS buffer b; every thread loads the weight of row tid % kTY
  // (duplicates store identical values)
  float pw = 0.f;
  auto stage_in = [&](int tile, int b) {
    const uint8_t* src = img + (int64_t)tile * G::SS;
    stage_copy<WAVES, YS>(src, ys[b], wave, lane);
    stage_copy<WAVES, YT>(src + G::YS + (int64_t)32 * nb0 * TS, yt[b], wave, lane);
    const int y = tile * kTY + (tid % kTY);
    pw = y < L ? (float)ldexp(wred[min(y, L - 1)], -E) : 0.f;
  };

  if (t0 < t1) {
    stage_in(t0, 0);
    ws[0][tid % kTY] = pw;
  }
  wait_vector_loads();
  __syncthreads();
  // one subtile's T + h (an MFMA chain over the packed row; the first MFMA
  // adds the loop-invariant block of h)
  floatx16 shv;
#pragma unroll
  for (int j = 0; j < 16; ++j) shv[j] = hv;
  // TP subtiles' chains at a time, interleaved k-step by k-step, so that
  // consecutive MFMAs are independent: all four of a stage when it has four,
  // else one (MI355X, C3, each against the build before it on one box: one
  // chain -> two, with the products paired, 912 -> 874 ms; two -> four 860
  // -> 849 ms; the same sums bit for bit)
  constexpr int TP = SUB >= 4 ? 4 : 1;
  auto tgrp = [&](int buf, int sub, floatx16 (&out)[TP]) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int u = 0; u < TP; ++u) {
        const uint8_t* arow = &ys[buf][((sub + u) * 32 + l32) * LS + h * O::SB];
        out[u] = mfma_step<kBF16>(lds_frag<kBF16>(arow, s), bfrag[s], s == 0 ? shv : out[u],
                                  127, 127);
      }
  };
  for (int tile = t0; tile < t1; ++tile) {
    const int buf = (tile - t0) & 1;
    // the other buffer was last read before the barrier that ended the
    // previous stage: the next stage's copies go out before this stage's work
    const bool more = tile + 1 < t1;
    if (more) stage_in(tile + 1, buf ^ 1);
    // the next group's T chains (if any in this stage) are issued ahead of
    // this group's exp2 and products, which do not depend on them
    floatx16 nxt[TP], cur[TP];
    tgrp(buf, 0, nxt);
#pragma unroll
    for (int sub = 0; sub < SUB; ++sub) {
      if (sub % TP == 0) {
#pragma unroll
        for (int u = 0; u < TP; ++u) cur[u] = nxt[u];
        if (sub + TP < SUB) tgrp(buf, sub + TP, nxt);
      }
      const floatx16 acc = cur[sub % TP];
      float p[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int yr = sub * 32 + 8 * (j >> 2) + 4 * h + (j & 3);
        p[j] = __builtin_amdgcn_exp2f(acc[j]) * ws[buf][yr];
      }
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        // B operand: this lane's P at K slots 8h..8h+7 (reduced rows
        // 16 ks + 8 (i / 4) + 4 h + i % 4), high and low BF16 parts
        // (hardware round-to-nearest-even conversions, two values each;
        // v - hi is exact in FP32)
        bf16x8 bh, bl;
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
          const floatx2 v = {p[8 * ks + i], p[8 * ks + i + 1]};
          const bf16x2 hv2 = __builtin_convertvector(v, bf16x2);
          const floatx2 rest2 = v - __builtin_convertvector(hv2, floatx2);
          const bf16x2 lv = __builtin_convertvector(rest2, bf16x2);
          bh[i] = hv2[0];
          bh[i + 1] = hv2[1];
          bl[i] = lv[0];
          bl[i + 1] = lv[1];
        }
        // A operand: value column 32 (nb0 + nb) + l32 at the same eight rows
        // (r0..r0+3, r0+8..r0+11, r0 = 32 sub + 16 ks + 4 h): positions
        // 16 sub + 8 ks .. + 7 of half h
        auto colfrag = [&](int nb) {
          const uint8_t* col = &yt[buf][(32 * nb + l32) * TS + h * kTY + sub * 32 + ks * 16];
          const intx4 av = *reinterpret_cast<const intx4*>(col);
          return *reinterpret_cast<const bf16x8*>(&av);
        };
        // all column blocks' high parts, then their low parts: consecutive
        // MFMAs never accumulate into the same sums, and each sum still
        // takes hi before lo, k-step 0 before 1
        bf16x8 acol[NBL];
#pragma unroll
        for (int nb = 0; nb < NBL; ++nb) acol[nb] = colfrag(nb);
#pragma unroll
        for (int nb = 0; nb < NBL; ++nb)
          g32[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(acol[nb], bh, g32[nb], 0, 0, 0);
#pragma unroll
        for (int nb = 0; nb < NBL; ++nb)
          g32[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(acol[nb], bl, g32[nb], 0, 0, 0);
      }
    }
    // lane (o, h) holds columns 32 (nb0 + nb) + 8 (j / 4) + 4 h + j % 4 of row o;
    // the FP32 products are folded into the FP64 sums every IPFP_GRAD_FOLD
    // stages (and after the last)
    if ((tile - t0) % IPFP_GRAD_FOLD == IPFP_GRAD_FOLD - 1 || tile == t1 - 1) {
#pragma unroll
      for (int nb = 0; nb < NBL; ++nb)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          g64[nb][j] += (double)g32[nb][j];
          g32[nb][j] = 0.f;
        }
    }
    if (more) ws[buf ^ 1][tid % kTY] = pw;
    wait_vector_loads();
    __syncthreads();
  }
  if (ok) {
    double* dst = gpart + ((int64_t)split * R + x) * KP + 32 * nb0;
#pragma unroll
    for (int nb = 0; nb < NBL; ++nb)
#pragma unroll
      for (int j = 0; j < 16; ++j) dst[32 * nb + 8 * (j >> 2) + 4 * h + (j & 3)] = g64[nb][j];
  }
}

// G_o,c = a_o 2^(E - h_o) / p * sum over splits (fixed order), columns c < 2d.
__global__ void __launch_bounds__(256)
    k_grad_combine(const double* __restrict__ gpart, int nsplit, int R, int kpad, int width,
                   const int* __restrict__ Eptr, const float* __restrict__ shift,
                   const double* __restrict__ a_out, double inv_p, double* __restrict__ g,
                   int64_t ld_g) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)R * width) return;
  const int o = (int)(i / width), c = (int)(i % width);
  int E = *Eptr;
  if (E == INT_MIN) E = 0;
  double sum = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) sum += gpart[((int64_t)sp * R + o) * kpad + c];
  g[(int64_t)o * ld_g + c] = sum * exp2((double)E - (double)shift[o]) * a_out[o] * inv_p;
}

template <int KP>
static size_t grad_t_scratch(int64_t L) {
  typedef GradImage<KP> G;
  return (size_t)((L + G::kTY - 1) / G::kTY) * (size_t)G::SS;
}

template <int KP>
static hipError_t grad_t(const FusedPass& fp, const int* Eptr, const double* a_out, double inv_p,
                         int splits, double* gpart, uint8_t* img, int width, double* g,
                         int64_t ld_g, hipStream_t s) {
  typedef GradImage<KP> G;
  constexpr int kTY = G::kTY;
  constexpr int NB = KP / 32, NBL = grad_col_blocks(KP);
  constexpr int FULL = NB / NBL, REM = NB % NBL;
  const int64_t rblocks = (fp.out.rows + kGradWaves * 32 - 1) / (kGradWaves * 32);
  const int L = (int)fp.red.rows;
  const int T = (L + kTY - 1) / kTY;
  const int Lp = T * kTY;
  const int tps = (T + splits - 1) / splits;
  const int64_t nrow = (int64_t)Lp * (G::LS / 16);
  hipLaunchKernelGGL((k_grad_image_rows<KP>), dim3((unsigned)((nrow + 255) / 256)), dim3(256), 0,
                     s, (const uint8_t*)fp.red.ops, L, nrow, img);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_grad_image_cols<KP>), dim3((unsigned)(Lp / 64), (unsigned)(KP / 32)),
                     dim3(256), 0, s, (const uint8_t*)fp.red.ops, L, img);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_grad_pass<KP, NBL>), dim3((unsigned)(rblocks * splits * FULL)),
                     dim3(kGradWaves * 64), 0, s, (const uint8_t*)fp.out.ops,
                     (const uint8_t*)img, fp.w_red, Eptr, fp.shift, (int)fp.out.rows, L, tps,
                     splits, FULL, 0, gpart);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if constexpr (REM > 0) {
    hipLaunchKernelGGL((k_grad_pass<KP, REM>), dim3((unsigned)(rblocks * splits)),
                       dim3(kGradWaves * 64), 0, s, (const uint8_t*)fp.out.ops,
                       (const uint8_t*)img, fp.w_red, Eptr, fp.shift, (int)fp.out.rows, L, tps,
                       splits, 1, FULL * NBL, gpart);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t n = fp.out.rows * width;
  hipLaunchKernelGGL(k_grad_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gpart,
                     splits, (int)fp.out.rows, (int)fp.kpad, width, Eptr, fp.shift, a_out,
                     inv_p, g, ld_g);
  return hipGetLastError();
}

#define IPFP_GRAD_KPADS(X) X(32) X(64) X(96) X(128) X(160) X(192) X(224) X(256)

// Workgroups of the gradient pass (its full column groups) that one compute
// unit holds at once (HIP occupancy query; 1 when the query fails).
template <int KP>
static int grad_wgs_per_cu() {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &n, reinterpret_cast<const void*>(&k_grad_pass<KP, grad_col_blocks(KP)>), kGradWaves * 64,
      0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

// Split count of the gradient pass, as fused_pass_splits does for the sum
// pass but with the gradient's own occupancy (one 140 KB workgroup per
// compute unit at kpad 128) and at most max_splits: minimises (waves of
// workgroups) x (stages per workgroup + 1), at least 8 stages per split, the
// smaller count on ties. At N = M = 10^6, d = 64 three splits leave the last
// wave of workgroups half full instead of a one-split grid's 52 %.
int gradient_splits(int64_t R, int64_t L, int kpad, int max_splits) {
  int per_cu = 1;
  switch (kpad) {
#define IPFP_GRAD_OCC(K) \
    case K: per_cu = grad_wgs_per_cu<K>(); break;
    IPFP_GRAD_KPADS(IPFP_GRAD_OCC)
#undef IPFP_GRAD_OCC
    default: break;
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    cus = 256;
  }
  const int64_t slots = (int64_t)cus * per_cu;
  const int nb = kpad / 32, nbl = grad_col_blocks(kpad);
  const int64_t groups = nb / nbl + (nb % nbl ? 1 : 0);
  const int64_t rblocks = (R + kGradWaves * 32 - 1) / (kGradWaves * 32);
  const int stage = ty_for(kpad * 2);
  const int64_t T = (L + stage - 1) / stage;
  int best = 1;
  int64_t best_cost = INT64_MAX;
  for (int S = 1; S <= max_splits; ++S) {
    if (S > 1 && T / S < 8) break;
    const int64_t waves = (rblocks * groups * S + slots - 1) / slots;
    const int64_t cost = waves * ((T + S - 1) / S + 1);
    if (cost < best_cost) {
      best_cost = cost;
      best = S;
    }
  }
  return best;
}

size_t gradient_scratch_bytes(int kpad, int64_t L) {
  switch (kpad) {
#define IPFP_GRAD_CASE(K) \
    case K: return grad_t_scratch<K>(L);
    IPFP_GRAD_KPADS(IPFP_GRAD_CASE)
#undef IPFP_GRAD_CASE
    default: return 0;
  }
}

hipError_t launch_gradient(const FusedPass& fp, const int* Eptr, const double* a_out,
                           double inv_p, int splits, double* gpart, uint8_t* img, int width,
                           double* g, int64_t ld_g, hipStream_t s) {
  if (fp.compute != IPFP_BF16) return hipErrorInvalidValue;
  switch (fp.kpad) {
#define IPFP_GRAD_CASE(K) \
    case K: return grad_t<K>(fp, Eptr, a_out, inv_p, splits, gpart, img, width, g, ld_g, s);
    IPFP_GRAD_KPADS(IPFP_GRAD_CASE)
#undef IPFP_GRAD_CASE
    default: return hipErrorInvalidValue;
  }
}
#undef IPFP_GRAD_KPADS

// ---- combine partial sums, update scalings -----------------------------------

// Finishes output row o given lS = log2((K w)_o): the residual of the current
// scaling (eq. 5) and the quadratic root of eq. 6. Returns the residual.
__device__ __forceinline__ double finish_row(int64_t o, double lS,
                                             const double* marg,
                                             const double* w_old, double* w_new,
                                             bool residual, Ctl* ctl) {
  const double nx = marg[o];
  double res = 0.0;
  if (residual) {
    const double wo = w_old[o];
    const double two_s_wo = wo > 0.0 ? exp2(log2(wo) + lS) : 0.0;
    res = fabs(fma(wo, wo, -nx) + two_s_wo) / nx;
  }
  const double w = lS < 1000.0 ? quad_root(nx, exp2(lS - 1.0)) : nx * exp2(-lS);
  if (!__builtin_isfinite(w)) atomicOr(&ctl->nonfinite, 1);
  w_new[o] = w;
  return res;
}

// Block-wide max of (residual, exponent) pairs: residual to *res_slot,
// exponent folded into *wexp by one atomic per block.
__device__ __forceinline__ void block_finish(double res, int ex, double* res_slot,
                                             int* wexp) {
  __shared__ double rred[4];
  __shared__ int ered[4];
  res = wave_max(res);
  ex = wave_max(ex);
  if ((threadIdx.x & 63) == 0) {
    rred[threadIdx.x >> 6] = res;
    ered[threadIdx.x >> 6] = ex;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *res_slot = fmax(fmax(rred[0], rred[1]), fmax(rred[2], rred[3]));
    const int e = max(max(ered[0], ered[1]), max(ered[2], ered[3]));
    if (e != INT_MIN) atomicMax(wexp, e);
  }
}

// Dot product of two packed rows in FP32, one FMA chain in index order, the
// operands read in 16-byte chunks (a row is a multiple of 64 bytes).
template <int OK>
__device__ __forceinline__ float dot_packed(const uint8_t* a, const uint8_t* b,
                                            int kpad) {
  const int nc = kpad * Op<OK>::ES / 16;
  float acc = 0.f;
  for (int c = 0; c < nc; ++c) {
    const intx4 va = *reinterpret_cast<const intx4*>(a + 16 * c);
    const intx4 vb = *reinterpret_cast<const intx4*>(b + 16 * c);
    if constexpr (OK == kFP8) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
        acc = fmaf(e4m3_val((uint8_t)((uint32_t)va[q >> 2] >> (8 * (q & 3)))),
                   e4m3_val((uint8_t)((uint32_t)vb[q >> 2] >> (8 * (q & 3)))), acc);
    } else if constexpr (OK == kF32) {
#pragma unroll
      for (int q = 0; q < 4; ++q) acc = fmaf(__int_as_float(va[q]), __int_as_float(vb[q]), acc);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint32_t ua = (uint32_t)va[q >> 1], ub = (uint32_t)vb[q >> 1];
        acc = fmaf(__uint_as_float((q & 1) ? (ua & 0xFFFF0000u) : (ua << 16)),
                   __uint_as_float((q & 1) ? (ub & 0xFFFF0000u) : (ub << 16)), acc);
      }
    }
  }
  return acc;
}

// Exact fallback for rows whose shifted sum left the safe range: two passes
// over the reduced side with FP32 dot products of the same packed operands and
// FP64 log2 weights, the first for the maximum exponent, the second for the
// sum. The workgroup takes up to fix_rows(OK) rows at a time: their packed
// rows are staged in LDS, and each reduced row's operands and weight logarithm
// are read once for all of them (each row's own arithmetic is that of a row
// taken alone). Writes log2 (K w)_o of rows[j] to lS[j], j < nr, in every
// thread. Four rows (one for FP8, whose decoding takes more registers) keep
// the combine kernels within 128 VGPRs, four workgroups per compute unit.
constexpr int fix_rows(int ok) { return ok == kFP8 ? 1 : 4; }

template <int OK, int kFixRows = fix_rows(OK)>
__device__ __forceinline__ void exact_rows_log2(const GroupHalf& p, const double* wred,
                                                const int64_t (&rows)[kFixRows], int nr,
                                                double (&lS)[kFixRows]) {
  __shared__ double dred[kFixRows][4];
  __shared__ __attribute__((aligned(16))) uint8_t xs[kFixRows][1024];
  constexpr bool FP8 = OK == kFP8;
  const int kpad = p.kpad, rbytes = kpad * Op<OK>::ES;   // at most 1024
  for (int j = 0; j < nr; ++j)
    for (int c = threadIdx.x; c < rbytes / 16; c += 256)
      reinterpret_cast<intx4*>(xs[j])[c] =
          reinterpret_cast<const intx4*>(p.Xo + rows[j] * rbytes)[c];
  float sx[kFixRows];
  double tmax[kFixRows], sum[kFixRows];
#pragma unroll
  for (int j = 0; j < kFixRows; ++j) {
    sx[j] = FP8 && j < nr ? p.xscale[rows[j]] : 1.f;
    tmax[j] = -INFINITY;
    sum[j] = 0.0;
  }
  __syncthreads();
  for (int64_t y = threadIdx.x; y < p.L; y += 256) {
    const float ysc = FP8 ? p.yscale[y] : 1.f;
    const double lw = log2(wred[y]);
    const uint8_t* yr = p.Yr + y * rbytes;
#pragma unroll
    for (int j = 0; j < kFixRows; ++j)
      if (j < nr) {
        const float sc = FP8 ? sx[j] * ysc : 1.f;
        tmax[j] = fmax(tmax[j], (double)(dot_packed<OK>(xs[j], yr, kpad) * sc) + lw);
      }
  }
#pragma unroll
  for (int j = 0; j < kFixRows; ++j) {
    if (j >= nr) break;
    const double m = wave_max(tmax[j]);
    if ((threadIdx.x & 63) == 0) dred[j][threadIdx.x >> 6] = m;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kFixRows; ++j)
    if (j < nr) tmax[j] = fmax(fmax(dred[j][0], dred[j][1]), fmax(dred[j][2], dred[j][3]));
  __syncthreads();
  for (int64_t y = threadIdx.x; y < p.L; y += 256) {
    const float ysc = FP8 ? p.yscale[y] : 1.f;
    const double lw = log2(wred[y]);
    const uint8_t* yr = p.Yr + y * rbytes;
#pragma unroll
    for (int j = 0; j < kFixRows; ++j)
      if (j < nr && tmax[j] > -INFINITY) {
        const float sc = FP8 ? sx[j] * ysc : 1.f;
        sum[j] += exp2((double)(dot_packed<OK>(xs[j], yr, kpad) * sc) + lw - tmax[j]);
      }
  }
#pragma unroll
  for (int j = 0; j < kFixRows; ++j) {
    if (j >= nr) break;
    const double t = wave_sum(sum[j]);
    if ((threadIdx.x & 63) == 0) dred[j][threadIdx.x >> 6] = t;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kFixRows; ++j) {
    if (j >= nr) break;
    const double t = (dred[j][0] + dred[j][1]) + (dred[j][2] + dred[j][3]);
    lS[j] = t > 0.0 ? tmax[j] + log2(t) : -INFINITY;
  }
  __syncthreads();
}

// Combine of one workgroup's 256 output rows: the split partial sums in fixed
// order (FP64), the residual of the old scaling and the quadratic update of
// eq. 6; rows whose sum left [2^-60, inf) are recomputed exactly by the whole
// workgroup (exact_rows_log2) before the block's residual and exponent maxima
// are published. For the row pass (p.residual) the last workgroup to finish
// (arrival counter in the control block) runs the convergence check, so a
// sweep needs no separate fallback or check launch.
template <int OK>
__device__ __forceinline__ void combine_body(const GroupHalf& p, const int bid,
                                             const int nblocks) {
  __shared__ int32_t bad[256];
  __shared__ int nbad;
  __shared__ int last;
  Ctl* ctl = p.ctl;
  if (ctl->done) return;
  const int64_t R = p.R;
  const int i = ctl->sweep;
  const double* w_old = p.dbuf ? p.w2 + (int64_t)(i & 1) * R : p.w2;
  double* w_new = p.dbuf ? p.w2 + (int64_t)((i + 1) & 1) * R : p.w2;
  int E = ctl->wexp[p.exp_red];
  if (E == INT_MIN) E = 0;
  if (threadIdx.x == 0) nbad = 0;
  __syncthreads();
  const int64_t o = (int64_t)bid * 256 + threadIdx.x;
  double res = 0.0;
  int ex = INT_MIN;
  if (o < R) {
    double l = 0.0;
    for (int k = 0; k < p.nsplit; ++k) l += p.part[(int64_t)k * R + o];
    if (!(l >= 0x1p-60) || l == INFINITY) {  // out of the safe range (or NaN)
      bad[atomicAdd(&nbad, 1)] = (int32_t)threadIdx.x;
    } else {
      const double lS = log2(l) + (double)E - (double)p.shift[o];
      res = finish_row(o, lS, p.marg, w_old, w_new, p.residual != 0, ctl);
      ex = exponent_of(w_new[o]);
    }
  }
  __syncthreads();
  const int nb = nbad;
  if (nb > 0) {
    const double* wred = p.red_dbuf ? p.wred + (int64_t)(i & 1) * p.L : p.wred;
    constexpr int kFixRows = fix_rows(OK);
    for (int k0 = 0; k0 < nb; k0 += kFixRows) {
      const int nr = min(kFixRows, nb - k0);
      int64_t rows[kFixRows];
      double lS[kFixRows];
#pragma unroll
      for (int j = 0; j < kFixRows; ++j) rows[j] = (int64_t)bid * 256 + bad[k0 + min(j, nr - 1)];
      exact_rows_log2<OK>(p, wred, rows, nr, lS);
#pragma unroll
      for (int j = 0; j < kFixRows; ++j)
        if (j < nr && (int)threadIdx.x == bad[k0 + j]) {
          res = finish_row(rows[j], lS[j], p.marg, w_old, w_new, p.residual != 0, ctl);
          ex = exponent_of(w_new[rows[j]]);
        }
    }
    if (threadIdx.x == 0) atomicAdd(&ctl->fix_total, nb);
  }
  block_finish(res, ex, &p.res_block[bid], &ctl->wexp[p.exp_out]);
  if (!p.residual) return;
  // arrival: this block's residual (and any flag it raised) is visible before
  // the counter moves; the last block resets the counter and runs the check
  __threadfence();
  if (threadIdx.x == 0) last = atomicAdd(&ctl->arrive, 1) == nblocks - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) ctl->arrive = 0;
  check_body(ctl, p.res_block, nblocks, p.hist, p.sp);
}

template <int OK>
__global__ void __launch_bounds__(256) k_fused_combine(GroupHalf p) {
  combine_body<OK>(p, (int)blockIdx.x, (int)gridDim.x);
}

template <int OK>
__global__ void __launch_bounds__(256)
    k_group_combine(const GroupHalf* __restrict__ g, const int32_t* __restrict__ first,
                    int count) {
  const int j = group_find(first, count, (int)blockIdx.x);
  const int b0 = __builtin_amdgcn_readfirstlane(first[j]);
  const int b1 = __builtin_amdgcn_readfirstlane(first[j + 1]);
  combine_body<OK>(g[j], (int)blockIdx.x - b0, b1 - b0);
}

// The max pass's combine: h_o = -max over splits.
__global__ void k_shift_from_max(const double* part, int splits, int64_t R,
                                 float* shift) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= R) return;
  double m = -INFINITY;
  for (int k = 0; k < splits; ++k) m = fmax(m, part[(int64_t)k * R + o]);
  shift[o] = (float)(-m);
}

// ctl->wexp[idx] = largest binary exponent of w (one workgroup).
__global__ void __launch_bounds__(256) k_init_exp(const double* w, int64_t len,
                                                  Ctl* ctl, int idx) {
  __shared__ int red[4];
  int e = INT_MIN;
  for (int64_t k = threadIdx.x; k < len; k += 256) e = max(e, exponent_of(w[k]));
  e = wave_max(e);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) ctl->wexp[idx] = max(max(red[0], red[1]), max(red[2], red[3]));
}

hipError_t launch_init_exp(const double* w, int64_t len, Ctl* ctl, int idx,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_init_exp, dim3(1), dim3(256), 0, s, w, len, ctl, idx);
  return hipGetLastError();
}

// ---- dispatch ---------------------------------------------------------------

template <int KP, int XT, int WAVES, int OK, bool MAXMODE>
static hipError_t pass_t(const FusedPass& fp, Ctl* ctl, hipStream_t s) {
  constexpr int kTY = ty_for(KP * Op<OK>::ES);
  const int rows_per_wg = WAVES * XT * 32;
  const int64_t rblocks = (fp.out.rows + rows_per_wg - 1) / rows_per_wg;
  const int T = (int)((fp.red.rows + kTY - 1) / kTY);
  const int tps = (T + fp.splits - 1) / fp.splits;
  const int64_t grid = rblocks * fp.splits;
  hipLaunchKernelGGL((k_fused_pass<KP, XT, WAVES, OK, MAXMODE>), dim3((unsigned)grid),
                     dim3(WAVES * 64), 0, s, (const uint8_t*)fp.out.ops,
                     fp.out.scale, (const uint8_t*)fp.red.ops, fp.red.scale,
                     fp.w_red, fp.red_dbuf, fp.exp_red, fp.exp_out, fp.shift, (int)fp.out.rows,
                     (int)fp.red.rows, tps, fp.splits, fp.part, ctl);
  return hipGetLastError();
}

template <int KP, int OK, bool MAXMODE>
static hipError_t pass_kp(const FusedPass& fp, Ctl* ctl, hipStream_t s) {
  constexpr int XT = xt_for(KP, OK);
  if constexpr (OK == kF32) {
    return pass_t<KP, XT, 4, OK, MAXMODE>(fp, ctl, s);
  } else {
    if (pass_waves(OK, XT, fp.tile_rows) == 8) return pass_t<KP, XT, 8, OK, MAXMODE>(fp, ctl, s);
    return pass_t<KP, XT, 4, OK, MAXMODE>(fp, ctl, s);
  }
}

template <bool MAXMODE>
static hipError_t pass_any(const FusedPass& fp, Ctl* ctl, hipStream_t s) {
#define IPFP_PASS_CASE(K, OKV) \
  case K: return pass_kp<K, OKV, MAXMODE>(fp, ctl, s);
  switch (op_kind(fp.compute)) {
    case kFP8:
      switch (fp.kpad) {
        IPFP_KP8(IPFP_PASS_CASE, kFP8)
        default: return hipErrorInvalidValue;
      }
    case kF32:
      switch (fp.kpad) {
        IPFP_KP16(IPFP_PASS_CASE, kF32)
        default: return hipErrorInvalidValue;
      }
    default:
      switch (fp.kpad) {
        IPFP_KP16(IPFP_PASS_CASE, kBF16)
        default: return hipErrorInvalidValue;
      }
  }
#undef IPFP_PASS_CASE
}

hipError_t launch_fused_pass(const FusedPass& fp, Ctl* ctl, hipStream_t s) {
  return pass_any<false>(fp, ctl, s);
}

// Set-up: h_o = -max_r T_or for the pass's output side (uses fp.part).
hipError_t launch_fused_shift(const FusedPass& fp, Ctl* ctl, hipStream_t s) {
  hipError_t e = pass_any<true>(fp, ctl, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_shift_from_max, dim3((unsigned)((fp.out.rows + 255) / 256)),
                     dim3(256), 0, s, fp.part, fp.splits, fp.out.rows, fp.shift);
  return hipGetLastError();
}

// Default workgroup height (tile_rows = 0). Measured on MI355X at N = M = 1e6:
// the two-tile kernels of BF16 with 2d = 64 and FP8 with 2d <= 128 run 8-16 %
// faster as 4-wave workgroups (several share a compute unit) than as 8-wave
// ones; BF16 with 2d = 128 is 1-2 % faster with 8 waves; one-tile kernels use
// 8 waves either way.
int fused_default_tile_rows(int64_t kpad, ipfp_dtype compute) {
  if (compute == IPFP_F32) return 128;
  const bool fp8 = compute == IPFP_FP8E4M3;
  if (fp8 ? kpad <= 128 : kpad == 64) return 256;
  return 512;
}

int fused_rows_per_wg(int64_t kpad, ipfp_dtype compute, int tile_rows) {
  const int ok = op_kind(compute);
  const int xt = xt_for((int)kpad, ok);
  return pass_waves(ok, xt, tile_rows) * xt * 32;
}

GroupHalf fused_half(const FusedPass& fp, Ctl* ctl, double* w2, int dbuf, double* hist,
                     SweepParams sp) {
  GroupHalf g{};
  g.Xo = (const uint8_t*)fp.out.ops;
  g.xscale = fp.out.scale;
  g.Yr = (const uint8_t*)fp.red.ops;
  g.yscale = fp.red.scale;
  g.wred = fp.w_red;
  g.shift = fp.shift;
  g.part = fp.part;
  g.ctl = ctl;
  g.marg = fp.marg;
  g.w2 = w2;
  g.res_block = fp.res_block;
  g.hist = hist;
  g.sp = sp;
  g.red_dbuf = fp.red_dbuf;
  g.exp_red = fp.exp_red;
  g.exp_out = fp.exp_out;
  g.R = (int32_t)fp.out.rows;
  g.L = (int32_t)fp.red.rows;
  int64_t blocks = 0;
  int tps = 0;
  fused_pass_grid(fp, &blocks, &tps);
  g.tiles_per_split = tps;
  g.nsplit = fp.splits;
  g.dbuf = dbuf;
  g.residual = fp.residual ? 1 : 0;
  g.kpad = (int32_t)fp.kpad;
  return g;
}

int fused_combine_blocks(int64_t rows) { return (int)((rows + 255) / 256); }

hipError_t launch_fused_combine(const FusedPass& fp, double* w2, int dbuf, Ctl* ctl,
                                double* hist, SweepParams sp, hipStream_t s) {
  const GroupHalf g = fused_half(fp, ctl, w2, dbuf, hist, sp);
  const dim3 grid((unsigned)fused_combine_blocks(fp.out.rows));
  switch (op_kind(fp.compute)) {
    case kFP8: hipLaunchKernelGGL(k_fused_combine<kFP8>, grid, dim3(256), 0, s, g); break;
    case kF32: hipLaunchKernelGGL(k_fused_combine<kF32>, grid, dim3(256), 0, s, g); break;
    default: hipLaunchKernelGGL(k_fused_combine<kBF16>, grid, dim3(256), 0, s, g); break;
  }
  return hipGetLastError();
}

// ---- grouped dispatch -----------------------------------------------------------

void fused_pass_grid(const FusedPass& fp, int64_t* blocks, int* tiles_per_split) {
  const int rows_per_wg = fused_rows_per_wg(fp.kpad, fp.compute, fp.tile_rows);
  const int ty = ty_for((int)fp.kpad * elem_bytes(op_kind(fp.compute)));
  const int64_t rblocks = (fp.out.rows + rows_per_wg - 1) / rows_per_wg;
  const int T = (int)((fp.red.rows + ty - 1) / ty);
  *tiles_per_split = (T + fp.splits - 1) / fp.splits;
  *blocks = rblocks * fp.splits;
}

template <int KP, int OK>
static hipError_t group_pass_kp(const GroupHalf* g, const int32_t* idx,
                                const int32_t* first, int count, int total, int tile_rows,
                                hipStream_t s) {
  constexpr int XT = xt_for(KP, OK);
  if (pass_waves(OK, XT, tile_rows) == 8)
    hipLaunchKernelGGL((k_group_pass<KP, XT, 8, OK>), dim3((unsigned)total), dim3(8 * 64),
                       0, s, g, idx, first, count);
  else
    hipLaunchKernelGGL((k_group_pass<KP, XT, 4, OK>), dim3((unsigned)total), dim3(4 * 64),
                       0, s, g, idx, first, count);
  return hipGetLastError();
}

hipError_t launch_group_pass(const GroupHalf* g, const int32_t* idx, const int32_t* first,
                             int count, int total, int64_t kpad, ipfp_dtype compute,
                             int tile_rows, hipStream_t s) {
  if (count <= 0 || total <= 0) return hipSuccess;
#define IPFP_GROUP_CASE(K, OKV) \
  case K: return group_pass_kp<K, OKV>(g, idx, first, count, total, tile_rows, s);
  switch (op_kind(compute)) {
    case kFP8:
      switch (kpad) {
        IPFP_KP8(IPFP_GROUP_CASE, kFP8)
        default: return hipErrorInvalidValue;
      }
    case kBF16:
      switch (kpad) {
        IPFP_KP16(IPFP_GROUP_CASE, kBF16)
        default: return hipErrorInvalidValue;
      }
    default: return hipErrorInvalidValue;   // the server runs BF16 and FP8 only
  }
#undef IPFP_GROUP_CASE
}

hipError_t launch_group_combine(const GroupHalf* g, const int32_t* first, int count,
                                int total, ipfp_dtype compute, hipStream_t s) {
  if (count <= 0 || total <= 0) return hipSuccess;
  if (compute == IPFP_FP8E4M3)
    hipLaunchKernelGGL(k_group_combine<kFP8>, dim3((unsigned)total), dim3(256), 0, s, g, first,
                       count);
  else
    hipLaunchKernelGGL(k_group_combine<kBF16>, dim3((unsigned)total), dim3(256), 0, s, g, first,
                       count);
  return hipGetLastError();
}

// Workgroups of the sum pass's instantiation for (kpad, type, tile_rows) that
// one compute unit holds at once (HIP occupancy query, cached; 1 when the
// query fails, e.g. without a device).
template <int KP, int OK>
static int pass_wgs_per_cu(int tile_rows) {
  constexpr int XT = xt_for(KP, OK);
  int n = 0;
  hipError_t e;
  if constexpr (OK == kF32) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, reinterpret_cast<const void*>(&k_fused_pass<KP, XT, 4, OK, false>), 256, 0);
  } else {
    if (pass_waves(OK, XT, tile_rows) == 8)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, reinterpret_cast<const void*>(&k_fused_pass<KP, XT, 8, OK, false>), 512, 0);
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, reinterpret_cast<const void*>(&k_fused_pass<KP, XT, 4, OK, false>), 256, 0);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

static int pass_wgs_cached(int64_t kpad, int ok, int tile_rows) {
  static std::atomic<int> cache[3][9][2];
  const int ki = (int)(kpad / 32), wi = pass_waves(ok, xt_for((int)kpad, ok), tile_rows) == 8;
  if (ki < 1 || ki > 8 || ok < 0 || ok > 2) return 1;
  const int hit = cache[ok][ki][wi].load(std::memory_order_relaxed);
  if (hit > 0) return hit;
  int n = 1;
#define IPFP_OCC_CASE(K, OKV) \
  case K: n = pass_wgs_per_cu<K, OKV>(tile_rows); break;
  switch (ok) {
    case kFP8:
      switch (kpad) {
        IPFP_KP8(IPFP_OCC_CASE, kFP8)
        default: break;
      }
      break;
    case kF32:
      switch (kpad) {
        IPFP_KP16(IPFP_OCC_CASE, kF32)
        default: break;
      }
      break;
    default:
      switch (kpad) {
        IPFP_KP16(IPFP_OCC_CASE, kBF16)
        default: break;
      }
      break;
  }
#undef IPFP_OCC_CASE
  cache[ok][ki][wi].store(n, std::memory_order_relaxed);
  return n;
}

// Split count of a sum pass (R output rows, L reduced rows). Workgroups run
// in waves of `slots` (compute units x resident workgroups per unit); a
// workgroup costs its stages plus about one stage of pipeline fill. The count
// minimises (waves of workgroups) x (stages per workgroup + 1) over 1..64,
// keeping at least 8 stages per split, the smaller count on ties. It depends
// only on the market's shape and the device, so results stay reproducible.
int fused_pass_splits(int64_t R, int64_t L, int64_t kpad, ipfp_dtype compute, int tile_rows) {
  const int ok = op_kind(compute);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    cus = 256;
  }
  const int64_t slots = (int64_t)cus * pass_wgs_cached(kpad, ok, tile_rows);
  const int rows = fused_rows_per_wg(kpad, compute, tile_rows);
  const int stage = ty_for((int)kpad * elem_bytes(ok));
  const int64_t rblocks = (R + rows - 1) / rows;
  const int64_t T = (L + stage - 1) / stage;
  int best = 1;
  int64_t best_cost = INT64_MAX;
  for (int S = 1; S <= 64; ++S) {
    if (S > 1 && T / S < 8) break;
    const int64_t waves = (rblocks * S + slots - 1) / slots;
    const int64_t cost = waves * ((T + S - 1) / S + 1);
    if (cost < best_cost) {
      best_cost = cost;
      best = S;
    }
  }
  return best;
}

// Split count of the top-k and gradient passes: enough workgroups to fill
// the 256 CUs several times over, while every split keeps at least 8 staged
// tiles.
int fused_auto_splits(int64_t R, int64_t L, int rows_per_wg) {
  const int64_t rblocks = (R + rows_per_wg - 1) / rows_per_wg;
  const int64_t T = (L + 63) / 64;
  int64_t S = 1;
  while (rblocks * S < 2048 && S * 2 <= 64 && T / (S * 2) >= 8) S *= 2;
  return (int)S;
}

}  // namespace ipfp
