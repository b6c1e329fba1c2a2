// Roofline probes: the throughput ceilings the fused and plain passes are
// measured against, taken on the device itself. Each probe is one kernel that
// does nothing but the measured operation at full occupancy, timed with HIP
// events on the caller's stream after one warm-up launch:
//  * exp2: independent chains of v_exp_f32 (results per second);
//  * MFMA: independent accumulator chains of the dense matrix instruction each
//    fused path uses (BF16 32x32x16, FP8 32x32x64 with unit scales, FP32
//    32x32x2), flops per second;
//  * HBM read: a streaming read of a buffer far larger than the caches, with
//    the plain path's 16-byte nontemporal loads, bytes per second.
// The kernels write one value per thread so nothing is optimised away.
#include <math.h>

#include <algorithm>

#include "handle.h"

namespace ipfp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int intx8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int kProbeBlocks = 256 * 8;   // 8 workgroups per compute unit
constexpr int kProbeThreads = 256;

// 8 independent chains x = 2^-x per thread: every x stays in [0.5, 1].
__global__ void __launch_bounds__(kProbeThreads) k_probe_exp2(int iters, float* out) {
  float x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = 0.5f + 0.01f * (float)(threadIdx.x & 7) + 0.001f * j;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = __builtin_amdgcn_exp2f(-x[j]);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += x[j];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// Pseudo-random operand bits (a 32-bit integer hash): the matrix cores' power,
// and with it the clock they run at, depends on how many operand bits toggle,
// so the probes feed data as varied as the passes' factors.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// A value of about N(0, 1/16) magnitude with random sign and mantissa bits.
__device__ __forceinline__ float rand_val(uint32_t h) {
  return __uint_as_float(0x3D800000u | (h & 0x807FFFFFu));   // +-[1/16, 1/8)
}

// Four independent accumulators per wave, `iters` rounds of one MFMA each.
template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) k_probe_mfma(int iters, float* out) {
  floatx16 c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) c[j][r] = 0.f;
  const uint32_t seed = blockIdx.x * kProbeThreads + threadIdx.x;
  const float f = rand_val(mix32(seed));
  if constexpr (KIND == 0) {
    bf16x8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a[k] = (__bf16)rand_val(mix32(seed * 16 + k));
      b[k] = (__bf16)rand_val(mix32(seed * 16 + 8 + k));
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) c[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[j], 0, 0, 0);
    }
  } else if constexpr (KIND == 1) {
    intx8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {   // random e4m3 codes of magnitude 2^-7 .. 240
      a[k] = (int)(mix32(seed * 16 + k) & 0xF7F7F7F7u);
      b[k] = (int)(mix32(seed * 16 + 8 + k) & 0xF7F7F7F7u);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        c[j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c[j], 0, 0, 0, 127, 0, 127);
    }
  } else {
    const float a = f, b = rand_val(mix32(seed * 16 + 1));
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) c[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c[j], 0, 0, 0);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += c[j][r];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// The matrix stream beside the fused passes' epilogue, at the passes'
// occupancy: 4-wave workgroups holding 64 KiB of LDS each, so two share a
// compute unit (two waves per SIMD), 2 workgroups per compute unit in all.
// Per round each wave issues two MFMAs on independent accumulators (the
// passes' paired chains), each followed by NE exp2 and NE FMAs on 16
// independent chains (x = 2^-x stays in [0.5, 1]); scheduling groups keep
// that order. NE = 0 is the bare matrix stream at this occupancy. The rate is
// the MFMA flops per second.
constexpr int kMixLds = 64 * 1024;
constexpr int kMixBlocks = 256 * 2;

template <int KIND, int NE>
__global__ void __launch_bounds__(kProbeThreads) k_probe_mix(int iters, float* out) {
  extern __shared__ float mix_lds[];
  floatx16 c[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) c[j][r] = 0.f;
  const uint32_t seed = blockIdx.x * kProbeThreads + threadIdx.x;
  float x[16], sum[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    x[q] = 0.5f + 0.03f * (float)q + 0.001f * (float)(threadIdx.x & 15);
    sum[q] = 0.f;
  }
  const float w = rand_val(mix32(seed));
  bf16x8 a, b;
  intx8 a8, b8;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a[k] = (__bf16)rand_val(mix32(seed * 16 + k));
    b[k] = (__bf16)rand_val(mix32(seed * 16 + 8 + k));
    a8[k] = (int)(mix32(seed * 16 + k) & 0xF7F7F7F7u);
    b8[k] = (int)(mix32(seed * 16 + 8 + k) & 0xF7F7F7F7u);
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if constexpr (KIND == 0)
        c[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[j], 0, 0, 0);
      else
        c[j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, c[j], 0, 0, 0, 127, 0, 127);
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int q = (j * NE + e) % 16;
        x[q] = __builtin_amdgcn_exp2f(-x[q]);
        sum[q] = fmaf(x[q], w, sum[q]);
      }
    }
    if constexpr (NE > 0) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x400, NE, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, NE, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += c[j][r];
#pragma unroll
  for (int q = 0; q < 16; ++q) s += sum[q];
  if (threadIdx.x == 0) mix_lds[0] = s;   // the workgroup's LDS is held, not used
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// Grid-stride streaming read of n16 16-byte chunks: each wave load covers 1 KiB
// of consecutive bytes (the plain path's access pattern), four loads in
// flight per thread (n16 a multiple of 4 x the grid's threads).
__global__ void __launch_bounds__(kProbeThreads) k_probe_read(const float4v* p, int64_t n16,
                                                              float* out) {
  float4v s[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) s[j] = float4v{};
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  for (int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x; i < n16; i += 4 * stride) {
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] += __builtin_nontemporal_load(p + i + j * stride);
  }
  float t = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) t += (s[j][0] + s[j][1]) + (s[j][2] + s[j][3]);
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = t;
}

}  // namespace
}  // namespace ipfp

using namespace ipfp;

extern "C" int ipfp_probe(ipfp_ctx* ctx, int kind, int64_t work, double* rate_out,
                          double* ms_out, void* stream) {
  if (!ctx || !rate_out || kind < IPFP_PROBE_EXP2 || kind > IPFP_PROBE_MFMA_FP8_EPI || work < 1)
    return IPFP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return IPFP_EHIP;
  const bool read = kind == IPFP_PROBE_HBM_READ;
  const size_t nout = (size_t)kProbeBlocks * kProbeThreads;
  const size_t bytes = nout * sizeof(float) + (read ? (size_t)work : 0) + 256;
  // the read covers whole rounds of four 16-byte loads per thread
  if (read && work % ((int64_t)nout * 4 * 16) != 0) return IPFP_EINVAL;
  if (ctx_reserve(ctx, bytes) != IPFP_OK) return IPFP_EBUDGET;
  char* mem = nullptr;
  if (hipMalloc((void**)&mem, bytes) != hipSuccess) {
    ctx_release(ctx, bytes);
    return IPFP_EBUDGET;
  }
  float* out = reinterpret_cast<float*>(mem);
  const float4v* buf =
      reinterpret_cast<const float4v*>(mem + align_up(nout * sizeof(float), 256));
  const int iters = (int)std::min<int64_t>(work, INT32_MAX);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = IPFP_OK;
  auto launch = [&]() {
    switch (kind) {
      case IPFP_PROBE_EXP2:
        hipLaunchKernelGGL(k_probe_exp2, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, iters, out);
        break;
      case IPFP_PROBE_MFMA_BF16:
        hipLaunchKernelGGL(k_probe_mfma<0>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, iters, out);
        break;
      case IPFP_PROBE_MFMA_FP8:
        hipLaunchKernelGGL(k_probe_mfma<1>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, iters, out);
        break;
      case IPFP_PROBE_MFMA_F32:
        hipLaunchKernelGGL(k_probe_mfma<2>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, iters, out);
        break;
      case IPFP_PROBE_MFMA_BF16_2W:
        hipLaunchKernelGGL((k_probe_mix<0, 0>), dim3(kMixBlocks), dim3(kProbeThreads), kMixLds, s,
                           iters, out);
        break;
      case IPFP_PROBE_MFMA_BF16_EPI:
        hipLaunchKernelGGL((k_probe_mix<0, 2>), dim3(kMixBlocks), dim3(kProbeThreads), kMixLds, s,
                           iters, out);
        break;
      case IPFP_PROBE_MFMA_FP8_EPI:
        hipLaunchKernelGGL((k_probe_mix<1, 8>), dim3(kMixBlocks), dim3(kProbeThreads), kMixLds, s,
                           iters, out);
        break;
      default:
        hipLaunchKernelGGL(k_probe_read, dim3(kProbeBlocks), dim3(kProbeThreads), 0, s, buf,
                           work / 16, out);
        break;
    }
    return hipGetLastError();
  };
  float ms = 0.f;
  if ((read && launch_zero(const_cast<float4v*>(buf), (size_t)work, s) != hipSuccess) ||
      launch() != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess || hipEventRecord(e0, s) != hipSuccess ||
      launch() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
      hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
    rc = IPFP_EHIP;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(mem);
  ctx_release(ctx, bytes);
  if (rc != IPFP_OK) return rc;
  const double waves = (double)kProbeBlocks * (kProbeThreads / 64);
  double units = 0.0;   // results, flops or bytes of one launch
  switch (kind) {
    case IPFP_PROBE_EXP2: units = (double)nout * 8.0 * iters; break;
    case IPFP_PROBE_MFMA_BF16: units = waves * 4.0 * iters * (2.0 * 32 * 32 * 16); break;
    case IPFP_PROBE_MFMA_FP8: units = waves * 4.0 * iters * (2.0 * 32 * 32 * 64); break;
    case IPFP_PROBE_MFMA_F32: units = waves * 4.0 * iters * (2.0 * 32 * 32 * 2); break;
    case IPFP_PROBE_MFMA_BF16_2W:
    case IPFP_PROBE_MFMA_BF16_EPI:
      units = (double)kMixBlocks * (kProbeThreads / 64) * 2.0 * iters * (2.0 * 32 * 32 * 16);
      break;
    case IPFP_PROBE_MFMA_FP8_EPI:
      units = (double)kMixBlocks * (kProbeThreads / 64) * 2.0 * iters * (2.0 * 32 * 32 * 64);
      break;
    default: units = (double)work; break;
  }
  *rate_out = units / (ms * 1e-3);
  if (ms_out) *ms_out = ms;
  return IPFP_OK;
}
