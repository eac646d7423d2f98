// peaks.hip -- microbenchmarks of the device rates the rooflines are quoted
// against: dense MFMA throughput of the three instructions the sigma GEMMs
// issue (FP64 16x16x4, FP32 16x16x4, BF16 16x16x32), with constant and with
// pseudo-random operands, FP64 vector FMA (the Chebyshev moment kernel), and
// HBM streaming read and copy bandwidth.
//
// MFMA and FMA probes keep CH independent accumulator chains per wave, so
// that issue rate, not latency, bounds them, and touch memory only to store
// one value per lane at the end.  HBM probes stream 16-byte loads (and
// stores) over buffers far larger than the L2 and last-level caches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.h"

namespace adc2 {
namespace {

typedef double pd4 __attribute__((ext_vector_type(4)));
typedef float pf4 __attribute__((ext_vector_type(4)));
typedef __bf16 pb8 __attribute__((ext_vector_type(8)));
typedef unsigned int pu4 __attribute__((ext_vector_type(4)));

// Independent accumulator chains.  The counts are those for which the loops
// compile to back-to-back MFMAs with no register copies (the BF16 loop with 8
// chains does not).
constexpr int CH = 8;
constexpr int CHB = 16;          // BF16 probe
constexpr int PGRID = 2048;      // workgroups of 256 (32 waves per CU)

__global__ __launch_bounds__(256) void k_peak_mfma_f64(double a, double b, int iters, double* __restrict__ out) {
  // the first product initialises the accumulators, so that every value the
  // loop carries comes from an MFMA (no register-class copies in the loop)
  pd4 acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, pd4{0.0, 0.0, 0.0, 0.0}, 0, 0, 0);
  for (int it = 1; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// Pseudo-random operands: a 32-bit integer hash of (block, lane, slot) mapped
// to [-1, 1).  The probes below feed each lane its own values and cycle four
// operand registers of each side through the chains, so that consecutive
// MFMAs see different, data-like bit patterns (the constant-operand probes
// above measure the matrix cores at minimal switching activity).
__device__ __forceinline__ float hash_unit(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return (float)(x >> 8) * (1.0f / 8388608.0f) - 1.0f;
}

__global__ __launch_bounds__(256) void k_peak_mfma_f64_rand(int iters, double* __restrict__ out) {
  const unsigned base = (blockIdx.x * 256u + threadIdx.x) * 16u;
  double av[4], bv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    av[q] = (double)hash_unit(base + q) + 1e-9 * hash_unit(base + 8 + q);
    bv[q] = (double)hash_unit(base + 4 + q) + 1e-9 * hash_unit(base + 12 + q);
  }
  pd4 acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c)
    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[c & 3], bv[(c >> 2) & 3], pd4{0.0, 0.0, 0.0, 0.0}, 0, 0, 0);
  for (int it = 1; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c)
      acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[c & 3], bv[(c >> 2) & 3], acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_mfma_bf16_rand(int iters, double* __restrict__ out) {
  const unsigned base = (blockIdx.x * 256u + threadIdx.x) * 64u;
  pb8 av[4], bv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      av[q][i] = (__bf16)hash_unit(base + q * 8 + i);
      bv[q][i] = (__bf16)hash_unit(base + 32 + q * 8 + i);
    }
  pf4 acc[CHB];
#pragma unroll
  for (int c = 0; c < CHB; ++c)
    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[c & 3], bv[(c >> 2) & 3], pf4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  for (int it = 1; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CHB; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[c & 3], bv[(c >> 2) & 3], acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < CHB; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_mfma_f32(float a, float b, int iters, double* __restrict__ out) {
  pf4 acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, pf4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  for (int it = 1; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_mfma_bf16(float a, float b, int iters, double* __restrict__ out) {
  pb8 av, bv;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    av[i] = (__bf16)(a * (float)(i + 1));
    bv[i] = (__bf16)(b * (float)(8 - i));
  }
  pf4 acc[CHB];
#pragma unroll
  for (int c = 0; c < CHB; ++c)
    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, pf4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  for (int it = 1; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CHB; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < CHB; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_fma_f64(double a, double b, int iters, double* __restrict__ out) {
  double x[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) x[c] = (double)(threadIdx.x + c);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) x[c] = __builtin_fma(x[c], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += x[c];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// n16: number of 16-byte words; four independent loads in flight per lane,
// each lane folds what it read into one word
__global__ __launch_bounds__(256) void k_peak_read(const pu4* __restrict__ in, size_t n16, pu4* __restrict__ out) {
  pu4 a0 = pu4{0u, 0u, 0u, 0u}, a1 = a0, a2 = a0, a3 = a0;
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    a0 ^= __builtin_nontemporal_load(in + i);
    a1 ^= __builtin_nontemporal_load(in + i + stride);
    a2 ^= __builtin_nontemporal_load(in + i + 2 * stride);
    a3 ^= __builtin_nontemporal_load(in + i + 3 * stride);
  }
  for (; i < n16; i += stride) a0 ^= in[i];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3;
}

__global__ __launch_bounds__(256) void k_peak_copy(const pu4* __restrict__ in, size_t n16, pu4* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const pu4 v0 = __builtin_nontemporal_load(in + i);
    const pu4 v1 = __builtin_nontemporal_load(in + i + stride);
    const pu4 v2 = __builtin_nontemporal_load(in + i + 2 * stride);
    const pu4 v3 = __builtin_nontemporal_load(in + i + 3 * stride);
    __builtin_nontemporal_store(v0, out + i);
    __builtin_nontemporal_store(v1, out + i + stride);
    __builtin_nontemporal_store(v2, out + i + 2 * stride);
    __builtin_nontemporal_store(v3, out + i + 3 * stride);
  }
  for (; i < n16; i += stride) out[i] = in[i];
}

adc2_status pfail(adc2_status s, const std::string& m) {
  set_error("adc2_peak_probe: " + m);
  return s;
}

}  // namespace
}  // namespace adc2

using namespace adc2;

extern "C" ADC2_API adc2_status adc2_peak_probe(int kind, size_t bytes, int reps, double* rate, void* stream) {
  if (!rate) return pfail(ADC2_ERR_ARG, "rate is NULL");
  *rate = 0.0;
  if (kind < ADC2_PEAK_MFMA_F64 || kind > ADC2_PEAK_MFMA_BF16_RAND) return pfail(ADC2_ERR_ARG, "unknown kind");
  if (reps < 1 || reps > 1000) return pfail(ADC2_ERR_ARG, "reps must be 1..1000");
  const bool hbm = kind == ADC2_PEAK_HBM_READ || kind == ADC2_PEAK_HBM_COPY;
  if (hbm) {
    if (bytes == 0) bytes = (size_t)2 << 30;
    bytes &= ~(size_t)15;
    if (bytes < ((size_t)64 << 20) || bytes > ((size_t)64 << 30))
      return pfail(ADC2_ERR_ARG, "bytes must be 64 MiB .. 64 GiB for the HBM probes");
  }
  hipStream_t st = (hipStream_t)stream;
  // output: one 16-byte word per lane of the grid (also the copy target's size
  // floor); HBM probes add the streamed buffers
  const size_t nout = (size_t)PGRID * 256;
  void* in = nullptr;
  void* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  adc2_status rc = ADC2_OK;
  std::string msg;
  auto check = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && rc == ADC2_OK) {
      rc = e == hipErrorOutOfMemory ? ADC2_ERR_OOM : ADC2_ERR_HIP;
      msg = std::string(what) + ": " + hipGetErrorString(e);
    }
    return rc == ADC2_OK;
  };
  const size_t out_bytes = kind == ADC2_PEAK_HBM_COPY ? bytes : nout * 16;
  if (check(hipMalloc(&out, out_bytes), "hipMalloc") && hbm && check(hipMalloc(&in, bytes), "hipMalloc") &&
      check(hipMemsetAsync(in, 1, bytes, st), "hipMemsetAsync"))
    (void)0;
  if (rc == ADC2_OK) check(hipEventCreate(&e0), "hipEventCreate");
  if (rc == ADC2_OK) check(hipEventCreate(&e1), "hipEventCreate");
  // flops (or bytes) of one launch; iteration counts give launches of ~5-20 ms
  const double waves = (double)PGRID * 4.0;
  int iters = 0;
  double work = 0.0;
  switch (kind) {
    case ADC2_PEAK_MFMA_F64: iters = 4096; work = waves * iters * CH * (16.0 * 16 * 4 * 2); break;
    case ADC2_PEAK_MFMA_F32: iters = 8192; work = waves * iters * CH * (16.0 * 16 * 4 * 2); break;
    case ADC2_PEAK_MFMA_BF16: iters = 8192; work = waves * iters * CHB * (16.0 * 16 * 32 * 2); break;
    case ADC2_PEAK_MFMA_F64_RAND: iters = 4096; work = waves * iters * CH * (16.0 * 16 * 4 * 2); break;
    case ADC2_PEAK_MFMA_BF16_RAND: iters = 8192; work = waves * iters * CHB * (16.0 * 16 * 32 * 2); break;
    case ADC2_PEAK_VALU_F64: iters = 65536; work = waves * 64.0 * iters * CH * 2.0; break;
    case ADC2_PEAK_HBM_READ: work = (double)bytes; break;
    default: work = 2.0 * (double)bytes; break;
  }
  auto launch = [&]() {
    switch (kind) {
      case ADC2_PEAK_MFMA_F64: k_peak_mfma_f64<<<PGRID, 256, 0, st>>>(1.0000001, 0.9999999, iters, (double*)out); break;
      case ADC2_PEAK_MFMA_F32: k_peak_mfma_f32<<<PGRID, 256, 0, st>>>(1.0001f, 0.9999f, iters, (double*)out); break;
      case ADC2_PEAK_MFMA_BF16: k_peak_mfma_bf16<<<PGRID, 256, 0, st>>>(0.01f, 0.02f, iters, (double*)out); break;
      case ADC2_PEAK_MFMA_F64_RAND: k_peak_mfma_f64_rand<<<PGRID, 256, 0, st>>>(iters, (double*)out); break;
      case ADC2_PEAK_MFMA_BF16_RAND: k_peak_mfma_bf16_rand<<<PGRID, 256, 0, st>>>(iters, (double*)out); break;
      case ADC2_PEAK_VALU_F64: k_peak_fma_f64<<<PGRID, 256, 0, st>>>(0.9999999, 1e-7, iters, (double*)out); break;
      case ADC2_PEAK_HBM_READ: k_peak_read<<<PGRID, 256, 0, st>>>((const pu4*)in, bytes / 16, (pu4*)out); break;
      default: k_peak_copy<<<PGRID, 256, 0, st>>>((const pu4*)in, bytes / 16, (pu4*)out); break;
    }
    return check(hipGetLastError(), "launch");
  };
  double best = 0.0;
  if (rc == ADC2_OK && launch() && check(hipStreamSynchronize(st), "hipStreamSynchronize")) {   // warm-up
    for (int r = 0; r < reps && rc == ADC2_OK; ++r) {
      float ms = 0.f;
      if (!check(hipEventRecord(e0, st), "hipEventRecord") || !launch() ||
          !check(hipEventRecord(e1, st), "hipEventRecord") || !check(hipEventSynchronize(e1), "hipEventSynchronize") ||
          !check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime"))
        break;
      if (ms > 0.f) best = std::max(best, work / (ms * 1e-3));
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (in) (void)hipFree(in);
  if (out) (void)hipFree(out);
  if (rc != ADC2_OK) return pfail(rc, msg);
  *rate = hbm ? best * 1e-9 : best * 1e-12;   // GB/s or TFLOP/s
  return ADC2_OK;
}
