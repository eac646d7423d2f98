// zgemm32.h -- large-tile complex FP32 GEMM engine for gfx950 (precision form).
//
// Same structure as the FP64 engine in zgemm.h (128 x 128 complex tile per
// 256-thread workgroup, four waves of 64 x 64, four real products per complex
// block product, double-buffered LDS, one barrier per 16-k chunk), built on
// v_mfma_f32_16x16x4_f32 with FP32 accumulation.  Operands are complex64.
//
// Fragment layouts of v_mfma_f32_16x16x4_f32 (checked on the device):
//   A (16x4): lane l holds A[l % 16][l / 16];  B (4x16): B[l / 16][l % 16]
//   C (16x16): lane l, register r holds C[4 * (l / 16) + r][l % 16]
#pragma once
#include "zgemm.h"

namespace adc2 {

typedef float f4 __attribute__((ext_vector_type(4)));

// Padded LDS row (floats).  A fragment read (and a stash of a K-major
// operand) touches 4 consecutive k rows x 16 consecutive floats per wave; a
// row stride of 16 mod 32 banks puts the four rows on disjoint banks (the
// stride BT + 1 made them overlap: half of the LDS cycles were conflicts).
constexpr int FLDP = BT + 16;

struct BigSmemF {
  float a_re[BK][FLDP];
  float a_im[BK][FLDP];
  float b_re[BK][FLDP];
  float b_im[BK][FLDP];
};

template <int N>
struct RegsF {
  float2 v[N];
};

template <int MAP>
__device__ __forceinline__ void stashF(float (*re)[FLDP], float (*im)[FLDP], const RegsF<8>& r, int tid) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    int kk, ii;
    big_coords<MAP>(tid, e, kk, ii);
    re[kk][ii] = r.v[e].x;
    im[kk][ii] = r.v[e].y;
  }
}

struct BigAccF {
  f4 re[4][4];
  f4 im[4][4];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        re[a][b] = f4{0.f, 0.f, 0.f, 0.f};
        im[a][b] = f4{0.f, 0.f, 0.f, 0.f};
      }
  }
};

__device__ __forceinline__ void big_mmaF(const BigSmemF& s, BigAccF& acc, int wr, int wc, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kg = 0; kg < BK; kg += 4) {
    float ar[4], ai[4], nai[4], br[4], bi[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ar[t] = s.a_re[kg + lk][wr + 16 * t + li];
      ai[t] = s.a_im[kg + lk][wr + 16 * t + li];
      nai[t] = -ai[t];
      br[t] = s.b_re[kg + lk][wc + 16 * t + li];
      bi[t] = s.b_im[kg + lk][wc + 16 * t + li];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc.re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[a], br[b], acc.re[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc.im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[a], bi[b], acc.im[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc.re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai[a], bi[b], acc.re[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc.im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[a], br[b], acc.im[a][b], 0, 0, 0);
  }
}

template <class SA, class SB>
__device__ __forceinline__ void big_mainloopF(BigSmemF (&s)[2], const SA& A, const SB& B, int kc0, int kc1,
                                              BigAccF& acc) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  if (kc0 >= kc1) return;
  RegsF<8> ra, rb;
  A.load(kc0, ra);
  B.load(kc0, rb);
  stashF<SA::MAP>(s[0].a_re, s[0].a_im, ra, tid);
  stashF<SB::MAP>(s[0].b_re, s[0].b_im, rb, tid);
  if (kc0 + 1 < kc1) {
    A.load(kc0 + 1, ra);
    B.load(kc0 + 1, rb);
  }
  __syncthreads();
  for (int c = kc0; c < kc1; ++c) {
    const int cur = (c - kc0) & 1;
    if (c + 1 < kc1) {
      stashF<SA::MAP>(s[cur ^ 1].a_re, s[cur ^ 1].a_im, ra, tid);
      stashF<SB::MAP>(s[cur ^ 1].b_re, s[cur ^ 1].b_im, rb, tid);
      if (c + 2 < kc1) {
        A.load(c + 2, ra);
        B.load(c + 2, rb);
      }
    }
    big_mmaF(s[cur], acc, wr, wc, lane);
    __syncthreads();
  }
}

template <class F>
__device__ __forceinline__ void big_for_eachF(const BigAccF& acc, F&& f) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr + 16 * a + 4 * (lane >> 4) + r;
        const int col = wc + 16 * b + (lane & 15);
        f(row, col, make_float2(acc.re[a][b][r], acc.im[a][b][r]));
      }
}

// K-major grouped-row source over complex64 data (see SrcGroupedK).
struct SrcGroupedKF {
  static constexpr int MAP = KMAJOR;
  const float2* base;
  long gstride;
  long ld;
  int inner, nrows, nk;
  long off[8];
  unsigned okmask;
  int kk;
  __device__ __forceinline__ void begin(int tid, int i0) {
    kk = tid >> 4;
    okmask = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int i = i0 + (tid & 15) + 16 * e;
      const int g = i / inner;
      off[e] = (long)g * gstride + (i - g * inner);
      if (i < nrows) okmask |= 1u << e;
    }
  }
  __device__ __forceinline__ void load(int kc, RegsF<8>& r) const {
    const int k = kc * BK + kk;
    const long ko = (long)k * ld;
#pragma unroll
    for (int e = 0; e < 8; ++e)
      r.v[e] = (((okmask >> e) & 1u) && k < nk) ? base[off[e] + ko] : make_float2(0.f, 0.f);
  }
};

}  // namespace adc2
