// zgemmb.h -- large-tile complex GEMM on the BF16 matrix cores with operand
// splitting (precision form, split-BF16 variant).
//
// Each complex64 operand element x (real and imaginary part separately) is
// split into hi = bf16(x) and lo = bf16(x - hi); a real product is
// accumulated in FP32 as  hi*hi + hi*lo + lo*hi  (the lo*lo term, of relative
// size 2^-16, is dropped).  A complex product uses four real products, so
// twelve v_mfma_f32_16x16x32_bf16 per 16x16 block and 32-k step.
//
// 128 x 128 output tile per 512-thread workgroup of two roles.  Waves 0-3
// (consumers) hold 64 x 64 of the tile each (4 x 4 blocks of 16 x 16) and
// only read LDS fragments and issue MFMAs; waves 4-7 (producers) read the
// K-major complex64 operands (contiguous along the output index), split them
// and store them in LDS as four planes (re hi, re lo, im hi, im lo) of
// [row][k] with k contiguous, so that a consumer lane's fragment (8
// consecutive k of one row) is one 16-byte read.  With two waves per SIMD the
// producers' vector ALU work runs beside the consumers' matrix work.  The
// four 16-byte k-groups of a row are permuted (kgrp) so that the consecutive
// rows one 16-byte read or write instruction touches fall on distinct banks.
// Two LDS buffers: while the consumers multiply chunk
// c, the producers stash chunk c+1 and load chunk c+3 (two chunks of global
// loads in flight in registers); one barrier per chunk.
//
// Fragment layouts of v_mfma_f32_16x16x32_bf16 (checked on the device):
//   A (16x32): lane l holds A[l % 16][8 (l / 16) + v], v = 0..7
//   B (32x16): lane l holds B[8 (l / 16) + v][l % 16]
//   C (16x16): lane l, register r holds C[4 (l / 16) + r][l % 16]
#pragma once
#include "zgemm32.h"

namespace adc2 {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef float fv2 __attribute__((ext_vector_type(2)));   // one complex64 value (re, im)
typedef __bf16 bv2 __attribute__((ext_vector_type(2)));

constexpr int BKB = 32;          // k per chunk (one MFMA step)
constexpr int BLDB = BKB;        // LDS row (bf16 elements, 64 bytes), k-groups swizzled

struct BigSmemB {
  __bf16 a[4][BT][BLDB];   // planes: re hi, re lo, im hi, im lo
  __bf16 b[4][BT][BLDB];
};

// element offset of the 8-wide k-group g (0..3) of a row (64-byte rows).
// XOR with bits 1-2 of the row: measured with the bank-conflict counter, this
// makes both the fragment reads (16 rows x 4 k-groups per instruction) and
// the row-sequential stash writes (64 rows, one k-group) conflict-free, where
// no permutation or XOR with bits 2-3 gives 2- to 4-way conflicts.
__device__ __forceinline__ int kgrp(int row, int g) { return 8 * (g ^ ((row >> 1) & 3)); }

// round-to-nearest-even split of a float into bf16 hi and lo parts
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// K-major complex64 source with grouped rows (row i = (g, x), x < inner,
// element (k, i) at base[g*gstride + x + k*ld]).  Producer thread t (0..255)
// stages row t % 128 of the tile and the 16 k of half t / 128 of the chunk.
// The tile's first group g0 gives a workgroup-uniform base; a lane's row is a
// 32-bit byte offset from it, and 16 k steps also fit in 32 bits (the
// launcher checks both).  Rows past nrows read row nrows-1: they feed only
// output rows or columns that are not written.  k past nk reads as zero.
struct SrcBF {
  const float2* base;
  long gstride;
  long ld;
  int inner, nrows, nk;
  const char* wbase;
  unsigned offb;
  int kh;
  __device__ __forceinline__ void begin(int ptid, int i0) {
    const int g0 = i0 / inner;
    wbase = (const char*)(base + (long)g0 * gstride);
    int i = i0 + (ptid & 127);
    if (i >= nrows) i = nrows - 1;
    const int g = i / inner;
    offb = (unsigned)(((long)(g - g0) * gstride + (i - g * inner)) * (long)sizeof(float2));
    kh = __builtin_amdgcn_readfirstlane(ptid >> 7);
  }
  // FULL: the caller guarantees that the chunk lies below nk (no clamping).
  template <bool FULL = false>
  __device__ __forceinline__ void load(int kc, fv2 (&r)[16]) const {
    // raw buffer loads: uniform row base in the descriptor, lane offset in a
    // VGPR, k step in the scalar offset (no per-load address arithmetic).  In
    // general k is clamped to nk-1 and values past nk are replaced by 0.
    const int k0 = kc * BKB + kh * 16;
    const int kb = FULL ? k0 : min(k0, nk - 1);   // descriptor base row; scalar offsets are >= 0
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(wbase + (long)kb * ld * (long)sizeof(float2)), 0, -1, 0x00020000);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int ee = FULL ? e : min(k0 + e, nk - 1) - kb;
      const fv2 v = __builtin_bit_cast(fv2, __builtin_amdgcn_raw_buffer_load_b64(
                                                rs, (int)offb, (int)(ee * ld * (long)sizeof(float2)), 0));
      r[e] = FULL || k0 + e < nk ? v : (fv2){0.f, 0.f};
    }
  }
};

// split of two floats (consecutive k) into packed bf16 hi and lo pairs
__device__ __forceinline__ void split2(float x0, float x1, bv2& hi, bv2& lo) {
  const fv2 x = {x0, x1};
  hi = __builtin_convertvector(x, bv2);
  const fv2 h = __builtin_convertvector(hi, fv2);
  lo = __builtin_convertvector(x - h, bv2);
}

__device__ __forceinline__ void stash_bf(__bf16 (*pl)[BT][BLDB], const fv2 (&r)[16], int ptid) {
  const int row = ptid & 127, k0 = (ptid >> 7) * 16;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    bf8 rh, rl, ih, il;
#pragma unroll
    for (int v = 0; v < 8; v += 2) {
      bv2 a, b;
      split2(r[8 * h + v].x, r[8 * h + v + 1].x, a, b);
      rh[v] = a[0]; rh[v + 1] = a[1];
      rl[v] = b[0]; rl[v + 1] = b[1];
      split2(r[8 * h + v].y, r[8 * h + v + 1].y, a, b);
      ih[v] = a[0]; ih[v + 1] = a[1];
      il[v] = b[0]; il[v + 1] = b[1];
    }
    const int ko = kgrp(row, (k0 >> 3) + h);
    *(bf8*)&pl[0][row][ko] = rh;
    *(bf8*)&pl[1][row][ko] = rl;
    *(bf8*)&pl[2][row][ko] = ih;
    *(bf8*)&pl[3][row][ko] = il;
  }
}

// sign flip of eight bf16 values (the sign bit of each half-word)
__device__ __forceinline__ bf8 neg_bf8(bf8 x) {
  u4 u = __builtin_bit_cast(u4, x);
  u ^= (u4){0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(bf8, u);
}

__device__ __forceinline__ f4 mfma_b(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// acc += A B for one 32-k chunk held in LDS (consumer waves).  For each of
// the four column blocks, every split product term sweeps the four
// independent row blocks before the next term, so consecutive MFMAs never
// wait on each other's results.
__device__ __forceinline__ void big_mmaB(const BigSmemB& s, BigAccF& acc, int wr, int wc, int lane) {
  const int li = lane & 15, g = lane >> 4;
  bf8 arh[4], arl[4], aih[4], ail[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = wr + 16 * a + li;
    const int ko = kgrp(row, g);
    arh[a] = *(const bf8*)&s.a[0][row][ko];
    arl[a] = *(const bf8*)&s.a[1][row][ko];
    aih[a] = *(const bf8*)&s.a[2][row][ko];
    ail[a] = *(const bf8*)&s.a[3][row][ko];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int col = wc + 16 * q + li;
    const int ko = kgrp(col, g);
    const bf8 brh = *(const bf8*)&s.b[0][col][ko];
    const bf8 brl = *(const bf8*)&s.b[1][col][ko];
    const bf8 bih = *(const bf8*)&s.b[2][col][ko];
    const bf8 bil = *(const bf8*)&s.b[3][col][ko];
    const bf8 nbih = neg_bf8(bih), nbil = neg_bf8(bil);
#define ADC2_SWEEP(ACC, AF, BF) \
  _Pragma("unroll") for (int a = 0; a < 4; ++a) acc.ACC[a][q] = mfma_b(AF[a], BF, acc.ACC[a][q]);
    // re += ar br - ai bi, each real product as hi*hi + hi*lo + lo*hi
    ADC2_SWEEP(re, arh, brh)
    ADC2_SWEEP(re, arh, brl)
    ADC2_SWEEP(re, arl, brh)
    ADC2_SWEEP(re, aih, nbih)
    ADC2_SWEEP(re, aih, nbil)
    ADC2_SWEEP(re, ail, nbih)
    // im += ar bi + ai br
    ADC2_SWEEP(im, arh, bih)
    ADC2_SWEEP(im, arh, bil)
    ADC2_SWEEP(im, arl, bih)
    ADC2_SWEEP(im, aih, brh)
    ADC2_SWEEP(im, aih, brl)
    ADC2_SWEEP(im, ail, brh)
#undef ADC2_SWEEP
  }
}

// Workgroup barrier that orders LDS only: every wave's LDS reads and writes
// before it complete before any wave passes it.  Unlike __syncthreads it does
// not wait for outstanding global loads, which stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Index of the calling wave, uniform across it (0..7 in a 512-thread block).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Main loop over chunks [kc0, kc1) of a 512-thread workgroup: consumers
// (waves 0-3) accumulate into acc, producers (waves 4-7) feed them.  Both
// roles pass the same number of barriers: one before the loop and one per
// chunk.  The role test is on a wave-uniform value, so each wave runs only
// its own branch.
template <class SA, class SB>
__device__ __forceinline__ void big_mainloopB(BigSmemB (&s)[2], const SA& A, const SB& B, int kc0, int kc1,
                                              BigAccF& acc) {
  if (kc0 >= kc1) return;
  const int w = wave_id();
  if (w >= 4) {
    // producers: chunk c+1 is stashed while chunks c+2 and c+3 are in flight
    // in two register sets (set = chunk parity relative to kc0).  Chunk
    // indices past kc1-1 are clamped to it: the extra loads and the stash into
    // the buffer nobody reads after the last chunk keep the loop branch-free.
    const int ptid = threadIdx.x - 256;
    const int kl = kc1 - 1;
    fv2 ra0[16], rb0[16], ra1[16], rb1[16];
    A.load(kc0, ra0);
    B.load(kc0, rb0);
    A.load(min(kc0 + 1, kl), ra1);
    B.load(min(kc0 + 1, kl), rb1);
    stash_bf(s[0].a, ra0, ptid);
    stash_bf(s[0].b, rb0, ptid);
    A.load(min(kc0 + 2, kl), ra0);
    B.load(min(kc0 + 2, kl), rb0);
    lds_barrier();
    auto step = [&](int c, fv2 (&ra)[16], fv2 (&rb)[16], int buf) {
      __builtin_amdgcn_sched_barrier(0);   // keep this split below the previous barrier
      stash_bf(s[buf].a, ra, ptid);
      stash_bf(s[buf].b, rb, ptid);
      A.load(min(c + 3, kl), ra);
      B.load(min(c + 3, kl), rb);
      lds_barrier();
    };
    // steady state: chunks c+3 and c+4 lie below nk in both operands, so the
    // loop body has no branch and two chunks of loads stay in flight
    auto step_full = [&](int c, fv2 (&ra)[16], fv2 (&rb)[16], int buf) {
      __builtin_amdgcn_sched_barrier(0);   // keep this split below the previous barrier
      stash_bf(s[buf].a, ra, ptid);
      stash_bf(s[buf].b, rb, ptid);
      A.template load<true>(c + 3, ra);
      B.template load<true>(c + 3, rb);
      lds_barrier();
    };
    const int kfull = min(kc1, min(A.nk, B.nk) / BKB);   // chunks [0, kfull) lie below nk
    int c = kc0;
    for (; c + 5 <= kfull; c += 2) {
      step_full(c, ra1, rb1, 1);
      step_full(c + 1, ra0, rb0, 0);
    }
    for (; c + 1 < kc1; c += 2) {
      step(c, ra1, rb1, 1);
      step(c + 1, ra0, rb0, 0);
    }
    if (c < kc1) step(c, ra1, rb1, 1);
  } else {
    const int lane = threadIdx.x & 63;
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    lds_barrier();
    for (int c = kc0; c < kc1; ++c) {
      big_mmaB(s[(c - kc0) & 1], acc, wr, wc, lane);
      lds_barrier();
    }
  }
}

}  // namespace adc2
