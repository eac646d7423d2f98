// zgemmb.h -- large-tile complex GEMM on the BF16 matrix cores with operand
// splitting (precision form, split-BF16 variant).
//
// Each complex64 operand element x (real and imaginary part separately) is
// split into hi = bf16(x) and lo = bf16(x - hi); a real product is
// accumulated in FP32 as  hi*hi + hi*lo + lo*hi  (the lo*lo term, of relative
// size 2^-16, is dropped).  A complex product uses four real products, so
// twelve v_mfma_f32_16x16x32_bf16 per 16x16 block and 32-k step.
//
// The operands are split once, outside the GEMM, into a blocked layout that
// is exactly the LDS tile (split_block_offset): for every 128-row tile and
// 32-k chunk a 32 KB block of four planes (re hi, re lo, im hi, im lo) of
// [128 rows][32 k] bf16, the 16-byte k-groups of a row permuted (kgrp),
// rows and k zero-padded to whole tiles.
//
// 128 x 128 output tile per 512-thread workgroup of two roles.  Waves 0-3
// (consumers) hold 64 x 64 of the tile each (4 x 4 blocks of 16 x 16) and
// only read LDS fragments and issue MFMAs; waves 4-7 (producers) copy the
// operand blocks into LDS with 16-byte loads and stores.  With two waves per
// SIMD the producers' memory work runs beside the consumers' matrix work.
// Two LDS buffers: while the consumers multiply chunk c, the producers store
// chunk c+1 and load chunk c+3 (two chunks of global loads in flight in
// registers); one barrier per chunk.
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


// Position of element (k, row) of plane p in the blocked split layout, in
// bf16 units; nkc = number of 32-k chunks (K padded).
__host__ __device__ inline long split_block_offset(int row, int k, int p, int nkc) {
  const int rt = row / BT, r = row % BT, kc = k / BKB, kk = k % BKB;
  return (((long)rt * nkc + kc) * 4 + p) * (BT * BLDB) + (long)r * BLDB + 8 * ((kk >> 3) ^ ((r >> 1) & 3)) + (kk & 7);
}

// round-to-nearest-even split of 8 floats into bf16 hi and lo parts
__device__ __forceinline__ void split8(const float (&x)[8], bf8& hi, bf8& lo) {
#pragma unroll
  for (int v = 0; v < 8; v += 2) {
    const fv2 xv = {x[v], x[v + 1]};
    const bv2 h = __builtin_convertvector(xv, bv2);
    const fv2 hf = __builtin_convertvector(h, fv2);
    const bv2 l = __builtin_convertvector(xv - hf, bv2);
    hi[v] = h[0];
    hi[v + 1] = h[1];
    lo[v] = l[0];
    lo[v + 1] = l[1];
  }
}

// Blocked split operand.  A chunk of one 128-row tile is 32 KB contiguous
// (2048 16-byte segments, the LDS tile byte for byte); producer thread t
// (0..255) moves segments t + 256 v, v = 0..7.
constexpr int BLOCK_BYTES = 4 * BT * BLDB * 2;
struct SrcBL {
  const char* base;   // the operand's blocked array
  int nkc;            // chunks per row tile
  const char* tbase;  // this workgroup's row tile
  int ptid;
  typedef u4 Reg[8];
  __device__ __forceinline__ void begin(int t, int i0) {
    tbase = base + (long)(i0 / BT) * nkc * BLOCK_BYTES;
    ptid = t;
  }
  __device__ __forceinline__ void load(int kc, Reg& r) const {
    // raw buffer loads: the chunk's block in the descriptor, the lane's
    // segment in the VGPR offset
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)(tbase + (long)kc * BLOCK_BYTES), 0, BLOCK_BYTES, 0x00020000);
#pragma unroll
    for (int v = 0; v < 8; ++v)
      r[v] = __builtin_bit_cast(u4, __builtin_amdgcn_raw_buffer_load_b128(rs, (ptid + 256 * v) * 16, 0, 0));
  }
  __device__ __forceinline__ void stash(__bf16 (*pl)[BT][BLDB], const Reg& r) const {
    char* dst = (char*)&pl[0][0][0];
#pragma unroll
    for (int v = 0; v < 8; ++v) *(u4*)(dst + (ptid + 256 * v) * 16) = r[v];
  }
};

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
    // producers: chunk c+1 is stored while chunks c+2 and c+3 are in flight
    // in two register sets (set = chunk parity relative to kc0).  Chunk
    // indices past kc1-1 are clamped to it: the extra loads and the store into
    // the buffer nobody reads after the last chunk keep the loop branch-free.
    const int kl = kc1 - 1;
    typename SA::Reg ra0, ra1;
    typename SB::Reg rb0, rb1;
    A.load(kc0, ra0);
    B.load(kc0, rb0);
    A.load(min(kc0 + 1, kl), ra1);
    B.load(min(kc0 + 1, kl), rb1);
    A.stash(s[0].a, ra0);
    B.stash(s[0].b, rb0);
    A.load(min(kc0 + 2, kl), ra0);
    B.load(min(kc0 + 2, kl), rb0);
    lds_barrier();
    auto step = [&](int c, typename SA::Reg& ra, typename SB::Reg& rb, int buf) {
      __builtin_amdgcn_sched_barrier(0);   // keep this chunk's stores below the previous barrier
      A.stash(s[buf].a, ra);
      B.stash(s[buf].b, rb);
      A.load(min(c + 3, kl), ra);
      B.load(min(c + 3, kl), rb);
      lds_barrier();
    };
    int c = kc0;
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
