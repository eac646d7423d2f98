// zgemm.h -- large-tile complex FP64 GEMM engines for gfx950.
//
// C[i][j] = sum_k A(k, i) B(k, j) over a 128 x 128 complex output tile per
// workgroup (256 threads = 4 waves, each wave a 64 x 64 quadrant made of
// 4 x 4 blocks of v_mfma_f64_16x16x4_f64, real and imaginary accumulators
// kept in the accumulation registers).  Compared with a 64 x 64 tile this
// halves the operand bytes per MFMA, so the sigma contractions stay
// matrix-bound with one wave per SIMD.  Operands stream through LDS in
// chunks of 16 complex k-values; the next chunk's global loads are issued
// into registers before the current chunk's MFMAs.
//
// Variants below: the same tile on eight waves of 64 x 32 (wide_*, two
// waves per SIMD; the sigma's default), 128 x 64 tiles at two workgroups per
// CU (mid_*), and the three-multiplication 128 x 64 engine (big_*3).
//
// A source provides
//   static constexpr int MAP;                      // KMAJOR or RMAJOR (tile.h)
//   void begin(int tid, int i0);                   // once per tile: row bases
//   void load(int kchunk, Regs8& r) const;         // 8 elements of a [16][128] chunk
// and decides element (k, i) of chunk kchunk for the 8 slots of thread tid
// with the same maps as tile.h, extended to 8 slots (i = base + 16*e).
#pragma once
#include "tile.h"

namespace adc2 {

constexpr int BT = 128;          // tile edge (rows and columns)
constexpr int BK = 16;           // complex k per chunk
constexpr int BLDP = BT + 1;     // padded LDS row (doubles): odd stride, no bank conflicts

struct BigSmem {
  double a_re[BK][BLDP];
  double a_im[BK][BLDP];
  double b_re[BK][BLDP];
  double b_im[BK][BLDP];
};

template <int N>
struct RegsN {
  double2 v[N];
};
using Regs8 = RegsN<8>;
using Regs4 = RegsN<4>;

template <int MAP>
__device__ __forceinline__ void big_coords(int tid, int e, int& kk, int& ii) {
  if (MAP == KMAJOR) {
    kk = tid >> 4;
    ii = (tid & 15) + 16 * e;
  } else {
    kk = tid & 15;
    ii = (tid >> 4) + 16 * e;
  }
}

template <int MAP>
__device__ __forceinline__ void big_stash(double (*re)[BLDP], double (*im)[BLDP], const Regs8& r, int tid) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    int kk, ii;
    big_coords<MAP>(tid, e, kk, ii);
    re[kk][ii] = r.v[e].x;
    im[kk][ii] = r.v[e].y;
  }
}

struct BigAcc {
  d4 re[4][4];
  d4 im[4][4];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        re[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        im[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      }
  }
};

__device__ __forceinline__ void big_mma(const BigSmem& s, BigAcc& acc, int wr, int wc, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kg = 0; kg < BK; kg += 4) {
    double ar[4], ai[4], br[4], bi[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ar[t] = s.a_re[kg + lk][wr + 16 * t + li];
      ai[t] = s.a_im[kg + lk][wr + 16 * t + li];
      br[t] = s.b_re[kg + lk][wc + 16 * t + li];
      bi[t] = s.b_im[kg + lk][wc + 16 * t + li];
    }
    double nai[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) nai[t] = -ai[t];
    // four passes of 16 independent MFMAs each, so consecutive MFMAs never
    // feed the same accumulator
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], acc.re[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], acc.im[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[a], bi[b], acc.re[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], acc.im[a][b], 0, 0, 0);
  }
}

// Double-buffered main loop: stage (c & 1) holds chunk c.  In iteration c
// the registers holding chunk c+1 are written into the other stage (whose
// previous contents were consumed in iteration c-1, fenced by the barrier
// that closed it), the global loads of chunk c+2 are issued, and the MFMAs
// of chunk c run; one barrier per chunk.
template <class SA, class SB>
__device__ __forceinline__ void big_mainloop(BigSmem (&s)[2], const SA& A, const SB& B, int kc0, int kc1,
                                             BigAcc& acc) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  if (kc0 >= kc1) return;
  Regs8 ra, rb;
  A.load(kc0, ra);
  B.load(kc0, rb);
  big_stash<SA::MAP>(s[0].a_re, s[0].a_im, ra, tid);
  big_stash<SB::MAP>(s[0].b_re, s[0].b_im, rb, tid);
  if (kc0 + 1 < kc1) {
    A.load(kc0 + 1, ra);
    B.load(kc0 + 1, rb);
  }
  __syncthreads();
  for (int c = kc0; c < kc1; ++c) {
    const int cur = (c - kc0) & 1;
    if (c + 1 < kc1) {
      big_stash<SA::MAP>(s[cur ^ 1].a_re, s[cur ^ 1].a_im, ra, tid);
      big_stash<SB::MAP>(s[cur ^ 1].b_re, s[cur ^ 1].b_im, rb, tid);
      if (c + 2 < kc1) {
        A.load(c + 2, ra);
        B.load(c + 2, rb);
      }
    }
    big_mma(s[cur], acc, wr, wc, lane);
    __syncthreads();
  }
}

template <class F>
__device__ __forceinline__ void big_for_each(const BigAcc& acc, F&& f) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr + 16 * a + (lane >> 4) + 4 * r;
        const int col = wc + 16 * b + (lane & 15);
        f(row, col, make_double2(acc.re[a][b][r], acc.im[a][b][r]));
      }
}

// Tile order: groups of GROUP_M row-tiles sweep all column tiles, so the
// row panels of A stay in L2 while B streams; consecutive tiles land on the
// same XCD through xcd_remap.
__device__ __forceinline__ void big_tile_coords(long lid, int nbm, int nbn, int& bm, int& bn) {
  const int GROUP_M = 8;
  const long per_group = (long)GROUP_M * nbn;
  const int g = (int)(lid / per_group);
  const int first = g * GROUP_M;
  const int gsize = min(GROUP_M, nbm - first);
  const int r = (int)(lid % per_group);
  bm = first + r % gsize;
  bn = r / gsize;
}


// ---------------------------------------------------------------------------
// Two-per-CU variant: 128 x 64 complex output tile per workgroup (4 waves as
// 2 x 2, each a 64 x 32 quadrant of 4 x 2 blocks), chunks of 8 complex k.
// The accumulators take 128 registers and the double-buffered LDS 48.5 KB,
// so two workgroups share a CU and one's barrier and chunk turn-over run
// under the other's MFMAs.  Each accumulator receives the same MFMAs in the
// same k order as in the 128 x 128 engine, so the results are identical.
// Sources: SrcGroupedK8<NS> (k-major, 8 k-rows per chunk, NS = rows / 32).
// ---------------------------------------------------------------------------
constexpr int MBK = 8;            // complex k per chunk
constexpr int MTN = 64;           // tile columns
constexpr int MLDN = MTN + 1;

struct MidSmem {
  double a_re[MBK][BLDP];
  double a_im[MBK][BLDP];
  double b_re[MBK][MLDN];
  double b_im[MBK][MLDN];
};

// thread -> (k, i) of a k-major [8][32 NS] chunk: 32 consecutive lanes read
// 32 consecutive i of one k row
template <int NS, int LD>
__device__ __forceinline__ void mid_stash(double (*re)[LD], double (*im)[LD], const RegsN<NS>& r, int tid) {
  const int kk = tid >> 5, i0 = tid & 31;
#pragma unroll
  for (int e = 0; e < NS; ++e) {
    re[kk][i0 + 32 * e] = r.v[e].x;
    im[kk][i0 + 32 * e] = r.v[e].y;
  }
}

struct MidAcc {
  d4 re[4][2];
  d4 im[4][2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        re[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        im[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      }
  }
};

__device__ __forceinline__ void mid_mma(const MidSmem& s, MidAcc& acc, int wr, int wc, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kg = 0; kg < MBK; kg += 4) {
    double ar[4], ai[4], br[2], bi[2];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ar[t] = s.a_re[kg + lk][wr + 16 * t + li];
      ai[t] = s.a_im[kg + lk][wr + 16 * t + li];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      br[t] = s.b_re[kg + lk][wc + 16 * t + li];
      bi[t] = s.b_im[kg + lk][wc + 16 * t + li];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], acc.re[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], acc.im[a][b], 0, 0, 0);
    // -Im(A) Im(B): the negation is the MFMA's own modifier on A (blgp bit 0)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], acc.re[a][b], 0, 0, 1);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], acc.im[a][b], 0, 0, 0);
  }
}

// Double-buffered main loop over chunks [kc0, kc1), as big_mainloop.
template <class SA, class SB>
__device__ __forceinline__ void mid_mainloop(MidSmem (&s)[2], const SA& A, const SB& B, int kc0, int kc1,
                                             MidAcc& acc) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 32;
  if (kc0 >= kc1) return;
  RegsN<4> ra;
  RegsN<2> rb;
  A.load(kc0, ra);
  B.load(kc0, rb);
  mid_stash<4, BLDP>(s[0].a_re, s[0].a_im, ra, tid);
  mid_stash<2, MLDN>(s[0].b_re, s[0].b_im, rb, tid);
  if (kc0 + 1 < kc1) {
    A.load(kc0 + 1, ra);
    B.load(kc0 + 1, rb);
  }
  __syncthreads();
  for (int c = kc0; c < kc1; ++c) {
    const int cur = (c - kc0) & 1;
    if (c + 1 < kc1) {
      mid_stash<4, BLDP>(s[cur ^ 1].a_re, s[cur ^ 1].a_im, ra, tid);
      mid_stash<2, MLDN>(s[cur ^ 1].b_re, s[cur ^ 1].b_im, rb, tid);
      if (c + 2 < kc1) {
        A.load(c + 2, ra);
        B.load(c + 2, rb);
      }
    }
    mid_mma(s[cur], acc, wr, wc, lane);
    __syncthreads();
  }
}

template <class F>
__device__ __forceinline__ void mid_for_each(const MidAcc& acc, F&& f) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 32;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr + 16 * a + (lane >> 4) + 4 * r;
        const int col = wc + 16 * b + (lane & 15);
        f(row, col, make_double2(acc.re[a][b][r], acc.im[a][b][r]));
      }
}

// k-major source for the two-per-CU and eight-wave engines: rows grouped as
// SrcGroupedK, element (k, i) at base[g*gstride + a + k*ld], chunks of CK k,
// thread tid reads k = tid / 32 of the chunk and rows (tid % 32) + 32 e,
// NS = rows / 32 (CK * 32 threads).
template <int NS, int CK = MBK>
struct SrcGroupedK8 {
  const double2* base;
  long gstride;
  long ld;
  int inner, nrows, nk;
  long off[NS];
  unsigned okmask;
  int kk;
  __device__ __forceinline__ void begin(int tid, int i0) {
    kk = tid >> 5;
    okmask = 0;
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      const int i = i0 + (tid & 31) + 32 * e;
      const int g = i / inner;
      off[e] = (long)g * gstride + (i - g * inner);
      if (i < nrows) okmask |= 1u << e;
    }
  }
  __device__ __forceinline__ void load(int kc, RegsN<NS>& r) const {
    const int k = kc * CK + kk;
    const long ko = (long)k * ld;
#pragma unroll
    for (int e = 0; e < NS; ++e) r.v[e] = ((okmask >> e) & 1u) && k < nk ? base[off[e] + ko] : czero();
  }
};

// ---------------------------------------------------------------------------
// Eight-wave variant: the 128 x 128 tile and 16-k chunks of the big engine
// (BigSmem, 132 KB) computed by 512 threads, each wave a 64 x 32 quadrant
// (waves as 2 x 4), so two waves share each SIMD with 128 accumulation
// registers each.  Same MFMAs per accumulator in the same k order as the
// other engines.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wide_mma(const BigSmem& s, MidAcc& acc, int wr, int wc, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kg = 0; kg < BK; kg += 4) {
    double ar[4], ai[4], br[2], bi[2];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ar[t] = s.a_re[kg + lk][wr + 16 * t + li];
      ai[t] = s.a_im[kg + lk][wr + 16 * t + li];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      br[t] = s.b_re[kg + lk][wc + 16 * t + li];
      bi[t] = s.b_im[kg + lk][wc + 16 * t + li];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], acc.re[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], acc.im[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], acc.re[a][b], 0, 0, 1);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], acc.im[a][b], 0, 0, 0);
  }
}

template <class SA, class SB>
__device__ __forceinline__ void wide_mainloop(BigSmem (&s)[2], const SA& A, const SB& B, int kc0, int kc1,
                                              MidAcc& acc) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 2) * 64, wc = (w & 3) * 32;
  if (kc0 >= kc1) return;
  RegsN<4> ra, rb;
  A.load(kc0, ra);
  B.load(kc0, rb);
  mid_stash<4, BLDP>(s[0].a_re, s[0].a_im, ra, tid);
  mid_stash<4, BLDP>(s[0].b_re, s[0].b_im, rb, tid);
  if (kc0 + 1 < kc1) {
    A.load(kc0 + 1, ra);
    B.load(kc0 + 1, rb);
  }
  __syncthreads();
  for (int c = kc0; c < kc1; ++c) {
    const int cur = (c - kc0) & 1;
    if (c + 1 < kc1) {
      mid_stash<4, BLDP>(s[cur ^ 1].a_re, s[cur ^ 1].a_im, ra, tid);
      mid_stash<4, BLDP>(s[cur ^ 1].b_re, s[cur ^ 1].b_im, rb, tid);
      if (c + 2 < kc1) {
        A.load(c + 2, ra);
        B.load(c + 2, rb);
      }
    }
    wide_mma(s[cur], acc, wr, wc, lane);
    __syncthreads();
  }
}

template <class F>
__device__ __forceinline__ void wide_for_each(const MidAcc& acc, F&& f) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 2) * 64, wc = (w & 3) * 32;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr + 16 * a + (lane >> 4) + 4 * r;
        const int col = wc + 16 * b + (lane & 15);
        f(row, col, make_double2(acc.re[a][b][r], acc.im[a][b][r]));
      }
}
// ---------------------------------------------------------------------------
// Three-multiplication variant (Gauss): for each 16x16 block
//   T1 += Ar Br,  T2 += Ai Bi,  T3 += (Ar + Ai)(Br + Bi)
//   Re = T1 - T2,  Im = T3 - T1 - T2
// 3 real MFMAs per complex block product instead of 4.  Three accumulator
// sets need 192 accumulation registers for a 64 x 32 wave tile, so the
// workgroup tile is 128 x 64 (4 waves as 2 x 2).
// ---------------------------------------------------------------------------
// Large-tile sources.  Rows of a K-major operand are grouped: row i = (g, a)
// with a < inner, element (k, i) at base[g*gstride + a + k*ld].
// ---------------------------------------------------------------------------
template <int NS>
struct SrcGroupedK {
  static constexpr int MAP = KMAJOR;
  const double2* base;
  long gstride;
  long ld;
  int inner, nrows, nk;
  long off[NS];
  unsigned okmask;
  int kk;
  __device__ __forceinline__ void begin(int tid, int i0) {
    kk = tid >> 4;
    okmask = 0;
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      const int i = i0 + (tid & 15) + 16 * e;
      const int g = i / inner;
      off[e] = (long)g * gstride + (i - g * inner);
      if (i < nrows) okmask |= 1u << e;
    }
  }
  __device__ __forceinline__ void load(int kc, RegsN<NS>& r) const {
    const int k = kc * BK + kk;
    const long ko = (long)k * ld;
#pragma unroll
    for (int e = 0; e < NS; ++e) r.v[e] = ((okmask >> e) & 1u) && k < nk ? base[off[e] + ko] : czero();
  }
};

// ---------------------------------------------------------------------------
constexpr int BT3N = 64;
constexpr int B3LDP = BT3N + 1;

struct BigSmem3 {
  double a_re[BK][BLDP];
  double a_im[BK][BLDP];
  double b_re[BK][B3LDP];
  double b_im[BK][B3LDP];
};

template <int MAP>
__device__ __forceinline__ void coords4(int tid, int e, int& kk, int& ii) {
  if (MAP == KMAJOR) {
    kk = tid >> 4;
    ii = (tid & 15) + 16 * e;
  } else {
    kk = tid & 15;
    ii = (tid >> 4) + 16 * e;
  }
}

template <int MAP>
__device__ __forceinline__ void stash4(double (*re)[B3LDP], double (*im)[B3LDP], const Regs4& r, int tid) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int kk, ii;
    coords4<MAP>(tid, e, kk, ii);
    re[kk][ii] = r.v[e].x;
    im[kk][ii] = r.v[e].y;
  }
}

struct BigAcc3 {
  d4 t1[4][2];
  d4 t2[4][2];
  d4 t3[4][2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        t1[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        t2[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        t3[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      }
  }
};

__device__ __forceinline__ void big_mma3(const BigSmem3& s, BigAcc3& acc, int wr, int wc, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kg = 0; kg < BK; kg += 4) {
    double ar[4], ai[4], as[4], br[2], bi[2], bs[2];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ar[t] = s.a_re[kg + lk][wr + 16 * t + li];
      ai[t] = s.a_im[kg + lk][wr + 16 * t + li];
      as[t] = ar[t] + ai[t];
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      br[t] = s.b_re[kg + lk][wc + 16 * t + li];
      bi[t] = s.b_im[kg + lk][wc + 16 * t + li];
      bs[t] = br[t] + bi[t];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.t1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], acc.t1[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.t2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], acc.t2[a][b], 0, 0, 0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc.t3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[a], bs[b], acc.t3[a][b], 0, 0, 0);
  }
}

template <class SA, class SB>
__device__ __forceinline__ void big_mainloop3(BigSmem3& s, const SA& A, const SB& B, int kc0, int kc1,
                                              BigAcc3& acc) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 32;
  if (kc0 >= kc1) return;
  Regs8 ra;
  Regs4 rb;
  A.load(kc0, ra);
  B.load(kc0, rb);
  for (int c = kc0; c < kc1; ++c) {
    __syncthreads();
    big_stash<SA::MAP>(s.a_re, s.a_im, ra, tid);
    stash4<SB::MAP>(s.b_re, s.b_im, rb, tid);
    __syncthreads();
    if (c + 1 < kc1) {
      A.load(c + 1, ra);
      B.load(c + 1, rb);
    }
    big_mma3(s, acc, wr, wc, lane);
  }
}

template <class F>
__device__ __forceinline__ void big_for_each3(const BigAcc3& acc, F&& f) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 32;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = wr + 16 * a + (lane >> 4) + 4 * r;
        const int col = wc + 16 * b + (lane & 15);
        const double t1 = acc.t1[a][b][r], t2 = acc.t2[a][b][r], t3 = acc.t3[a][b][r];
        f(row, col, make_double2(t1 - t2, t3 - t1 - t2));
      }
}

}  // namespace adc2
