// tile.h -- complex FP64 MFMA tile engine for gfx950 (CDNA4).
//
// A workgroup of 256 threads (4 waves of 64) owns a 64 x 64 complex output
// tile.  Each wave owns a 32 x 32 quadrant computed as 2 x 2 blocks of the
// 16x16x4 FP64 matrix instruction.  Complex products use four real products
// (re*re - im*im, re*im + im*re) on separate real / imaginary accumulators.
// Operands stream through LDS in chunks of TK complex k-values, stored as
// separate real and imaginary planes [k][i] so that every MFMA fragment read
// is 16 consecutive doubles.  The next chunk's global loads are issued into
// registers before the current chunk's MFMAs, so HBM/L2 latency overlaps the
// matrix work.
//
// Fragment layouts of v_mfma_f64_16x16x4_f64 (checked on the device):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   C (16x16): lane l, register r holds C[(l / 16) + 4 * r][l % 16]
// (the FP32 16x16x4 instruction instead packs rows 4*(l/16)+r).
#pragma once
#include <hip/hip_runtime.h>

namespace adc2 {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64;          // tile rows (i)
constexpr int TN = 64;          // tile columns (j)
constexpr int TK = 16;          // complex k per LDS chunk
constexpr int LDP = TM + 1;     // padded LDS row length in doubles
constexpr int NTHR = 256;

struct TileSmem {
  double a_re[TK][LDP];
  double a_im[TK][LDP];
  double b_re[TK][LDP];
  double b_im[TK][LDP];
};

// Four complex values a thread carries from global memory to LDS.
struct Regs {
  double2 v[4];
};

__device__ __forceinline__ double2 czero() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cneg(double2 a) { return make_double2(-a.x, -a.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// conj(a) * b
__device__ __forceinline__ double2 cdotc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Thread -> element maps for one [TK][64] operand chunk (4 elements/thread).
//  KMAJOR: the source is contiguous along i; 16 consecutive lanes read 16
//          consecutive i of one k row.
//  RMAJOR: the source is contiguous along k; 16 consecutive lanes read the 16
//          k of one row i.
enum MapKind { KMAJOR = 0, RMAJOR = 1 };

template <int MAP>
__device__ __forceinline__ void elem_coords(int tid, int e, int& kk, int& ii) {
  if (MAP == KMAJOR) {
    kk = tid >> 4;
    ii = (tid & 15) + 16 * e;
  } else {
    kk = tid & 15;
    ii = (tid >> 4) + 16 * e;
  }
}

// A source S provides:  static constexpr int MAP;  double2 get(int k, int i) const
// returning the (already conjugated / scaled) element or zero out of range.
template <class S>
__device__ __forceinline__ void fetch(const S& s, int k0, Regs& r, int tid) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int kk, ii;
    elem_coords<S::MAP>(tid, e, kk, ii);
    r.v[e] = s.get(k0 + kk, ii);
  }
}

template <int MAP>
__device__ __forceinline__ void stash(double (*re)[LDP], double (*im)[LDP], const Regs& r, int tid) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int kk, ii;
    elem_coords<MAP>(tid, e, kk, ii);
    re[kk][ii] = r.v[e].x;
    im[kk][ii] = r.v[e].y;
  }
}

struct Acc {
  d4 re[2][2];
  d4 im[2][2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        re[a][b] = d4{0.0, 0.0, 0.0, 0.0};
        im[a][b] = d4{0.0, 0.0, 0.0, 0.0};
      }
  }
};

__device__ __forceinline__ void mma_chunk(const TileSmem& s, Acc& acc, int wr, int wc, int lane) {
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kg = 0; kg < TK; kg += 4) {
    double ar[2], ai[2], br[2], bi[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      ar[t] = s.a_re[kg + lk][wr + 16 * t + li];
      ai[t] = s.a_im[kg + lk][wr + 16 * t + li];
      br[t] = s.b_re[kg + lk][wc + 16 * t + li];
      bi[t] = s.b_im[kg + lk][wc + 16 * t + li];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], acc.re[a][b], 0, 0, 0);
        acc.re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[a], bi[b], acc.re[a][b], 0, 0, 0);
        acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], acc.im[a][b], 0, 0, 0);
        acc.im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], br[b], acc.im[a][b], 0, 0, 0);
      }
  }
}

// C += sum over chunks [kc0, kc1) of A(k, i) B(k, j): A and B are sources
// already positioned at the tile origin (get(k, i) with i in [0, 64)).
template <class SA, class SB>
__device__ __forceinline__ void mainloop(TileSmem& s, const SA& A, const SB& B, int kc0, int kc1, Acc& acc) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  if (kc0 >= kc1) return;
  Regs ra, rb;
  fetch(A, kc0 * TK, ra, tid);
  fetch(B, kc0 * TK, rb, tid);
  for (int c = kc0; c < kc1; ++c) {
    __syncthreads();
    stash<SA::MAP>(s.a_re, s.a_im, ra, tid);
    stash<SB::MAP>(s.b_re, s.b_im, rb, tid);
    __syncthreads();
    if (c + 1 < kc1) {
      fetch(A, (c + 1) * TK, ra, tid);
      fetch(B, (c + 1) * TK, rb, tid);
    }
    mma_chunk(s, acc, wr, wc, lane);
  }
}

// Visit every accumulator element with its tile-local (row, col).
template <class F>
__device__ __forceinline__ void for_each_acc(const Acc& acc, F&& f) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
  for (int a = 0; a < 2; ++a)
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
// Generic sources
// ---------------------------------------------------------------------------
// element (k, i) = op(base[k*ld + i]) for k < nk, i < ni   (contiguous in i)
template <bool CONJ>
struct SrcK {
  static constexpr int MAP = KMAJOR;
  const double2* base;
  long ld;
  int nk, ni;
  double scale;
  __device__ __forceinline__ double2 get(int k, int i) const {
    if (k >= nk || i >= ni) return czero();
    double2 v = base[(long)k * ld + i];
    if (CONJ) v.y = -v.y;
    return make_double2(v.x * scale, v.y * scale);
  }
};

// element (k, i) = op(base[i*ld + k]) for k < nk, i < ni   (contiguous in k)
template <bool CONJ>
struct SrcR {
  static constexpr int MAP = RMAJOR;
  const double2* base;
  long ld;
  int nk, ni;
  double scale;
  __device__ __forceinline__ double2 get(int k, int i) const {
    if (k >= nk || i >= ni) return czero();
    double2 v = base[(long)i * ld + k];
    if (CONJ) v.y = -v.y;
    return make_double2(v.x * scale, v.y * scale);
  }
};

// Two stacked K-major sources: k < k1 from (b1, ld1); k1 <= k < k1+k2 from (b2, ld2).
struct SrcK2 {
  static constexpr int MAP = KMAJOR;
  const double2* b1;
  long ld1;
  int k1;
  const double2* b2;
  long ld2;
  int k2;
  int ni;
  double scale;
  __device__ __forceinline__ double2 get(int k, int i) const {
    if (i >= ni) return czero();
    double2 v;
    if (k < k1) v = b1[(long)k * ld1 + i];
    else if (k < k1 + k2) v = b2[(long)(k - k1) * ld2 + i];
    else return czero();
    return make_double2(v.x * scale, v.y * scale);
  }
};

// Physical workgroup id -> logical tile id so that consecutive logical tiles
// (which share operands) land on the same XCD; the hardware deals workgroups
// to the 8 XCDs round-robin.
__device__ __forceinline__ long xcd_remap(long pid, long nblocks) {
  const long nx = 8;
  const long per = (nblocks + nx - 1) / nx;
  const long x = pid % nx, q = pid / nx;
  const long full = nblocks % nx == 0 ? nx : nblocks % nx;  // XCDs with 'per' blocks
  long lid = (x < full) ? x * per + q : full * per + (x - full) * (per - 1) + q;
  return lid;
}

}  // namespace adc2
