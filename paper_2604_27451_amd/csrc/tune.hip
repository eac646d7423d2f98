// tune.hip -- autotuner of the sigma build's dominant GEMM.
//
// The Y-build contracts K = no*nv per output tile; its K-split (partials
// summed afterwards) decides how many workgroups one launch has, against
// the cost of the extra partial traffic and the summation.  In the FP64
// form the tile shape is a choice too: four engines (128 x 128 on eight
// waves, 128 x 64 at two workgroups per CU, 128 x 128 on four waves, 128 x 64
// three-multiplication).  The best
// choice depends on the system's shape, the block size and the precision
// form, so adc2_autotune times the candidates on the device and keeps the
// fastest: first each FP64 engine at its own size-rule K-split, then every
// K-split of the fastest engine.  Choices are cached per (device, shape,
// block size, form) for the process and, if ADC2_TUNE_CACHE names a file,
// across processes (one text line per key, appended after each tuning).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "internal.h"

namespace adc2 {
namespace {

// p[e] = uniform [-1, 1) from a 32-bit hash of (e, seed)
template <class T>
__global__ void k_fill_unit(T* __restrict__ p, size_t n, unsigned seed) {
  for (size_t e = blockIdx.x * 256ul + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    unsigned x = (unsigned)e * 0x9e3779b1u ^ (unsigned)(e >> 32) ^ seed;
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    p[e] = (T)((float)(x >> 8) * (1.0f / 8388608.0f) - 1.0f);
  }
}

unsigned grid_fill(size_t n) { return (unsigned)std::max<size_t>(1, std::min<size_t>(8192, (n + 255) / 256)); }

struct TuneChoice {
  int engine;   // FP64 GEMM engine (ZGEMM_*), -1: the handle's own
  int ysplit;
};
std::mutex tune_mu;
std::map<std::string, TuneChoice> tune_mem;
bool tune_file_read = false;

const int CANDS[] = {1, 2, 3, 4, 6, 8, 12, 16};
constexpr int NCAND = sizeof(CANDS) / sizeof(CANDS[0]);
constexpr double YMAX_BYTES = 8.0 * (1 << 30);   // Y partial workspace limit for the search

// search: the FP64 engine is part of the choice (else the handle's engine is part of the key)
std::string tune_key(adc2_handle h, int m, bool search) {
  int dev = 0;
  hipDeviceProp_t p;
  std::string name = "gpu";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) name = p.gcnArchName;
  for (char& c : name)
    if (c == ' ') c = '_';
  const Dims& d = h->d;
  std::ostringstream k;
  k << name << " nc=" << d.nc << " no=" << d.no << " nv=" << d.nv << " naux=" << d.naux << " m=" << m
    << " prec=" << h->prec << " zgemm=";
  if (search) k << "search";
  else k << h->zgemm;
  return k.str();
}

// file lines: "<key>[ engine=<e>] ysplit=<n>"
void read_cache_file() {
  if (tune_file_read) return;
  tune_file_read = true;
  const char* path = getenv("ADC2_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t p = line.rfind(" ysplit=");
    if (p == std::string::npos) continue;
    const int v = atoi(line.c_str() + p + 8);
    std::string head = line.substr(0, p);
    int e = -1;
    const size_t q = head.rfind(" engine=");
    if (q != std::string::npos) {
      e = atoi(head.c_str() + q + 8);
      head = head.substr(0, q);
    }
    if (v >= 1 && v <= 16 && e >= -1 && e <= ZGEMM_WIDE) tune_mem[head] = TuneChoice{e, v};
  }
}

void append_cache_file(const std::string& key, const TuneChoice& c) {
  const char* path = getenv("ADC2_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  if (!f) return;
  f << key;
  if (c.engine >= 0) f << " engine=" << c.engine;
  f << " ysplit=" << c.ysplit << "\n";
}

adc2_status tfail(adc2_status s, const std::string& m) {
  set_error("adc2_autotune: " + m);
  return s;
}

}  // namespace
}  // namespace adc2

using namespace adc2;

extern "C" ADC2_API adc2_status adc2_autotune(adc2_handle h, int m, adc2_tune_info* info, void* stream) {
  if (!h) return tfail(ADC2_ERR_ARG, "NULL handle");
  if (m < 1 || m > 4096) return tfail(ADC2_ERR_ARG, "m must be 1..4096");
  hipStream_t st = (hipStream_t)stream;
  adc2_tune_info loc;
  adc2_tune_info& I = info ? *info : loc;
  memset(&I, 0, sizeof(I));
  // the FP64 engine is searched unless the environment fixes it
  const bool search = h->prec == ADC2_FP64 && !getenv("ADC2_ZGEMM");
  const std::string key = tune_key(h, m, search);
  {
    std::lock_guard<std::mutex> lk(tune_mu);
    read_cache_file();
    auto it = tune_mem.find(key);
    if (it != tune_mem.end()) {
      if (search && it->second.engine >= 0) h->zgemm = it->second.engine;
      h->ysplit_tuned = it->second.ysplit;
      h->ws_m = 0;   // workspaces are re-sized for this split on the next sigma
      I.ysplit = it->second.ysplit;
      I.zgemm = h->zgemm;
      I.from_cache = 1;
      return ADC2_OK;
    }
  }
  const Dims& d = h->d;
  adc2_status rc;
  if (h->prec != ADC2_FP64 && (rc = build_c64(h, st)) != ADC2_OK) return rc;
  if (h->prec == ADC2_BF16X3 && (rc = build_b3(h, st)) != ADC2_OK) return rc;
  const double ybytes = 16.0 * m * d.nc * (double)d.naux * d.nv;   // one partial of Y
  const long kdim = (long)d.no * d.nv;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ADC2_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return tfail(ADC2_ERR_HIP, "hipEventCreate");
  }
  // best time of the Y-build (and its partial sum) with the handle's current engine at K-split ys
  auto time_ybuild = [&](int ys, double& tmin) -> adc2_status {
    h->ysplit_tuned = ys;
    h->ws_m = 0;
    adc2_status r = ensure_ws(h, m);
    if (r == ADC2_OK && h->prec == ADC2_BF16X3) r = ensure_ws_b3(h, m);
    if (r != ADC2_OK) return r;
    // data-like operands, uniform in [-1, 1): the matrix cores draw more power
    // on them than on zeros, and the power limit can hold the clock lower
    // (the split-BF16 Y-build at nc=6, no=60, nv=300 runs 40% longer on such
    // data than on zeros)
    const size_t nzb = (size_t)2 * m * d.nc * d.no * d.nv * d.nv;   // real values of the doubles
    if (h->prec == ADC2_FP64) k_fill_unit<double><<<grid_fill(nzb), 256, 0, st>>>((double*)h->Zb, nzb, 0x9e3779b9u);
    else k_fill_unit<float><<<grid_fill(nzb), 256, 0, st>>>((float*)h->Zb, nzb, 0x9e3779b9u);
    if (h->prec == ADC2_BF16X3) {
      const size_t nrb = (size_t)split_bytes((long)m * d.nc * d.nv, (long)d.no * d.nv) / 2;   // bf16 values
      k_fill_unit<__bf16><<<grid_fill(nrb), 256, 0, st>>>((__bf16*)h->RB, nrb, 0x85ebca6bu);
    }
    if (hipGetLastError() != hipSuccess) return tfail(ADC2_ERR_HIP, "k_fill_unit");
    tmin = 1e300;
    for (int rep = 0; rep < 4; ++rep) {   // one warm-up, three timed
      if (hipEventRecord(e0, st) != hipSuccess) return tfail(ADC2_ERR_HIP, "hipEventRecord");
      if ((r = ybuild_launch(h, m, st)) != ADC2_OK || (r = ybuild_sum(h, m, st)) != ADC2_OK) return r;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return tfail(ADC2_ERR_HIP, "timing events");
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return tfail(ADC2_ERR_HIP, "hipEventElapsedTime");
      if (rep > 0) tmin = std::min(tmin, (double)ms);
    }
    return ADC2_OK;
  };
  const int saved_ys = h->ysplit_tuned, saved_engine = h->zgemm;
  rc = ADC2_OK;
  // stage 1 (FP64): each engine at its own size-rule K-split
  if (search) {
    const int engines[] = {ZGEMM_WIDE, ZGEMM_MID, ZGEMM_BIG, ZGEMM_3M};
    double best_ms = 1e300;
    int best_e = saved_engine;
    for (int e : engines) {
      h->zgemm = e;
      double t = 0.0;
      if ((rc = time_ybuild(ysplit_rule(h, m), t)) != ADC2_OK) break;
      I.engine[I.nengine] = e;
      I.engine_ms[I.nengine] = t;
      ++I.nengine;
      if (t < best_ms) {
        best_ms = t;
        best_e = e;
      }
    }
    h->zgemm = best_e;
  }
  // stage 2: every K-split of the (chosen) engine
  int best = 0;
  double best_ms = 1e300;
  for (int c = 0; c < NCAND && rc == ADC2_OK; ++c) {
    const int ys = CANDS[c];
    if (ys > 1 && (ys * ybytes > YMAX_BYTES || (long)ys * 64 > kdim)) continue;
    double t = 0.0;
    if ((rc = time_ybuild(ys, t)) != ADC2_OK) break;
    if (I.ncand < 8) {
      I.cand[I.ncand] = ys;
      I.ms[I.ncand] = t;
      ++I.ncand;
    }
    if (t < best_ms) {
      best_ms = t;
      best = ys;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != ADC2_OK || best == 0) {
    h->ysplit_tuned = saved_ys;
    h->zgemm = saved_engine;
    h->ws_m = 0;
    return rc != ADC2_OK ? rc : tfail(ADC2_ERR_ARG, "no K-split candidate fits");
  }
  h->ysplit_tuned = best;
  h->ws_m = 0;   // re-sized for the chosen split on the next sigma
  I.ysplit = best;
  I.zgemm = h->zgemm;
  {
    std::lock_guard<std::mutex> lk(tune_mu);
    const TuneChoice c{search ? h->zgemm : -1, best};
    tune_mem[key] = c;
    append_cache_file(key, c);
  }
  return ADC2_OK;
}
