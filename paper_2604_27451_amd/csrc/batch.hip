// batch.hip -- batching form: several systems of uneven size set up, applied
// and solved together.
//
// Batched sigma: sigma_multi runs every phase of the sigma build for all
// requests before the next phase; the two heavy contractions of the complex64
// and split-BF16 forms are one grouped launch each over the ragged
// (system, K-split, tile) item list (k_sigma.hip).
//
// Batched Davidson: one host thread and one HIP stream per system run the
// ordinary solver.  In rounds mode their sigma requests meet at a rendezvous:
// a request waits until every system still iterating has one pending (or has
// left), then the last arrival runs all pending requests as one sigma_multi
// on the batch stream and releases the others.  In streams mode each solver
// keeps its sigma builds on its own stream.  Every system sees exactly the
// sigma results (and so the iterates) of a solve on its own.
//
// Graph-captured batched sigma: the launch sequence of one batched sigma is
// recorded as a HIP graph (stream capture of sigma_multi, which makes no
// allocation, memset or host synchronisation once the work spaces exist) and
// replayed with one launch.  The graph holds the handles' buffer addresses,
// so a replay first checks that each handle still has the state recorded at
// capture.
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

namespace adc2 {
namespace {

adc2_status bfail(adc2_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

struct Rendezvous {
  std::mutex mu;
  std::condition_variable cv;
  int active = 0;               // systems still iterating
  std::vector<SigReq> pend;     // requests of the current round
  long round = 0;               // completed rounds
  adc2_status status = ADC2_OK; // result of the last round
  std::string msg;
  hipStream_t st = nullptr;

  // Run the pending round (mu held on entry and on return).
  void fire(std::unique_lock<std::mutex>& lk) {
    std::vector<SigReq> reqs;
    reqs.swap(pend);
    lk.unlock();
    adc2_status r = sigma_multi((int)reqs.size(), reqs.data(), st);
    std::string m;
    if (r != ADC2_OK) {
      m = adc2_last_error();
    } else {
      const hipError_t e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        r = ADC2_ERR_HIP;
        m = std::string("batched sigma: ") + hipGetErrorString(e);
      }
    }
    lk.lock();
    status = r;
    msg = m;
    ++round;
    cv.notify_all();
  }

  adc2_status submit(const SigReq& q, hipStream_t own) {
    // the request's input was produced on the system's own stream
    const hipError_t e = hipStreamSynchronize(own);
    if (e != hipSuccess) return bfail(ADC2_ERR_HIP, std::string("batched sigma: ") + hipGetErrorString(e));
    std::unique_lock<std::mutex> lk(mu);
    pend.push_back(q);
    const long my = round;
    if ((int)pend.size() == active)
      fire(lk);
    else
      cv.wait(lk, [&] { return round != my; });
    if (status != ADC2_OK) set_error(msg);
    return status;
  }

  void leave() {
    std::unique_lock<std::mutex> lk(mu);
    --active;
    if (active > 0 && (int)pend.size() == active) fire(lk);
  }
};

// What the captured launch sequence of a handle depends on: its buffer
// addresses and capacities (a work space re-sized to fewer vectors can come
// back at the same address), precision form, method and split counts.
struct SigState {
  int prec, method, zgemm, ysplit, nsplit, ws_m, wsb_m;
  const void* buf[18];
  bool operator==(const SigState& o) const {
    if (prec != o.prec || method != o.method || zgemm != o.zgemm || ysplit != o.ysplit || nsplit != o.nsplit ||
        ws_m != o.ws_m || wsb_m != o.wsb_m)
      return false;
    for (int i = 0; i < 18; ++i)
      if (buf[i] != o.buf[i]) return false;
    return true;
  }
};

SigState sig_state(adc2_handle h) {
  SigState s;
  s.prec = h->prec;
  s.method = h->method;
  s.zgemm = h->zgemm;
  s.ysplit = h->ysplit;
  s.nsplit = h->nsplit;
  s.ws_m = h->ws_m;
  s.wsb_m = h->wsb_m;
  const void* b[18] = {h->X,    h->Y,     h->Zb,  h->Tp,  h->part, h->XB,  h->RB, h->Lv32, h->LvT32,
                       h->LvB,  h->LvTB,  h->LvT, h->Lvo, h->Lvv,  h->Vt,  h->eps, h->M11, nullptr};
  for (int i = 0; i < 18; ++i) s.buf[i] = b[i];
  return s;
}

// Requests of a batched sigma (shared argument checks of the batched entry points).
adc2_status batch_requests(const char* who, int nmol, const adc2_handle* hs, const int* m, const void* const* X,
                           void* const* S, std::vector<SigReq>& rq) {
  if (nmol < 1 || !hs || !m || !X || !S) return bfail(ADC2_ERR_ARG, std::string(who) + ": bad arguments");
  rq.resize(nmol);
  for (int i = 0; i < nmol; ++i) {
    if (!hs[i] || !X[i] || !S[i] || m[i] < 1)
      return bfail(ADC2_ERR_ARG, std::string(who) + ": system " + std::to_string(i) + ": NULL pointer or m < 1");
    if (X[i] == S[i]) return bfail(ADC2_ERR_ARG, std::string(who) + ": S must not alias X");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return bfail(ADC2_ERR_ARG, std::string(who) + ": a handle appears twice");
    rq[i] = SigReq{hs[i], m[i], (const double2*)X[i], (double2*)S[i], SIGMA_SINGLES_IN | SIGMA_DOUBLES_IN};
  }
  return ADC2_OK;
}

}  // namespace
}  // namespace adc2

struct adc2_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<adc2_handle> hs;
  std::vector<adc2::SigState> state;
};

using namespace adc2;

extern "C" {

ADC2_API adc2_status adc2_setup_batch(int nmol, const adc2_mol* mols, int prec, const adc2_alloc* alloc, void* stream,
                                      adc2_handle* out) {
  if (!out) return bfail(ADC2_ERR_ARG, "adc2_setup_batch: out is NULL");
  if (nmol < 1 || nmol > 64) return bfail(ADC2_ERR_ARG, "adc2_setup_batch: nmol must be 1..64");
  for (int i = 0; i < nmol; ++i) out[i] = nullptr;
  if (!mols) return bfail(ADC2_ERR_ARG, "adc2_setup_batch: mols is NULL");
  for (int i = 0; i < nmol; ++i) {
    const adc2_mol& mo = mols[i];
    adc2_status r = adc2_setup(mo.L, mo.eps, mo.nc, mo.no, mo.nv, mo.naux, prec, alloc, stream, &out[i]);
    if (r != ADC2_OK) {
      const std::string m = std::string("adc2_setup_batch: system ") + std::to_string(i) + ": " + adc2_last_error();
      for (int j = 0; j < i; ++j) {
        adc2_destroy(out[j]);
        out[j] = nullptr;
      }
      return bfail(r, m);
    }
  }
  return ADC2_OK;
}

ADC2_API adc2_status adc2_sigma_batch(int nmol, const adc2_handle* hs, const int* m, const void* const* X,
                                      void* const* S, void* stream) {
  std::vector<SigReq> rq;
  const adc2_status rc = batch_requests("adc2_sigma_batch", nmol, hs, m, X, S, rq);
  if (rc != ADC2_OK) return rc;
  return sigma_multi(nmol, rq.data(), (hipStream_t)stream);
}

ADC2_API adc2_status adc2_graph_sigma_batch(int nmol, const adc2_handle* hs, const int* m, const void* const* X,
                                            void* const* S, void* stream, adc2_graph* out) {
  static const char* who = "adc2_graph_sigma_batch";
  if (!out) return bfail(ADC2_ERR_ARG, std::string(who) + ": out is NULL");
  *out = nullptr;
  std::vector<SigReq> rq;
  adc2_status rc = batch_requests(who, nmol, hs, m, X, S, rq);
  if (rc != ADC2_OK) return rc;
  for (int i = 0; i < nmol; ++i)
    if (hs[i]->method != ADC2_METHOD_ADC2)
      return bfail(ADC2_ERR_ARG, std::string(who) + ": system " + std::to_string(i) +
                                     ": only the ADC(2) method is captured (the ADC(2)-x doubles block is not)");
  // eager run: sizes every work space and operand copy, and gives S
  hipStream_t us = (hipStream_t)stream;
  if ((rc = sigma_multi(nmol, rq.data(), us)) != ADC2_OK) return rc;
  {
    const hipError_t e = hipStreamSynchronize(us);
    if (e != hipSuccess) return bfail(ADC2_ERR_HIP, std::string(who) + ": " + hipGetErrorString(e));
  }
  auto* g = new adc2_graph_s;
  g->hs.assign(hs, hs + nmol);
  for (int i = 0; i < nmol; ++i) g->state.push_back(sig_state(hs[i]));
  std::vector<int> prof(nmol);
  for (int i = 0; i < nmol; ++i) {   // profiling records events and synchronises: off while capturing
    prof[i] = hs[i]->profiling;
    hs[i]->profiling = 0;
  }
  hipStream_t cs = nullptr;
  std::string msg;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    rc = ADC2_ERR_HIP;
    msg = std::string("stream capture: ") + hipGetErrorString(e);
  } else {
    rc = sigma_multi(nmol, rq.data(), cs);
    if (rc != ADC2_OK) msg = adc2_last_error();
    e = hipStreamEndCapture(cs, &g->graph);   // ends the capture on every path
    if (rc == ADC2_OK && e != hipSuccess) {
      rc = ADC2_ERR_HIP;
      msg = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
    }
  }
  if (cs) hipStreamDestroy(cs);
  for (int i = 0; i < nmol; ++i) hs[i]->profiling = prof[i];
  for (int i = 0; rc == ADC2_OK && i < nmol; ++i)
    if (!(sig_state(hs[i]) == g->state[i])) {
      rc = ADC2_ERR_HIP;
      msg = "a work space changed while capturing";
    }
  if (rc == ADC2_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      rc = ADC2_ERR_HIP;
      msg = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
    }
  }
  if (rc != ADC2_OK) {
    adc2_graph_destroy(g);
    return bfail(rc, std::string(who) + ": " + msg);
  }
  *out = g;
  return ADC2_OK;
}

ADC2_API adc2_status adc2_graph_launch(adc2_graph g, void* stream) {
  if (!g || !g->exec) return bfail(ADC2_ERR_ARG, "adc2_graph_launch: NULL graph");
  for (size_t i = 0; i < g->hs.size(); ++i)
    if (!(sig_state(g->hs[i]) == g->state[i]))
      return bfail(ADC2_ERR_ARG, "adc2_graph_launch: system " + std::to_string(i) +
                                     ": its work spaces, precision form, method or splits changed since the "
                                     "capture; capture the batch again");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return bfail(ADC2_ERR_HIP, std::string("adc2_graph_launch: ") + hipGetErrorString(e));
  return ADC2_OK;
}

ADC2_API adc2_status adc2_graph_destroy(adc2_graph g) {
  if (!g) return ADC2_OK;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
  return ADC2_OK;
}

ADC2_API adc2_status adc2_davidson_batch(int nmol, const adc2_handle* hs, int nroots, const adc2_dav_opts* opt,
                                         int mode, double* omega, void* const* X, adc2_dav_info* info,
                                         void* stream) {
  if (nmol < 1 || nmol > 64 || !hs || !omega) return bfail(ADC2_ERR_ARG, "adc2_davidson_batch: bad arguments");
  if (mode != ADC2_BATCH_ROUNDS && mode != ADC2_BATCH_STREAMS)
    return bfail(ADC2_ERR_ARG, "adc2_davidson_batch: unknown mode");
  for (int i = 0; i < nmol; ++i) {
    if (!hs[i]) return bfail(ADC2_ERR_ARG, "adc2_davidson_batch: NULL handle");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return bfail(ADC2_ERR_ARG, "adc2_davidson_batch: a handle appears twice");
  }
  hipStream_t st = (hipStream_t)stream;
  {
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bfail(ADC2_ERR_HIP, std::string("adc2_davidson_batch: ") + hipGetErrorString(e));
  }
  std::vector<hipStream_t> own(nmol, nullptr);
  for (int i = 0; i < nmol; ++i) {
    const hipError_t e = hipStreamCreateWithFlags(&own[i], hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) hipStreamDestroy(own[j]);
      return bfail(ADC2_ERR_HIP, std::string("adc2_davidson_batch: hipStreamCreate: ") + hipGetErrorString(e));
    }
  }
  Rendezvous rv;
  rv.active = nmol;
  rv.st = st;
  std::vector<adc2_status> rc(nmol, ADC2_OK);
  std::vector<std::string> msg(nmol);
  if (mode == ADC2_BATCH_ROUNDS)
    for (int i = 0; i < nmol; ++i) {
      adc2_handle h = hs[i];
      hs[i]->sigma_hook = [&rv, h, i, &own](int m, const double2* xin, double2* sout, int parts, hipStream_t) {
        return rv.submit(SigReq{h, m, xin, sout, parts}, own[i]);
      };
    }
  std::vector<std::thread> th;
  th.reserve(nmol);
  for (int i = 0; i < nmol; ++i) {
    try {
      th.emplace_back([&, i]() {
        rc[i] = adc2_davidson(hs[i], nroots, opt, nullptr, omega + (size_t)i * (size_t)std::max(nroots, 0),
                              X ? X[i] : nullptr, info ? &info[i] : nullptr, own[i]);
        if (rc[i] != ADC2_OK) msg[i] = adc2_last_error();
        rv.leave();
      });
    } catch (...) {   // no thread for this system: it never joins the rendezvous
      rc[i] = ADC2_ERR_ARG;
      msg[i] = "could not start a host thread";
      rv.leave();
    }
  }
  for (auto& t : th) t.join();
  for (int i = 0; i < nmol; ++i) {
    hs[i]->sigma_hook = nullptr;
    hipStreamDestroy(own[i]);
  }
  for (int i = 0; i < nmol; ++i)
    if (rc[i] != ADC2_OK) return bfail(rc[i], "adc2_davidson_batch: system " + std::to_string(i) + ": " + msg[i]);
  return ADC2_OK;
}

}  // extern "C"
