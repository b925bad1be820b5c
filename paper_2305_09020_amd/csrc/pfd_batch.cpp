// Batches of independent contexts (instances of uneven mesh, order and parameters) stepped
// together: one hipGraph per step holds every instance's step, captured as parallel branches
// (the instances are spread over a few capture streams forked from one origin and joined
// again), so one graph launch runs all instances with the branches free to overlap on the
// device.  Instances keep their own workspaces, autotuned kernels and state; the graph only
// orders and groups their launches.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pfd_internal.h"

using namespace pfd;

struct pfd_batch {
  std::vector<pfd_ctx*> ctx;
  hipStream_t stream = nullptr;           // the stream the instances were created on
  hipStream_t cap = nullptr;              // capture origin
  std::vector<hipStream_t> lanes;         // capture branches
  std::vector<hipEvent_t> ev;             // fork event + one join event per lane
  hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  // members' graph generations when each graph was captured: a member whose kernels or
  // kernel arguments changed since (parameters, variants, tuning) makes the graph stale
  std::vector<unsigned long> gen[2][2];
  std::string err;
};

static thread_local std::string g_batch_err;

#define BCHK(x)                                              \
  do {                                                       \
    hipError_t e_ = (x);                                     \
    if (e_ != hipSuccess) {                                  \
      b->err = std::string("HIP error: ") + hipGetErrorString(e_); \
      return PFD_EHIP;                                       \
    }                                                        \
  } while (0)

static void batch_free(pfd_batch* b) {
  for (auto& row : b->gexec)
    for (auto& g : row)
      if (g) (void)hipGraphExecDestroy(g);
  for (auto e : b->ev) (void)hipEventDestroy(e);
  for (auto s : b->lanes) (void)hipStreamDestroy(s);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

extern "C" pfd_status pfd_batch_create(pfd_ctx* const* ctxs, int n, int nlanes, pfd_batch** out) {
  if (!out) return PFD_EINVAL;
  *out = nullptr;
  if (!ctxs || n < 1) { g_batch_err = "need at least one context"; return PFD_EINVAL; }
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) { g_batch_err = "null context"; return PFD_EINVAL; }
    if (ctxs[i]->stream != ctxs[0]->stream) {
      g_batch_err = "the contexts of a batch must share one stream";
      return PFD_EINVAL;
    }
  }
  pfd_batch* b = new pfd_batch;
  b->ctx.assign(ctxs, ctxs + n);
  b->stream = ctxs[0]->stream;
  const int L = std::max(1, std::min(std::min(nlanes < 1 ? 4 : nlanes, n), 16));
  hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  for (int l = 0; l < L && !e; ++l) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (!e) b->lanes.push_back(s);
  }
  for (int l = 0; l <= L && !e; ++l) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (!e) b->ev.push_back(ev);
  }
  if (e) {
    g_batch_err = std::string("HIP error in batch create: ") + hipGetErrorString(e);
    batch_free(b);
    return PFD_EHIP;
  }
  *out = b;
  return PFD_OK;
}

extern "C" void pfd_batch_destroy(pfd_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  batch_free(b);
}

extern "C" const char* pfd_batch_last_error(const pfd_batch* b) {
  return b ? b->err.c_str() : g_batch_err.c_str();
}

static hipError_t eager_step(pfd_ctx* c, int eq) { return c->is3d ? step_once_3d(c, eq) : step_once(c, eq); }

// capture one step of every instance as parallel branches of one graph
static hipError_t capture(pfd_batch* b, int eq, hipGraphExec_t* ex) {
  const int L = (int)b->lanes.size();
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e) return e;
  hipError_t es = hipEventRecord(b->ev[0], b->cap);
  for (int l = 0; l < L && !es; ++l) es = hipStreamWaitEvent(b->lanes[l], b->ev[0], 0);
  for (size_t i = 0; i < b->ctx.size() && !es; ++i) {
    pfd_ctx* c = b->ctx[i];
    const int cur = c->cur;
    hipStream_t own = c->stream;
    c->stream = b->lanes[i % L];
    es = eager_step(c, eq);
    c->stream = own;
    c->cur = cur;
  }
  for (int l = 0; l < L && !es; ++l) {
    es = hipEventRecord(b->ev[l + 1], b->lanes[l]);
    if (!es) es = hipStreamWaitEvent(b->cap, b->ev[l + 1], 0);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (!e) e = es;
  if (!e) e = hipGraphInstantiate(ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e) *ex = nullptr;
  return e;
}

extern "C" pfd_status pfd_batch_step(pfd_batch* b, int nsteps, int equilibrium) {
  if (!b || nsteps < 0) return PFD_EINVAL;
  const int eq = equilibrium ? 1 : 0;
  bool aligned = true, profiling = false;
  for (pfd_ctx* c : b->ctx) {
    if (c->failed) {
      b->err = "an instance failed earlier; set its fields again";
      return PFD_ESTATE;
    }
    aligned = aligned && c->cur == b->ctx[0]->cur;
    profiling = profiling || c->prof_on;
  }
  for (int s = 0; s < nsteps; ++s) {
    // refined instances recycle their right sides once two steps are recorded; the graph holds
    // that form only, so until every refined instance is there the steps run eagerly
    bool rec_ok = true;
    for (pfd_ctx* c : b->ctx) {
      begin_step(c, eq);
      if (c->prob.precision == PFD_REFINED_FP32 && !c->rec_on) rec_ok = false;
    }
    if (!aligned || profiling || !rec_ok) {
      // instances at different time-level parities (or instrumented): plain launches in order
      for (pfd_ctx* c : b->ctx) BCHK(eager_step(c, eq));
    } else {
      for (pfd_ctx* c : b->ctx)
        if (c->is3d) refresh_spectral_sources(c);   // host-decided transforms stay outside
      const int cur = b->ctx[0]->cur;
      hipGraphExec_t& ex = b->gexec[cur][eq];
      std::vector<unsigned long>& gen = b->gen[cur][eq];
      bool stale = gen.size() != b->ctx.size();
      for (size_t i = 0; i < b->ctx.size() && !stale; ++i) stale = gen[i] != b->ctx[i]->graph_gen;
      if (ex && stale) {
        BCHK(hipStreamSynchronize(b->stream));
        (void)hipGraphExecDestroy(ex);
        ex = nullptr;
      }
      if (!ex) {
        BCHK(capture(b, eq, &ex));
        gen.resize(b->ctx.size());
        for (size_t i = 0; i < b->ctx.size(); ++i) gen[i] = b->ctx[i]->graph_gen;
      }
      BCHK(hipGraphLaunch(ex, b->stream));
      for (pfd_ctx* c : b->ctx) c->cur = 1 - cur;
    }
    for (pfd_ctx* c : b->ctx) {
      end_step(c, eq);
      ++c->steps;
    }
  }
  // non-finite and refinement checks of every instance (one synchronisation)
  std::vector<int> st(2 * b->ctx.size(), 0);
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    BCHK(hipMemcpyAsync(&st[2 * i], b->ctx[i]->d_status, 2 * sizeof(int), hipMemcpyDeviceToHost, b->stream));
    BCHK(hipMemsetAsync(b->ctx[i]->d_status + 1, 0, sizeof(int), b->stream));
  }
  BCHK(hipStreamSynchronize(b->stream));
  pfd_status ret = PFD_OK;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    if (st[2 * i] & 1) {
      b->ctx[i]->failed = 1;
      b->ctx[i]->err = "non-finite value in the state";
      b->err = "non-finite value in instance " + std::to_string(i);
      ret = PFD_ENONFINITE;
    } else if (st[2 * i + 1] && ret == PFD_OK) {
      b->ctx[i]->err = unconverged_msg(st[2 * i + 1]);
      b->err = "instance " + std::to_string(i) + ": " + b->ctx[i]->err;
      ret = PFD_ENOCONV;
    }
  }
  return ret;
}
