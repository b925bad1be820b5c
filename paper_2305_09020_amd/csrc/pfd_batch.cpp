// Batches of independent contexts (instances of uneven mesh, order and parameters) stepped
// together, one hipGraph launch per step, in one of two forms:
//  * branches: every instance's step captured as parallel branches (the instances are spread
//    over a few capture streams forked from one origin and joined again), so the graph holds
//    each instance's own launches, free to overlap on the device;
//  * multi-instance launches: every instance's step is recorded (its launches, in order, with
//    their packed arguments), and the k-th launches of all instances that run the same kernel
//    with the same work-group shape become one launch of that kernel's multi-instance form,
//    whose work-groups are the concatenation of the instances' grids; the step's graph is built
//    node by node from these launches.  A step is then about as many launches as one
//    instance's step (times the number of distinct kernels at a position, e.g. one per element
//    order for order-specialised kernels), whatever the number of instances.
// Instances keep their own workspaces, autotuned kernels and state in both forms; the batch
// only orders and groups their launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "pfd_internal.h"
#include "pfd_launch.h"

using namespace pfd;

// one launch of a multi-instance step: the kernel's multi-instance form over `total`
// work-groups, and the offsets of its member table, work-group table and argument packs in the
// plan's device buffer
struct MultiLaunch {
  const void* fn = nullptr;
  size_t pos = 0;                  // position in the instances' launch sequences
  unsigned total = 0, block[3] = {1, 1, 1};
  size_t shm = 0, o_ent = 0, o_tab = 0, o_args = 0;
};
struct MultiPlan {
  char* dmem = nullptr;            // device buffer of all tables and argument packs
  std::vector<MultiLaunch> L;
};

struct pfd_batch {
  std::vector<pfd_ctx*> ctx;
  int mode = PFD_BATCH_MULTI;
  MultiPlan plan[2][2];
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

// graphs and plans of both forms (the device must have finished with them)
static void drop_all(pfd_batch* b) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      if (b->gexec[i][j]) (void)hipGraphExecDestroy(b->gexec[i][j]);
      b->gexec[i][j] = nullptr;
      b->gen[i][j].clear();
      if (b->plan[i][j].dmem) (void)hipFree(b->plan[i][j].dmem);
      b->plan[i][j] = MultiPlan();
    }
}

static void batch_free(pfd_batch* b) {
  drop_all(b);
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

// Multi-instance plan of one step: record every instance's step (launches only; the host-side
// state each step leaves is restored), then group the k-th launches of all instances by kernel
// and work-group shape.  Instances whose sequences differ (another precision, boundary type or
// kernel variant) still run correctly: each launch position is issued in order, one launch per
// group, so every instance's launches keep their order.
static hipError_t build_plan(pfd_batch* b, int eq, MultiPlan& P) {
  const size_t n = b->ctx.size();
  std::vector<std::vector<RecLaunch>> rec(n);
  hipError_t es = hipSuccess;
  for (size_t i = 0; i < n && !es; ++i) {
    pfd_ctx* c = b->ctx[i];
    const int cur = c->cur;
    c->rec = &rec[i];
    es = eager_step(c, eq);
    c->rec = nullptr;
    c->cur = cur;
  }
  if (es) return es;
  size_t maxlen = 0;
  for (auto& r : rec) maxlen = std::max(maxlen, r.size());
  std::vector<unsigned char> host;
  auto carve = [&host](size_t bytes, size_t align) {
    const size_t o = (host.size() + align - 1) / align * align;
    host.resize(o + bytes);
    return o;
  };
  for (size_t j = 0; j < maxlen; ++j) {
    std::vector<std::vector<size_t>> groups;   // member instances of each launch at position j
    for (size_t i = 0; i < n; ++i) {
      if (j >= rec[i].size()) continue;
      const RecLaunch& r = rec[i][j];
      if ((unsigned long long)r.grid[0] * r.grid[1] * r.grid[2] == 0) continue;
      size_t g = 0;
      for (; g < groups.size(); ++g) {
        const RecLaunch& q = rec[groups[g][0]][j];
        if (q.fn == r.fn && std::memcmp(q.block, r.block, sizeof(q.block)) == 0) break;
      }
      if (g == groups.size()) groups.emplace_back();
      groups[g].push_back(i);
    }
    for (auto& grp : groups) {
      const RecLaunch& r0 = rec[grp[0]][j];
      MultiLaunch m;
      m.fn = r0.fn;
      m.pos = j;
      std::memcpy(m.block, r0.block, sizeof(m.block));
      unsigned long long total = 0;
      for (size_t i : grp) {
        const RecLaunch& r = rec[i][j];
        m.shm = std::max(m.shm, r.shm);
        total += (unsigned long long)r.grid[0] * r.grid[1] * r.grid[2];
      }
      if (total >= (1ull << 31)) return hipErrorInvalidConfiguration;
      m.total = (unsigned)total;
      m.o_ent = carve(sizeof(MEnt) * grp.size(), 16);
      m.o_tab = carve(sizeof(unsigned) * total, 16);
      m.o_args = carve(r0.asize * grp.size(), std::max<size_t>(r0.aalign, 16));
      unsigned b0 = 0;
      for (size_t q = 0; q < grp.size(); ++q) {
        const RecLaunch& r = rec[grp[q]][j];
        const unsigned nb = r.grid[0] * r.grid[1] * r.grid[2];
        const MEnt me{r.grid[0], r.grid[1], r.grid[2], b0};
        std::memcpy(host.data() + m.o_ent + q * sizeof(MEnt), &me, sizeof(me));
        unsigned* tab = reinterpret_cast<unsigned*>(host.data() + m.o_tab);
        for (unsigned k = 0; k < nb; ++k) tab[b0 + k] = (unsigned)q;
        std::memcpy(host.data() + m.o_args + q * r0.asize, r.args.data(), r0.asize);
        b0 += nb;
      }
      P.L.push_back(m);
    }
  }
  if (host.empty()) return hipSuccess;
  hipError_t e = hipMalloc(&P.dmem, host.size());
  if (!e) e = hipMemcpy(P.dmem, host.data(), host.size(), hipMemcpyHostToDevice);
  return e;
}

// the plan as the step's graph, built node by node: one kernel node per launch, each depending
// on every node of the previous position; the launches of one position (instances on different
// kernels, e.g. one per element order) are independent of each other
static hipError_t build_multi_graph(pfd_batch* b, int eq, MultiPlan& P, hipGraphExec_t* ex) {
  hipError_t e = build_plan(b, eq, P);
  hipGraph_t g = nullptr;
  if (!e) e = hipGraphCreate(&g, 0);
  std::vector<hipGraphNode_t> prev, cur;
  for (size_t k = 0; k < P.L.size() && !e;) {
    cur.clear();
    const size_t pos = P.L[k].pos;
    for (; k < P.L.size() && P.L[k].pos == pos && !e; ++k) {
      const MultiLaunch& m = P.L[k];
      unsigned total = m.total;
      const void* tab = P.dmem + m.o_tab;
      const void* ent = P.dmem + m.o_ent;
      const void* args = P.dmem + m.o_args;
      void* ka[] = {&total, &tab, &ent, &args};   // copied into the node
      hipKernelNodeParams kp = {};
      kp.func = const_cast<void*>(m.fn);
      kp.gridDim = dim3(total);
      kp.blockDim = dim3(m.block[0], m.block[1], m.block[2]);
      kp.sharedMemBytes = (unsigned)m.shm;
      kp.kernelParams = ka;
      kp.extra = nullptr;
      hipGraphNode_t node = nullptr;
      e = hipGraphAddKernelNode(&node, g, prev.empty() ? nullptr : prev.data(), prev.size(), &kp);
      if (!e) cur.push_back(node);
    }
    prev.swap(cur);
  }
  if (!e) e = hipGraphInstantiate(ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e) {
    *ex = nullptr;
    if (P.dmem) (void)hipFree(P.dmem);
    P = MultiPlan();
  }
  return e;
}

extern "C" pfd_status pfd_batch_set_mode(pfd_batch* b, int mode) {
  if (!b || (mode != PFD_BATCH_BRANCHES && mode != PFD_BATCH_MULTI)) return PFD_EINVAL;
  if (mode != b->mode) {
    BCHK(hipStreamSynchronize(b->stream));
    drop_all(b);
    b->mode = mode;
  }
  return PFD_OK;
}

extern "C" int pfd_batch_launches(const pfd_batch* b) {
  if (!b) return -1;
  int m = -1;
  for (auto& row : b->plan)
    for (auto& p : row)
      if (!p.L.empty()) m = std::max(m, (int)p.L.size());
  return m;
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
      MultiPlan& plan = b->plan[cur][eq];
      if (ex && stale) {
        BCHK(hipStreamSynchronize(b->stream));
        (void)hipGraphExecDestroy(ex);
        ex = nullptr;
        if (plan.dmem) (void)hipFree(plan.dmem);
        plan = MultiPlan();
      }
      if (!ex) {
        if (b->mode == PFD_BATCH_MULTI)
          BCHK(build_multi_graph(b, eq, plan, &ex));
        else
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
