// Solve driver: Algorithm 1 on the device, one or many grids at a time.
//
// One outer step is a fixed sequence of launches -- the outer residual and
// update, then `inner` Krylov iterations -- over the block table.  All
// scalars (alpha, beta, eps_R, convergence flags) live in device State
// records, so the sequence is captured once as a HIP graph (several outer
// steps unrolled) and replayed; the host only polls the done flags, and it
// overlaps each poll with the next replays.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "pi_kernels.h"
#include "pi_plan.h"

using namespace pi;

namespace {

constexpr int kUnroll = 8;  // outer steps per graph replay
constexpr int64_t kAsyncMaxIter = 1 << 22;  // bound on max_iter of PI_ASYNC solves

struct Group {               // instances of one launch shape (shape_of)
  BlockEnt *tab = nullptr;   // device
  int ntab = 0;
};

struct Launcher {
  bool fp64 = false;
  Inst *insts = nullptr;
  State *sts = nullptr;
  double *part = nullptr;
  int count = 0;             // instances
  bool cg_finalize = false;  // some instance's CG passes need the finalize kernel
  bool cg_rq = false;        // single plan whose CG passes evaluate q again
  bool cg_rq_opl = false;    // ... with the fixed point's operator
  Group rq;                  // ... and the table of its CG passes
  Group grp[kShapes];

  // the kernel over every instance, then (if it reduces) its finalize; the
  // CG passes of instances of at most kInlineMaxBlocks blocks sum the
  // previous pass's partials themselves and need none
  hipError_t go(KernelId k, hipStream_t s, int iarg = 0, const void *x = nullptr, void *y = nullptr,
                bool finalize = true) const {
    for (int g = 0; g < kShapes; ++g) {
      if (grp[g].ntab <= 0) continue;
      hipError_t e;
      if (k == K_CG_STEP && cg_rq) {
        // every CG pass over the table with the boundary-layer blocks, so
        // that all of a pass's partial-sum slots are written
        LaunchArgs la{rq.tab, insts, sts, part, rq.ntab, s, iarg, x, y};
        e = iarg > 0 ? launch_cg_rq(cg_rq_opl, la) : launch(k, fp64, g, la);
      } else {
        LaunchArgs la{grp[g].tab, insts, sts, part, grp[g].ntab, s, iarg, x, y};
        e = launch(k, fp64, g, la);
      }
      if (e != hipSuccess) return e;
    }
    if (k == K_CG_STEP && !cg_finalize) return hipSuccess;
    if (finalize && reduces(k)) return launch_finalize(k, insts, sts, part, count, s, iarg);
    return hipSuccess;
  }

  hipError_t outer_steps(hipStream_t s, int unroll, int inner, bool bicg) const {
    for (int u = 0; u < unroll; ++u) {
      hipError_t e = go(K_OUTER, s);
      if (e != hipSuccess) return e;
      if (bicg && (e = go(K_COPY_RES, s)) != hipSuccess) return e;
      for (int i = 0; i < inner; ++i) {
        if (bicg) {
          if ((e = go(K_BICG_P, s)) != hipSuccess) return e;
          if ((e = go(K_BICG_S, s)) != hipSuccess) return e;
          if ((e = go(K_BICG_UPDATE, s)) != hipSuccess) return e;
        } else {
          // one pass per CG iteration; each folds in the previous one's
          // update, and the outer kernel folds in the last one's
          if ((e = go(K_CG_STEP, s, i)) != hipSuccess) return e;
        }
      }
    }
    return hipSuccess;
  }
};

// outer steps per graph replay: about kUnroll * 8 inner iterations
int unroll_for(int inner) { return std::max(1, std::min(kUnroll, 64 / std::max(1, inner))); }

hipError_t capture(const Launcher &L, hipStream_t cap, int inner, bool bicg, hipGraphExec_t *exec) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t e2 = L.outer_steps(cap, unroll_for(inner), inner, bicg);
  e = hipStreamEndCapture(cap, &g);
  if (e2 != hipSuccess) e = e2;
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return e;
  }
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e;
}

State fresh_state() {
  State s;
  memset(&s, 0, sizeof(s));
  s.first = 1;
  s.alpha = 1.0;
  s.omega = 1.0;
  s.stop_at = kNoStop;
  return s;
}

// Replay the outer-step graph until every instance reports done.  `hstate`
// is a pinned buffer of 2 * count records.  Each poll checks a snapshot of
// the states while the next replays run.  If `rebuild` is given and returns
// true for a snapshot in which some instance is still running, the loop
// stops there (*stopped = true) so that the caller can shrink the work list;
// `launched` counts replays across such restarts against max_iter.
pi_status iterate(hipGraphExec_t exec, hipStream_t stream, State *dstate, State *hstate, int64_t count,
                  int64_t max_iter, int unroll, int64_t *launched,
                  const std::function<bool(const State *)> &rebuild = nullptr, bool *stopped = nullptr) {
  if (stopped) *stopped = false;
  hipEvent_t ev[2];
  if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess) return PI_ERR_DEVICE;
  if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return PI_ERR_DEVICE;
  }
  // every replay advances each unfinished instance by `unroll` outer steps
  const int64_t bound = max_iter / unroll + 4;
  int replays = 1;
  int cur = 0;
  bool pending = false;
  pi_status rc = PI_ERR_DEVICE;
  const size_t bytes = (size_t)count * sizeof(State);
  auto all_done = [&](const State *snap) {
    for (int64_t i = 0; i < count; ++i)
      if (!snap[i].done) return false;
    return true;
  };
  for (;;) {
    const int r = (int)std::min<int64_t>(replays, bound - *launched);
    for (int i = 0; i < r; ++i)
      if (hipGraphLaunch(exec, stream) != hipSuccess) goto out;
    *launched += r;
    if (hipMemcpyAsync(hstate + cur * count, dstate, bytes, hipMemcpyDeviceToHost, stream) != hipSuccess) goto out;
    if (hipEventRecord(ev[cur], stream) != hipSuccess) goto out;
    if (pending) {
      // check the previous snapshot while the latest replays run
      const State *snap = hstate + (cur ^ 1) * count;
      if (hipEventSynchronize(ev[cur ^ 1]) != hipSuccess) goto out;
      if (all_done(snap)) {
        rc = PI_OK;
        break;
      }
      if (rebuild && rebuild(snap)) {
        if (stopped) *stopped = true;
        rc = PI_OK;
        break;
      }
    }
    pending = true;
    cur ^= 1;
    if (*launched >= bound) {
      if (hipEventSynchronize(ev[cur ^ 1]) != hipSuccess) goto out;
      rc = all_done(hstate + (cur ^ 1) * count) ? PI_OK : PI_ERR_DEVICE;
      break;
    }
    replays = std::min(replays * 2, 16);
  }
out:
  // the events of the replays still in flight are ordered on `stream`
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  return rc;
}

pi_status finish(const Launcher &L, hipStream_t stream, State *dstate, State *hstate, int64_t count) {
  if (L.go(K_GAUGE_SUM, stream) != hipSuccess || L.go(K_GAUGE_GROUPS, stream) != hipSuccess ||
      L.go(K_GAUGE_APPLY, stream) != hipSuccess)
    return PI_ERR_DEVICE;
  if (hipMemcpyAsync(hstate, dstate, (size_t)count * sizeof(State), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return PI_ERR_DEVICE;
  return PI_OK;
}

void fill_info(pi_info *info, const State &s, const pi_plan_s *p, double ms) {
  if (!info) return;
  info->outer_iters = s.outer;
  info->inner_iters_total = s.inner_total;
  info->eps_R = s.epsR;
  info->eps_P = s.epsP;
  info->ms = ms;
  info->status = s.status;
  info->components = p->ncomp;
  info->worklist_rebuilds = 0;
}

int worst(int a, int b) {
  // any error outranks PI_OK; keep the first error seen
  return a != PI_OK ? a : b;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

bool set_user(Inst &in, const pi_plan_s *p, const void *gx, const void *gy, const void *gz, void *P, double tol,
              int64_t max_iter, uint32_t flags) {
  if (!gx || !gy || !P) return false;
  if (p->ndim == 3 && !gz) return false;
  if (!(tol >= 0.0) || max_iter < 0) return false;
  in.g[0] = gx;
  in.g[1] = gy;
  in.g[2] = p->ndim == 3 ? gz : nullptr;
  in.Pout = P;
  in.P0 = (flags & PI_WARM_START) ? P : nullptr;
  in.tol = tol;
  in.max_iter = max_iter;
  in.inner_iters = p->inner_iters;
  return true;
}

hipStream_t cap_stream(pi_plan_s *p) {
  if (!p->cap_stream) (void)hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  return p->cap_stream;
}

// A plan whose pi_set_tile failed to allocate its block table has none
// (ntab == 0): its calls report PI_ERR_OOM until a tile is set again.
bool has_table(const pi_plan_s *p) { return p->ntab > 0 && p->d_tab && p->d_part; }

Launcher single_launcher(pi_plan_s *p) {
  Launcher L;
  L.fp64 = p->fp64;
  L.insts = p->d_inst;
  L.sts = p->d_state;
  L.part = p->d_part;
  L.count = 1;
  L.cg_finalize = !p->bicgstab && !p->inst.cg_inline;
  L.cg_rq = p->inst.cg_rq != 0 && p->d_tab_rq != nullptr;
  L.cg_rq_opl = p->inst.inner_op != 0;
  L.rq = Group{p->d_tab_rq, p->ntab_rq};
  L.grp[shape_of(p->ndim, p->inst.vw, p->inst.gen, p->inst.cc)] = Group{p->d_tab, p->ntab};
  return L;
}

}  // namespace

extern "C" pi_status pi_solve(pi_plan_t p, const void *gx, const void *gy, const void *gz, void *P, double tol,
                              int64_t max_iter, uint32_t flags, pi_info *info, void *stream_) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!p || (flags & ~(PI_WARM_START | PI_ASYNC))) return PI_ERR_INVALID_ARG;
  if (!has_table(p)) return PI_ERR_OOM;
  const bool async = (flags & PI_ASYNC) != 0;
  // the asynchronous form enqueues one replay per `unroll` outer steps up
  // to max_iter: it needs a bound the caller can afford
  if (async && max_iter > kAsyncMaxIter) return PI_ERR_INVALID_ARG;
  hipStream_t stream = (hipStream_t)stream_;
  Inst in = p->inst;
  if (!set_user(in, p, gx, gy, gz, P, tol, max_iter, flags)) return PI_ERR_INVALID_ARG;
  State st0 = fresh_state();
  if (hipMemcpyAsync(p->d_inst, &in, sizeof(Inst), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(p->d_state, &st0, sizeof(State), hipMemcpyHostToDevice, stream) != hipSuccess)
    return PI_ERR_DEVICE;
  const Launcher L = single_launcher(p);
  if (L.go(K_INIT, stream, (flags & PI_WARM_START) ? 1 : 0) != hipSuccess || L.go(K_SOURCE, stream) != hipSuccess)
    return PI_ERR_DEVICE;
  const int key = p->inner_iters * 2 + (p->bicgstab ? 1 : 0);
  if (!p->graph || p->graph_key != key) {
    if (p->graph) (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
    if (capture(L, cap_stream(p), p->inner_iters, p->bicgstab, &p->graph) != hipSuccess) return PI_ERR_DEVICE;
    p->graph_key = key;
  }
  if (async) {
    // enough replays to reach max_iter outer steps (each replay advances an
    // unfinished instance by `unroll`; after the stop every kernel of a
    // replay returns at once), then the gauge and a copy of the final state
    // into the plan's pinned record, all on `stream`
    const int unroll = unroll_for(p->inner_iters);
    const int64_t reps = (max_iter + 1 + unroll - 1) / unroll;
    for (int64_t r = 0; r < reps; ++r)
      if (hipGraphLaunch(p->graph, stream) != hipSuccess) return PI_ERR_DEVICE;
    if (L.go(K_GAUGE_SUM, stream) != hipSuccess || L.go(K_GAUGE_GROUPS, stream) != hipSuccess ||
        L.go(K_GAUGE_APPLY, stream) != hipSuccess ||
        hipMemcpyAsync(p->h_state, p->d_state, sizeof(State), hipMemcpyDeviceToHost, stream) != hipSuccess)
      return PI_ERR_DEVICE;
    return PI_OK;
  }
  // h_state holds three records: [0] final snapshot, [1..2] polling buffers
  int64_t launched = 0;
  pi_status rc =
      iterate(p->graph, stream, p->d_state, p->h_state + 1, 1, max_iter, unroll_for(p->inner_iters), &launched);
  if (rc != PI_OK) return rc;
  rc = finish(L, stream, p->d_state, p->h_state, 1);
  if (rc != PI_OK) return rc;
  fill_info(info, *p->h_state, p, ms_since(t0));
  return (pi_status)p->h_state->status;
}

extern "C" pi_status pi_last_info(pi_plan_t p, pi_info *info) {
  if (!p || !info) return PI_ERR_INVALID_ARG;
  fill_info(info, *p->h_state, p, 0.0);
  return (pi_status)p->h_state->status;
}

namespace {

// Host side of a batched call: validated instance records, and the block
// table of each launch shape with partial slots numbered across all.
struct BatchSetup {
  bool fp64 = false;
  bool bicg = false;
  int inner = 1;
  int parts = 0;
  bool cg_finalize = false;
  std::vector<Inst> host;
  std::vector<int64_t> idx[kShapes];  // batch index of the instances of each launch shape
  std::vector<BlockEnt> tabs[kShapes];

  // block table of launch shape g holding only the instances marked live
  // (their partial-sum slots unchanged)
  std::vector<BlockEnt> live_table(int g, const std::vector<char> &live) {
    std::vector<Inst *> sub;
    std::vector<int64_t> id;
    for (int64_t i : idx[g])
      if (live[i]) {
        sub.push_back(&host[i]);
        id.push_back(i);
      }
    if (sub.empty()) return {};
    int unused = 0;
    std::vector<BlockEnt> t = build_table(sub, 0, &unused, false);
    for (auto &e : t)
      if (e.inst >= 0) e.inst = (int32_t)id[e.inst];
    return t;
  }
};

// Between replay bundles the work list drops finished instances once they
// hold a quarter of the listed blocks: their blocks would only read the done
// flag and exit.
struct WorkList {
  std::vector<char> live;
  int64_t listed = 0;  // blocks in the current tables
  int rebuilds = 0;

  explicit WorkList(const BatchSetup &b) : live(b.host.size(), 1) {
    for (const auto &h : b.host) listed += h.nblocks;
  }
  // from a snapshot of the states: shrink now?
  bool shrink(const BatchSetup &b, const State *snap) {
    int64_t running = 0;
    for (size_t i = 0; i < b.host.size(); ++i)
      if (!snap[i].done) running += b.host[i].nblocks;
    if (running > listed * 3 / 4) return false;
    for (size_t i = 0; i < b.host.size(); ++i) live[i] = snap[i].done ? 0 : 1;
    listed = running;
    ++rebuilds;
    return true;
  }
};

// Write the live instances' tables over the launcher's (each no longer than
// before) on `stream`.
hipError_t upload_live_tables(BatchSetup &b, const WorkList &wl, Launcher &L, hipStream_t stream) {
  for (int g = 0; g < kShapes; ++g) {
    if (L.grp[g].ntab <= 0) continue;
    b.tabs[g] = b.live_table(g, wl.live);
    L.grp[g].ntab = (int)b.tabs[g].size();
    if (!b.tabs[g].empty() && hipMemcpyAsync(L.grp[g].tab, b.tabs[g].data(), b.tabs[g].size() * sizeof(BlockEnt),
                                             hipMemcpyHostToDevice, stream) != hipSuccess)
      return hipErrorUnknown;
  }
  return hipStreamSynchronize(stream);
}

pi_status batch_setup(int64_t count, const pi_plan_t *plans, const void *const *gx, const void *const *gy,
                      const void *const *gz, void *const *P, const double *tol, int64_t max_iter, uint32_t flags,
                      BatchSetup &b) {
  if (count < 1 || !plans || !gx || !gy || !P || !tol || (flags & ~PI_WARM_START)) return PI_ERR_INVALID_ARG;
  b.fp64 = plans[0] ? plans[0]->fp64 : false;
  b.bicg = plans[0] ? plans[0]->bicgstab : false;
  b.host.resize(count);
  for (int64_t i = 0; i < count; ++i) {
    pi_plan_s *p = plans[i];
    if (!p || p->fp64 != b.fp64 || p->bicgstab != b.bicg) return PI_ERR_INVALID_ARG;
    for (int64_t j = 0; j < i; ++j)
      if (plans[j] == p) return PI_ERR_INVALID_ARG;
    b.host[i] = p->inst;
    if (!set_user(b.host[i], p, gx[i], gy[i], gz ? gz[i] : nullptr, P[i], tol[i], max_iter, flags))
      return PI_ERR_INVALID_ARG;
    b.inner = std::max(b.inner, p->inner_iters);
  }
  std::vector<Inst *> by[kShapes];
  for (int64_t i = 0; i < count; ++i) {
    const Inst &h = b.host[i];
    const int g = shape_of(h.ndim, h.vw, h.gen, h.cc);
    by[g].push_back(&b.host[i]);
    b.idx[g].push_back(i);
  }
  b.parts = 0;
  for (int g = 0; g < kShapes; ++g) {
    if (by[g].empty()) continue;
    int total = 0;
    b.tabs[g] = build_table(by[g], b.parts, &total);
    // the table names instances by position inside the group; map to batch index
    for (auto &e : b.tabs[g])
      if (e.inst >= 0) e.inst = (int32_t)b.idx[g][e.inst];
    b.parts = total;
  }
  b.cg_finalize = false;
  for (auto &h : b.host) {
    h.part_stride = b.parts;
    h.cg_rq = 0;  // batched launches store q
    h.cg_slots = h.nblocks;
    h.cg_inline = h.nblocks <= kInlineMaxBlocks ? 1 : 0;
    if (!b.bicg && !h.cg_inline) b.cg_finalize = true;
  }
  return PI_OK;
}

pi_status batch_report(int64_t count, const pi_plan_t *plans, const State *hst, pi_info *infos,
                       std::chrono::steady_clock::time_point t0, int rebuilds) {
  const double ms = ms_since(t0);
  int w = PI_OK;
  for (int64_t i = 0; i < count; ++i) {
    fill_info(infos ? infos + i : nullptr, hst[i], plans[i], ms);
    if (infos) infos[i].worklist_rebuilds = rebuilds;
    w = worst(w, hst[i].status);
  }
  return (pi_status)w;
}

}  // namespace

extern "C" pi_status pi_solve_batched(int64_t count, const pi_plan_t *plans, const void *const *gx,
                                      const void *const *gy, const void *const *gz, void *const *P,
                                      const double *tol, int64_t max_iter, uint32_t flags, pi_info *infos,
                                      void *stream_) {
  const auto t0 = std::chrono::steady_clock::now();
  BatchSetup b;
  pi_status rc = batch_setup(count, plans, gx, gy, gz, P, tol, max_iter, flags, b);
  if (rc != PI_OK) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  Launcher L;
  L.fp64 = b.fp64;
  L.count = (int)count;
  L.cg_finalize = b.cg_finalize;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  State *hst = nullptr;
  rc = PI_ERR_DEVICE;
  std::vector<State> init(count, fresh_state());
  if (hipMalloc((void **)&L.insts, count * sizeof(Inst)) != hipSuccess ||
      hipMalloc((void **)&L.sts, count * sizeof(State)) != hipSuccess ||
      hipMalloc((void **)&L.part, (size_t)std::max(b.parts, 1) * 3 * 4 * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void **)&hst, 2 * count * sizeof(State), hipHostMallocDefault) != hipSuccess) {
    rc = PI_ERR_OOM;
    goto done;
  }
  for (int g = 0; g < kShapes; ++g) {
    if (b.tabs[g].empty()) continue;
    if (hipMalloc((void **)&L.grp[g].tab, b.tabs[g].size() * sizeof(BlockEnt)) != hipSuccess) {
      rc = PI_ERR_OOM;
      goto done;
    }
    L.grp[g].ntab = (int)b.tabs[g].size();
    if (hipMemcpyAsync(L.grp[g].tab, b.tabs[g].data(), b.tabs[g].size() * sizeof(BlockEnt), hipMemcpyHostToDevice,
                       stream) != hipSuccess)
      goto done;
  }
  if (hipMemcpyAsync(L.insts, b.host.data(), count * sizeof(Inst), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(L.sts, init.data(), count * sizeof(State), hipMemcpyHostToDevice, stream) != hipSuccess)
    goto done;
  if (L.go(K_INIT, stream, (flags & PI_WARM_START) ? 1 : 0) != hipSuccess || L.go(K_SOURCE, stream) != hipSuccess)
    goto done;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) goto done;
  {
    WorkList wl(b);
    int64_t launched = 0;
    auto shrink = [&](const State *snap) { return wl.shrink(b, snap); };
    for (;;) {
      if (capture(L, cap, b.inner, b.bicg, &exec) != hipSuccess) {
        rc = PI_ERR_DEVICE;
        goto done;
      }
      bool stopped = false;
      rc = iterate(exec, stream, L.sts, hst, count, max_iter, unroll_for(b.inner), &launched, shrink, &stopped);
      if (rc != PI_OK) goto done;
      if (!stopped) break;
      // the replays still in flight finish before the tables change
      if (hipStreamSynchronize(stream) != hipSuccess) {
        rc = PI_ERR_DEVICE;
        goto done;
      }
      (void)hipGraphExecDestroy(exec);
      exec = nullptr;
      if (upload_live_tables(b, wl, L, stream) != hipSuccess) {
        rc = PI_ERR_DEVICE;
        goto done;
      }
    }
    // the gauge runs over every instance
    for (int g = 0; g < kShapes; ++g) {
      if (b.idx[g].empty()) continue;
      std::vector<char> all(count, 1);
      b.tabs[g] = b.live_table(g, all);
      L.grp[g].ntab = (int)b.tabs[g].size();
      if (hipMemcpyAsync(L.grp[g].tab, b.tabs[g].data(), b.tabs[g].size() * sizeof(BlockEnt), hipMemcpyHostToDevice,
                         stream) != hipSuccess) {
        rc = PI_ERR_DEVICE;
        goto done;
      }
    }
    rc = finish(L, stream, L.sts, hst, count);
    if (rc != PI_OK) goto done;
    rc = batch_report(count, plans, hst, infos, t0, wl.rebuilds);
  }
done:
  if (exec) (void)hipGraphExecDestroy(exec);
  if (cap) (void)hipStreamDestroy(cap);
  (void)hipStreamSynchronize(stream);
  if (L.insts) (void)hipFree(L.insts);
  if (L.sts) (void)hipFree(L.sts);
  if (L.part) (void)hipFree(L.part);
  for (int g = 0; g < kShapes; ++g)
    if (L.grp[g].tab) (void)hipFree(L.grp[g].tab);
  if (hst) (void)hipHostFree(hst);
  return rc;
}

// ---------------------------------------------------------------------------
// pi_solve_batched_noalloc: the batched solve with its per-call device
// buffers (instance records, scalars, partial sums, block tables) carved
// out of one static device array instead of allocated
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kNaInsts = PI_NOALLOC_MAX_INSTANCES;
constexpr int64_t kNaParts = PI_NOALLOC_MAX_PARTIALS;
constexpr int64_t kNaTab = PI_NOALLOC_MAX_TABLE;

constexpr size_t align256(size_t v) { return (v + 255) / 256 * 256; }
constexpr size_t kNaOffSts = align256(kNaInsts * sizeof(Inst));
constexpr size_t kNaOffPart = kNaOffSts + align256(kNaInsts * sizeof(State));
constexpr size_t kNaOffTab = kNaOffPart + align256(kNaParts * 3 * 4 * sizeof(double));
constexpr size_t kNaBytes = kNaOffTab + align256(kNaTab * sizeof(BlockEnt));

}  // namespace

// One per GPU the library runs on, held until the process ends.  Host code
// never passes this name to a kernel or a copy: it is a host-side stand-in;
// the device address comes from hipGetSymbolAddress (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_na_mu;
unsigned char *g_na_ptr[kMaxDevices] = {};
State g_na_host[2 * kNaInsts];  // polling snapshots (pageable host memory)

// Device address of this GPU's scratch array, looked up once per device
// with that device current.
hipError_t noalloc_scratch(unsigned char **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_na_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_na_ptr[dev] = (unsigned char *)ptr;
  }
  *out = g_na_ptr[dev];
  return hipSuccess;
}

// Replays of the outer-step sequence without a graph: the launches go
// straight onto the stream; the done flags are copied back to pageable host
// memory and checked every `unroll` outer steps, and the work list shrinks
// as in pi_solve_batched (the tables are rewritten in place).
pi_status noalloc_iterate(BatchSetup &b, Launcher &L, hipStream_t stream, int64_t count, int64_t max_iter,
                          int *rebuilds) {
  const int unroll = unroll_for(b.inner);
  const int64_t bound = max_iter / unroll + 4;
  const size_t bytes = (size_t)count * sizeof(State);
  WorkList wl(b);
  pi_status rc = PI_ERR_DEVICE;
  for (int64_t r = 0; r < bound; ++r) {
    if (L.outer_steps(stream, unroll, b.inner, b.bicg) != hipSuccess) return PI_ERR_DEVICE;
    if (hipMemcpyAsync(g_na_host, L.sts, bytes, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return PI_ERR_DEVICE;
    bool all = true;
    for (int64_t i = 0; i < count && all; ++i) all = g_na_host[i].done != 0;
    if (all) {
      rc = PI_OK;
      break;
    }
    if (wl.shrink(b, g_na_host) && upload_live_tables(b, wl, L, stream) != hipSuccess) return PI_ERR_DEVICE;
  }
  *rebuilds = wl.rebuilds;
  if (rc != PI_OK) return rc;
  // the gauge runs over every instance
  std::vector<char> all(count, 1);
  for (int g = 0; g < kShapes; ++g) {
    if (b.idx[g].empty()) continue;
    b.tabs[g] = b.live_table(g, all);
    L.grp[g].ntab = (int)b.tabs[g].size();
    if (hipMemcpyAsync(L.grp[g].tab, b.tabs[g].data(), b.tabs[g].size() * sizeof(BlockEnt), hipMemcpyHostToDevice,
                       stream) != hipSuccess)
      return PI_ERR_DEVICE;
  }
  return PI_OK;
}

}  // namespace

extern "C" pi_status pi_solve_batched_noalloc(int64_t count, const pi_plan_t *plans, const void *const *gx,
                                              const void *const *gy, const void *const *gz, void *const *P,
                                              const double *tol, int64_t max_iter, uint32_t flags, pi_info *infos,
                                              void *stream_) {
  const auto t0 = std::chrono::steady_clock::now();
  if (count > kNaInsts) return PI_ERR_TOO_LARGE;
  BatchSetup b;
  pi_status rc = batch_setup(count, plans, gx, gy, gz, P, tol, max_iter, flags, b);
  if (rc != PI_OK) return rc;
  int64_t ntab = 0;
  for (int g = 0; g < kShapes; ++g) ntab += (int64_t)b.tabs[g].size();
  if (b.parts > kNaParts || ntab > kNaTab) return PI_ERR_TOO_LARGE;
  // one caller at a time: the scratch array and the host snapshots are shared
  std::lock_guard<std::mutex> guard(g_na_mu);
  unsigned char *base = nullptr;
  if (noalloc_scratch(&base) != hipSuccess) return PI_ERR_DEVICE;
  hipStream_t stream = (hipStream_t)stream_;
  Launcher L;
  L.fp64 = b.fp64;
  L.count = (int)count;
  L.cg_finalize = b.cg_finalize;
  L.insts = (Inst *)(base);
  L.sts = (State *)(base + kNaOffSts);
  L.part = (double *)(base + kNaOffPart);
  BlockEnt *tab = (BlockEnt *)(base + kNaOffTab);
  for (int g = 0; g < kShapes; ++g) {
    if (b.tabs[g].empty()) continue;
    L.grp[g].tab = tab;
    L.grp[g].ntab = (int)b.tabs[g].size();
    if (hipMemcpyAsync(tab, b.tabs[g].data(), b.tabs[g].size() * sizeof(BlockEnt), hipMemcpyHostToDevice,
                       stream) != hipSuccess)
      return PI_ERR_DEVICE;
    tab += b.tabs[g].size();
  }
  // every record and scalar the kernels read is written here first: the
  // array keeps the previous call's contents
  for (int64_t i = 0; i < count; ++i) g_na_host[i] = fresh_state();
  if (hipMemcpyAsync(L.insts, b.host.data(), count * sizeof(Inst), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(L.sts, g_na_host, count * sizeof(State), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return PI_ERR_DEVICE;
  if (L.go(K_INIT, stream, (flags & PI_WARM_START) ? 1 : 0) != hipSuccess || L.go(K_SOURCE, stream) != hipSuccess)
    return PI_ERR_DEVICE;
  int rebuilds = 0;
  rc = noalloc_iterate(b, L, stream, count, max_iter, &rebuilds);
  if (rc == PI_OK) rc = finish(L, stream, L.sts, g_na_host, count);
  if (rc == PI_OK) rc = batch_report(count, plans, g_na_host, infos, t0, rebuilds);
  (void)hipStreamSynchronize(stream);
  return rc;
}

extern "C" pi_status pi_source(pi_plan_t p, const void *gx, const void *gy, const void *gz, void *S, void *stream_) {
  if (!p || !gx || !gy || !S || (p->ndim == 3 && !gz)) return PI_ERR_INVALID_ARG;
  if (!has_table(p)) return PI_ERR_OOM;
  hipStream_t stream = (hipStream_t)stream_;
  Inst in = p->inst;
  in.g[0] = gx;
  in.g[1] = gy;
  in.g[2] = p->ndim == 3 ? gz : nullptr;
  in.S = S;
  State st0 = fresh_state();
  const Launcher L = single_launcher(p);
  if (hipMemcpyAsync(p->d_inst, &in, sizeof(Inst), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(p->d_state, &st0, sizeof(State), hipMemcpyHostToDevice, stream) != hipSuccess ||
      L.go(K_SOURCE, stream) != hipSuccess ||
      hipMemcpyAsync(p->h_state, p->d_state, sizeof(State), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return PI_ERR_DEVICE;
  return p->h_state->nonfinite ? PI_ERR_NONFINITE : PI_OK;
}

extern "C" pi_status pi_apply(pi_plan_t p, int op, const void *x, void *y, void *stream_) {
  if (!p || !x || !y || op < PI_OP_M || op > PI_OP_L || x == y) return PI_ERR_INVALID_ARG;
  // four cells per lane move 16-byte vectors
  const size_t vbytes = (size_t)p->inst.vw * (p->fp64 ? 8 : 4);
  if (p->inst.vw > 1 && (((uintptr_t)x | (uintptr_t)y) & (std::min<size_t>(vbytes, 16) - 1)) != 0)
    return PI_ERR_INVALID_ARG;
  if (!has_table(p)) return PI_ERR_OOM;
  hipStream_t stream = (hipStream_t)stream_;
  // the operator reads only plan fields of the device instance record, which
  // every call leaves in place
  const Launcher L = single_launcher(p);
  if (L.go(K_APPLY, stream, op, x, y) != hipSuccess) return PI_ERR_DEVICE;
  return PI_OK;
}

namespace {

// A mid-solve state for timing single launches: a correction is pending, the
// search direction is not the first one, no convergence, never reaching the
// tolerance.  CG pass 2 (reads and writes the correction) and the outer
// kernel read pass 1's partial sums: alpha = 1e-3 and beta = 1, finite and
// fixed.
pi_status timing_state(pi_plan_t p, hipStream_t stream) {
  Inst in = p->inst;
  in.tol = -1.0;
  in.max_iter = INT64_MAX;
  in.inner_iters = 1 << 30;
  State st = fresh_state();
  st.first = 0;
  st.have_delta = 1;  // a correction is pending (CG: from every pass)
  st.dvalid = 1;
  st.rr = 1.0;
  st.alpha = 1e-3;
  st.beta = 0.5;
  st.normS2 = 1.0;
  std::vector<double> slots((size_t)p->inst.cg_slots * 4);
  for (int i = 0; i < p->inst.cg_slots; ++i) {
    slots[4 * i + 0] = 1e3;  // p.q
    slots[4 * i + 1] = 0.0;  // r.q
    slots[4 * i + 2] = 0.0;  // q.q
    slots[4 * i + 3] = 1.0;  // r.r
  }
  if (hipMemcpyAsync(p->d_inst, &in, sizeof(Inst), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(p->d_state, &st, sizeof(State), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipMemcpyAsync(p->d_part + (size_t)(1 + 1) * in.part_stride * 4 + (size_t)in.part_base * 4, slots.data(),
                     slots.size() * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return PI_ERR_DEVICE;
  return PI_OK;
}

// Average time of `reps` back-to-back launches of f (after one warm-up).
template <class F>
pi_status time_launches(hipStream_t stream, int32_t reps, double *avg_ms, F &&f) {
  hipEvent_t a = nullptr, b = nullptr;
  pi_status rc = PI_ERR_DEVICE;
  float ms = 0.f;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) goto out;
  if (f() != hipSuccess) goto out;  // warm-up launch
  if (hipEventRecord(a, stream) != hipSuccess) goto out;
  for (int i = 0; i < reps; ++i)
    if (f() != hipSuccess) goto out;
  if (hipEventRecord(b, stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
      hipEventElapsedTime(&ms, a, b) != hipSuccess)
    goto out;
  *avg_ms = (double)ms / reps;
  rc = PI_OK;
out:
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipStreamSynchronize(stream);
  return rc;
}

// Per-pass cost of inner CG pass `kpass` (0: the first of an outer step,
// which reads only the residual; 2: one of the later passes) as a solve runs
// it: kCgPassesTimed
// passes, each with its finalize kernel where the tile needs one, captured
// in a HIP graph as the solve captures them and replayed (back-to-back
// stream launches hide the cost of the graph's dependency between a pass
// and its finalize).  The finalize moves the state on between passes; the
// values do not change the amount of work.
constexpr int kCgPassesTimed = 8;
pi_status time_cg_pass(pi_plan_t p, int32_t reps, double *avg_ms, hipStream_t stream, int kpass) {
  pi_status rc = timing_state(p, stream);
  if (rc != PI_OK) return rc;
  const Launcher L = single_launcher(p);
  hipStream_t cap = cap_stream(p);
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return PI_ERR_DEVICE;
  hipError_t e2 = hipSuccess;
  for (int i = 0; i < kCgPassesTimed && e2 == hipSuccess; ++i) e2 = L.go(K_CG_STEP, cap, kpass, nullptr, nullptr, true);
  hipError_t e = hipStreamEndCapture(cap, &g);
  if (e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess || e2 != hipSuccess) return PI_ERR_DEVICE;
  double ms = 0.0;
  rc = time_launches(stream, std::max(1, reps / 2), &ms, [&] { return hipGraphLaunch(ge, stream); });
  (void)hipGraphExecDestroy(ge);
  *avg_ms = ms / kCgPassesTimed;
  return rc;
}

}  // namespace

extern "C" int32_t pi_get_cg_recompute(pi_plan_t p) { return p && p->inst.cg_rq ? 1 : 0; }

extern "C" pi_status pi_time_kernel(pi_plan_t p, int kernel, int32_t reps, double *avg_ms, void *stream_) {
  if (!p || !avg_ms || reps < 1 || (kernel != PI_K_OUTER && kernel != PI_K_INNER)) return PI_ERR_INVALID_ARG;
  if (kernel == PI_K_INNER && p->bicgstab) return PI_ERR_INVALID_ARG;
  if (!has_table(p)) return PI_ERR_OOM;
  hipStream_t stream = (hipStream_t)stream_;
  const Launcher L = single_launcher(p);
  const KernelId k = kernel == PI_K_OUTER ? K_OUTER : K_CG_STEP;
  pi_status rc = timing_state(p, stream);
  if (rc != PI_OK) return rc;
  // the kernel alone: without its finalize the state, and so every launch,
  // stays the same
  const int kpass = 2;
  return time_launches(stream, reps, avg_ms, [&] { return L.go(k, stream, kpass, nullptr, nullptr, false); });
}

// tile cache of pi_autotune: (ndim, nx, ny, nz, fp64, bicgstab) -> (mseg, lane cells, non-temporal outer)
static std::mutex g_tune_mu;
static std::map<std::array<int64_t, 6>, std::array<int32_t, 3>> g_tune;

extern "C" pi_status pi_autotune(pi_plan_t p, int32_t reps, int32_t *mseg_out, void *stream) {
  if (!p || reps < 1) return PI_ERR_INVALID_ARG;
  const std::array<int64_t, 6> key = {p->ndim, p->dims[0], p->dims[1], p->dims[2], p->fp64,
                                      (p->bicgstab ? 1 : 0) | (p->cc ? 2 : 0)};
  std::array<int32_t, 3> best = {-1, 0, 0};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) best = it->second;
  }
  pi_status rc;
  if (best[0] < 0) {
    std::vector<std::array<int32_t, 2>> cand;
    p->inst.nt_outer = 0;
    std::vector<int32_t> widths;
    if (p->dims[0] % 4 == 0) widths.push_back(4);
    if (p->dims[0] % 2 == 0 && !p->cc) widths.push_back(2);
    widths.push_back(1);
    for (int32_t vw : widths) {
      if ((rc = pi_set_tile(p, 0, vw)) != PI_OK) return rc;
      cand.push_back({p->inst.mseg, vw});
      for (int32_t m = 2; m <= 256; m *= 2)
        if (m < p->inst.nm && m != p->inst.mseg) cand.push_back({m, vw});
    }
    // time of one outer step at a candidate tile
    auto step_ms = [&](const std::array<int32_t, 2> &c, int32_t r, double *ms) -> pi_status {
      pi_status e;
      if ((e = pi_set_tile(p, c[0], c[1])) != PI_OK) return e;
      double t_outer = 0.0, t_first = 0.0, t_inner = 0.0;
      if ((e = pi_time_kernel(p, PI_K_OUTER, r, &t_outer, stream)) != PI_OK) return e;
      if (!p->bicgstab && p->inner_iters > 0) {
        if ((e = time_cg_pass(p, r, &t_first, (hipStream_t)stream, 0)) != PI_OK) return e;
        if (p->inner_iters > 1 && (e = time_cg_pass(p, r, &t_inner, (hipStream_t)stream, 2)) != PI_OK) return e;
      }
      *ms = t_outer + t_first + std::max(0, p->inner_iters - 1) * t_inner;
      return PI_OK;
    };
    // every candidate once, then the three fastest again with four times the
    // launches: single short timings differ by a few percent from run to run,
    // about as much as neighbouring tiles do
    std::vector<std::pair<double, size_t>> first;
    for (size_t i = 0; i < cand.size(); ++i) {
      double ms = 0.0;
      if ((rc = step_ms(cand[i], reps, &ms)) != PI_OK) return rc;
      first.push_back({ms, i});
    }
    std::sort(first.begin(), first.end());
    double best_ms = 1e300;
    for (size_t j = 0; j < first.size() && j < 3; ++j) {
      const auto &c = cand[first[j].second];
      double ms = 0.0;
      if ((rc = step_ms(c, 4 * reps, &ms)) != PI_OK) return rc;
      if (ms < best_ms) {
        best_ms = ms;
        best = {c[0], c[1], 0};
      }
    }
    // at the chosen tile: the outer kernel's streams plain or non-temporal
    if ((rc = pi_set_tile(p, best[0], best[1])) != PI_OK) return rc;
    double t_nt[2] = {0.0, 0.0};
    for (int nt = 0; nt < 2; ++nt) {
      p->inst.nt_outer = nt;
      if ((rc = pi_time_kernel(p, PI_K_OUTER, 4 * reps, &t_nt[nt], stream)) != PI_OK) return rc;
    }
    best[2] = t_nt[1] < t_nt[0] ? 1 : 0;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = best;
  }
  p->inst.nt_outer = best[2];
  rc = pi_set_tile(p, best[0], best[1]);
  if (rc == PI_OK && mseg_out) *mseg_out = p->inst.mseg;
  return rc;
}

extern "C" const char *pi_status_string(pi_status s) {
  switch (s) {
    case PI_OK: return "ok";
    case PI_ERR_INVALID_ARG: return "invalid argument";
    case PI_ERR_OOM: return "out of memory";
    case PI_ERR_NONFINITE: return "non-finite gradient in a data cell";
    case PI_ERR_NOT_CONVERGED: return "not converged within max_iter outer steps";
    case PI_ERR_DIVERGED: return "residual became non-finite";
    case PI_ERR_DEVICE: return "HIP runtime error";
    case PI_ERR_TOO_LARGE: return "exceeds the fixed scratch size of the no-allocation entry point";
  }
  return "unknown status";
}
