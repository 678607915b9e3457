// Serving loop for steady solves (the method's target, Sec. 5.1: each
// problem is marched to its steady state).  A server owns `slots` contexts,
// each with its own HIP stream and host thread; requests are admitted first
// in, first out, when a slot is free and the device memory of the live solves
// plus the new one's estimate fits the budget, so a request that arrives
// while others run starts as soon as one of them ends (continuous batching),
// and the steps of the live solves overlap on the device.
//
// A solve in a slot is blr_steady_solve on that slot's context: the same
// kernels in the same order as alone, with reductions of fixed order, so its
// result does not depend on what runs beside it.  With batch_collisions the
// FP32 pair collisions of all live solves on the fused grids run together
// (Batcher below): per step, one launch sequence over all their bases.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include "internal.hpp"
#include "rendezvous.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
  blr_request req{};
  double t_submit = 0.0;
  size_t need = 0;  // estimated device bytes of the solve's context
};

struct Slot {
  int index = 0;
  blr_ctx ctx = nullptr;  // created on first use; freed when the budget needs the room
  hipStream_t stream = nullptr;
  std::thread th;
  bool assigned = false;  // `job` is this slot's to run
  Job job;
  size_t held = 0;        // device bytes its context holds (after its last solve)
};

// Device bytes a context holds: named workspace and table copies.
size_t ctx_bytes(blr_ctx ctx) {
  if (!ctx) return 0;
  size_t b = 0;
  for (const auto& kv : ctx->bufs) b += kv.second.bytes;
  for (const auto& kv : ctx->tables) {
    const blr::HostTables& h = kv.second->h;
    const size_t es = kv.second->prec == BLR_FP32 ? 4 : 8;
    b += (h.phase.size() + h.fw.size() + h.gloss.size()) * es;
  }
  return b;
}

void copy_message(char* dst, size_t cap, const char* msg) {
  std::snprintf(dst, cap, "%s", msg ? msg : "");
}

// Collisions of the live solves in shared launches.  A solve that batches
// (join) hands each step's FP32 pair collisions to collide() and waits.  When
// every joined solve has handed in a step's collisions (or left), the thread
// that completes the set runs them all: on the batcher's own context and
// stream, after each solve's inputs are ready (an event on its stream), as
// blr::collision_batch per velocity grid; every solve's stream then waits on
// the end of the batch.  The batch's device work is recorded as a HIP graph
// the second time a composition (grids, bases, pair lists, addresses) is
// seen and replayed from then on.
struct Batcher : blr_ctx_t::CollideHook {
  struct Pending {
    blr_vgrid vg{};
    blr::BatchJob job;
    hipEvent_t ready = nullptr;
  };
  struct Graph {
    std::string key;
    int seen = 0;
    uint64_t gen = 0;
    hipGraphExec_t exec = nullptr;
  };

  int device = 0;
  blr::Rendezvous<Pending> rv{[this](const std::vector<Pending*>& b) { return run(b); }};
  std::mutex ev_mu;
  std::map<blr_ctx, hipEvent_t> ready;  // one per solve context, reused every step
  // the round's state (used by one round at a time)
  blr_ctx bctx = nullptr;
  hipStream_t bstream = nullptr;
  hipEvent_t done_ev = nullptr;
  std::vector<Graph> graphs;

  ~Batcher() {
    if (bstream) (void)hipStreamSynchronize(bstream);
    for (auto& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (auto& kv : ready) (void)hipEventDestroy(kv.second);
    if (done_ev) (void)hipEventDestroy(done_ev);
    if (bctx) (void)blr_destroy(bctx);
    if (bstream) (void)hipStreamDestroy(bstream);
  }

  void join() { rv.join(); }
  void leave() { rv.leave(); }
  void stop() { rv.stop(); }

  void collide(blr_ctx ctx, const blr_vgrid& vg, const float* V, int r,
               const std::vector<int32_t>& pairs, float* Q) override {
    Pending p;
    p.vg = vg;
    p.job = blr::BatchJob{V, r, pairs, Q};
    {
      std::lock_guard<std::mutex> lk(ev_mu);
      hipEvent_t& ev = ready[ctx];
      if (!ev) BLR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      p.ready = ev;
    }
    // the step's inputs are ready where this solve's stream stands now
    BLR_HIP(hipEventRecord(p.ready, ctx->stream));
    blr::Rendezvous<Pending>::Outcome o;
    if (!rv.submit(&p, &o)) throw blr::Error(BLR_ERR_ARG, "server stopping");
    if (o.code != 0) throw blr::Error(o.code > 0 ? (blr_status)o.code : BLR_ERR_HIP, o.err);
    BLR_HIP(hipStreamWaitEvent(ctx->stream, done_ev, 0));
  }

 private:
  blr::Rendezvous<Pending>::Outcome run(const std::vector<Pending*>& batch) {
    blr::Rendezvous<Pending>::Outcome o;
    try {
      launch(batch);
    } catch (const blr::Error& e) {
      o.code = e.code;
      o.err = e.what();
    }
    return o;
  }

  void enqueue(const std::vector<std::pair<blr_vgrid, std::vector<blr::BatchJob>>>& groups) {
    for (const auto& g : groups) blr::collision_batch(bctx, g.first, g.second);
  }

  void launch(const std::vector<Pending*>& batch) {
    if (!bctx) {
      BLR_HIP(hipSetDevice(device));
      BLR_HIP(hipStreamCreateWithFlags(&bstream, hipStreamNonBlocking));
      BLR_HIP(hipEventCreateWithFlags(&done_ev, hipEventDisableTiming));
      const blr_status rc = blr_create(device, bstream, &bctx);
      if (rc != BLR_OK) throw blr::Error(rc, "server: batch context creation failed");
      bctx->batch_mode = true;
    }
    // jobs grouped by velocity grid, in order of first appearance
    std::vector<std::pair<blr_vgrid, std::vector<blr::BatchJob>>> groups;
    std::string key;
    for (Pending* p : batch) {
      BLR_HIP(hipStreamWaitEvent(bstream, p->ready, 0));
      size_t gi = groups.size();
      for (size_t k = 0; k < groups.size(); ++k)
        if (std::memcmp(&groups[k].first, &p->vg, sizeof(blr_vgrid)) == 0) gi = k;
      if (gi == groups.size()) groups.push_back({p->vg, {}});
      groups[gi].second.push_back(p->job);
    }
    for (const auto& g : groups) {
      key.append((const char*)&g.first, sizeof(blr_vgrid));
      for (const auto& j : g.second) {
        key.append((const char*)&j.V, sizeof(j.V));
        key.append((const char*)&j.Q, sizeof(j.Q));
        key.append((const char*)&j.r, sizeof(j.r));
        key.append((const char*)j.pairs.data(), j.pairs.size() * sizeof(int32_t));
        key.push_back('|');
      }
    }
    Graph* g = nullptr;
    for (auto& x : graphs)
      if (x.key == key) g = &x;
    if (!g) {
      if (graphs.size() >= 16) {
        if (graphs.front().exec) (void)hipGraphExecDestroy(graphs.front().exec);
        graphs.erase(graphs.begin());
      }
      graphs.push_back(Graph{key, 0, 0, nullptr});
      g = &graphs.back();
    }
    if (g->exec && g->gen != bctx->buf_gen) {  // addresses moved
      (void)hipGraphExecDestroy(g->exec);
      g->exec = nullptr;
      g->seen = 0;
    }
    if (!g->exec && g->seen >= 1) {
      g->exec = record(groups);
      g->gen = bctx->buf_gen;
    }
    if (g->exec) {
      BLR_HIP(hipGraphLaunch(g->exec, bstream));
    } else {
      enqueue(groups);  // first sight, or not recordable: directly
      g->seen = 1;
      g->gen = bctx->buf_gen;
    }
    BLR_HIP(hipEventRecord(done_ev, bstream));
  }

  // The batch's work recorded on a capture stream (nullptr if it cannot be)
  hipGraphExec_t record(const std::vector<std::pair<blr_vgrid, std::vector<blr::BatchJob>>>& groups) {
    if (!bctx->cap_stream)
      BLR_HIP(hipStreamCreateWithFlags(&bctx->cap_stream, hipStreamNonBlocking));
    const uint64_t gen0 = bctx->buf_gen;
    hipGraph_t graph = nullptr;
    hipStream_t s = bctx->stream;
    bctx->stream = bctx->cap_stream;
    bctx->capturing = true;
    bctx->capture_broken = false;
    hipError_t e = hipStreamBeginCapture(bctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        enqueue(groups);
      } catch (...) {
        (void)hipStreamEndCapture(bctx->cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        graph = nullptr;
        e = hipErrorUnknown;
      }
      if (e == hipSuccess) e = hipStreamEndCapture(bctx->cap_stream, &graph);
    }
    bctx->stream = s;
    bctx->capturing = false;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess && graph && !bctx->capture_broken && bctx->buf_gen == gen0)
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return exec;
  }
};

}  // namespace

struct blr_server_t {
  int device = 0;
  int64_t budget = 0;
  std::vector<std::unique_ptr<Slot>> slots;
  std::mutex mu;
  std::condition_variable cv_slot, cv_done;
  std::deque<Job> queue;
  std::deque<blr_completion> done;
  int64_t running = 0;
  std::atomic<bool> stop{false};
  Clock::time_point t0 = Clock::now();
  std::string err;
  std::unique_ptr<Batcher> batcher;  // batch_collisions

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // Device bytes held or claimed by the slots, with `pick` taking `need`.
  size_t used_with(const Slot* pick, size_t need) const {
    size_t u = 0;
    for (const auto& s : slots) {
      if (s.get() == pick) u += std::max(s->held, need);
      else u += s->assigned ? std::max(s->held, s->job.need) : s->held;
    }
    return u;
  }

  static void trim(Slot* s) {
    if (s->ctx) (void)blr_destroy(s->ctx);
    s->ctx = nullptr;
    s->held = 0;
  }

  // Admit queued requests while a slot is free and the budget allows (mu held).
  void dispatch_locked() {
    while (!queue.empty() && !stop.load()) {
      const Job& j = queue.front();
      // an idle slot: the smallest workspace that already covers the request,
      // else the largest one (most of it is reused)
      Slot* pick = nullptr;
      for (auto& s : slots) {
        if (s->assigned) continue;
        if (!pick) {
          pick = s.get();
          continue;
        }
        const bool sc = s->held >= j.need, pc = pick->held >= j.need;
        if (sc && (!pc || s->held < pick->held)) pick = s.get();
        else if (!sc && !pc && s->held > pick->held) pick = s.get();
      }
      if (!pick) return;
      if (budget > 0) {
        const size_t cap = (size_t)budget;
        for (auto& s : slots)  // free idle workspaces until the request fits
          if (used_with(pick, j.need) > cap && !s->assigned && s.get() != pick && s->held > 0)
            trim(s.get());
        if (used_with(pick, j.need) > cap && pick->held > j.need) trim(pick);
        if (used_with(pick, j.need) > cap) return;  // wait for a running solve to end
      }
      pick->job = queue.front();
      queue.pop_front();
      pick->assigned = true;
      ++running;
      cv_slot.notify_all();
    }
  }

  void worker(Slot* sl) {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_slot.wait(lk, [&] { return stop.load() || sl->assigned; });
      if (stop.load()) break;
      const Job job = sl->job;
      lk.unlock();

      blr_completion c{};
      c.tag = job.req.tag;
      c.slot = sl->index;
      c.t_submit = job.t_submit;
      c.t_admit = now();
      blr_status status = BLR_OK;
      try {
        if (!sl->ctx) {
          blr_ctx cx = nullptr;
          const blr_status rc = blr_create(device, sl->stream, &cx);
          if (rc != BLR_OK) throw blr::Error(rc, "server: slot context creation failed");
          sl->ctx = cx;
        }
        blr_problem pb = job.req.problem;
        // this solve's collisions join the batch when they take the fused path
        const bool batched = batcher && pb.ny < 2 && blr::fused_f32_grid(pb.v) &&
                             !(job.req.solve.step.flags & BLR_STEP_FP64_COLLISION);
        if (batched) {
          sl->ctx->collide_hook = batcher.get();
          batcher->join();
        }
        try {
          blr::steady_solve(sl->ctx, &pb, job.req.state, &job.req.solve, &c.info, &stop);
        } catch (...) {
          if (batched) {
            batcher->leave();
            sl->ctx->collide_hook = nullptr;
          }
          throw;
        }
        if (batched) {
          batcher->leave();
          sl->ctx->collide_hook = nullptr;
        }
        status = c.info.converged ? BLR_OK : BLR_ERR_NOT_CONVERGED;
      } catch (const blr::Error& e) {
        status = e.code;
        copy_message(c.message, sizeof(c.message), e.what());
      } catch (const std::bad_alloc&) {
        status = BLR_ERR_NOMEM;
        copy_message(c.message, sizeof(c.message), "host allocation failed");
      } catch (const std::exception& e) {
        status = BLR_ERR_HIP;
        copy_message(c.message, sizeof(c.message), e.what());
      }
      c.status = status;
      c.t_done = now();
      const size_t held = ctx_bytes(sl->ctx);

      lk.lock();
      sl->held = held;
      sl->assigned = false;
      c.bytes = (int64_t)held;
      --running;
      if (!stop.load()) done.push_back(c);
      dispatch_locked();
      cv_done.notify_all();
    }
  }
};

// ------------------------------------------------------------------ C ABI --
extern "C" {

blr_status blr_server_create(int device, const blr_server_params* params, blr_server* out) {
  if (!out || !params) return BLR_ERR_ARG;
  *out = nullptr;
  if (params->slots < 1 || params->slots > 16) return BLR_ERR_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return BLR_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return BLR_ERR_HIP;
  blr_server sv = new (std::nothrow) blr_server_t();
  if (!sv) return BLR_ERR_NOMEM;
  sv->device = device;
  sv->budget = params->hbm_budget;
  if (params->batch_collisions) {
    sv->batcher = std::make_unique<Batcher>();
    sv->batcher->device = device;
  }
  for (int k = 0; k < params->slots; ++k) {
    auto s = std::make_unique<Slot>();
    s->index = k;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      for (auto& t : sv->slots) (void)hipStreamDestroy(t->stream);
      delete sv;
      return BLR_ERR_HIP;
    }
    sv->slots.push_back(std::move(s));
  }
  for (auto& s : sv->slots) {
    Slot* p = s.get();
    p->th = std::thread([sv, p] { sv->worker(p); });
  }
  *out = sv;
  return BLR_OK;
}

blr_status blr_server_submit(blr_server sv, const blr_request* req) {
  if (!sv) return BLR_ERR_ARG;
  try {
    blr::require(req != nullptr && req->state != nullptr, "null request or state");
    const blr_state* st = req->state;
    blr::require(st->X && st->S && st->V, "null state arrays");
    blr::require(st->r_cap >= 1 && st->r_cap <= 64 && st->r >= 1 && st->r <= st->r_cap,
                 "state r / r_cap out of range");
    blr::require(req->problem.nx >= 2 && req->problem.f_left && req->problem.f_right,
                 "bad problem (nx >= 2, inflow arrays)");
    blr::require(req->solve.max_steps >= 1, "max_steps must be >= 1");
    blr::validate_vgrid(req->problem.v);
    const bool fp64c = (req->solve.step.flags & BLR_STEP_FP64_COLLISION) != 0;
    // cells: nx, or nx ny on a rectangle (the x-side arrays scale with them)
    const long cells = (long)req->problem.nx * (req->problem.ny >= 2 ? req->problem.ny : 1);
    if (cells > (1L << 22)) throw blr::Error(BLR_ERR_ARG, "problem.nx * ny must be <= 2^22");
    const bool defect = (req->solve.step.flags & BLR_STEP_FP64_DEFECT) != 0;
    const size_t need =
        blr::solve_workspace_bytes(req->problem.v, (int)cells, st->r_cap, fp64c, defect);
    blr::require(sv->budget <= 0 || need <= (size_t)sv->budget,
                 "request needs " + std::to_string(need) + " bytes of device memory, more than the "
                 "server's budget of " + std::to_string(sv->budget), BLR_ERR_NOMEM);
    std::lock_guard<std::mutex> lk(sv->mu);
    blr::require(!sv->stop.load(), "server is stopping");
    Job j;
    j.req = *req;
    j.t_submit = sv->now();
    j.need = need;
    sv->queue.push_back(j);
    sv->dispatch_locked();
    return BLR_OK;
  } catch (const blr::Error& e) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->err = e.what();
    return BLR_ERR_HIP;
  }
}

blr_status blr_server_wait(blr_server sv, int32_t max_out, double timeout_s, blr_completion* out,
                           int32_t* n_out) {
  if (!sv || !n_out || max_out < 0 || (max_out > 0 && !out)) return BLR_ERR_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto ready = [&] { return !sv->done.empty() || (sv->queue.empty() && sv->running == 0); };
  if (timeout_s < 0)
    sv->cv_done.wait(lk, ready);
  else
    sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
  int32_t n = 0;
  while (n < max_out && !sv->done.empty()) {
    out[n++] = sv->done.front();
    sv->done.pop_front();
  }
  *n_out = n;
  return BLR_OK;
}

blr_status blr_server_load(blr_server sv, int64_t* queued, int64_t* running) {
  if (!sv || !queued || !running) return BLR_ERR_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  *queued = (int64_t)sv->queue.size();
  *running = sv->running;
  return BLR_OK;
}

blr_status blr_server_clock(blr_server sv, double* t) {
  if (!sv || !t) return BLR_ERR_ARG;
  *t = sv->now();
  return BLR_OK;
}

blr_status blr_server_batch_stats(blr_server sv, int64_t* rounds, int64_t* jobs) {
  if (!sv || !rounds || !jobs) return BLR_ERR_ARG;
  *rounds = *jobs = 0;
  if (sv->batcher) {
    *rounds = sv->batcher->rv.rounds();
    *jobs = sv->batcher->rv.items();
  }
  return BLR_OK;
}

const char* blr_server_last_error(blr_server sv) { return sv ? sv->err.c_str() : "null server"; }

blr_status blr_server_destroy(blr_server sv) {
  if (!sv) return BLR_ERR_ARG;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop.store(true);
    sv->queue.clear();
  }
  sv->cv_slot.notify_all();
  if (sv->batcher) sv->batcher->stop();
  for (auto& s : sv->slots)
    if (s->th.joinable()) s->th.join();
  (void)hipSetDevice(sv->device);
  for (auto& s : sv->slots) {
    blr_server_t::trim(s.get());
    if (s->stream) (void)hipStreamDestroy(s->stream);
  }
  delete sv;
  return BLR_OK;
}

}  // extern "C"
