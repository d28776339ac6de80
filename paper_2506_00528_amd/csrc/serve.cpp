// serve.cpp -- continuous-batching server over a resident database.
//
// Requests (nq query codes and a k each) are submitted from any thread and
// queue as pending.  One host thread runs the serve loop:
//
//   * admission: pending requests are admitted in arrival order while their
//     queries fit in free query slots (contiguous, first fit) and their bytes
//     fit in the device-memory budget; an admitted request's codes are copied
//     to the device, re-coded into scan rows, and its running top-k lists are
//     cleared;
//   * ticks: the database is cut into S segments; tick t scans segment
//     (t mod S) for every active query with the batched kernel and merges the
//     segment's top-k into each query's running list.  A request that joined
//     at tick t0 has seen every segment after tick t0 + S - 1 and retires: its
//     lists are turned into ids / scores and copied to pinned host memory;
//   * completion: when a tick's event fires the loop copies the retired
//     results into the request, stamps the time and frees slots and budget.
//
// The top-k of every query is over the same total order of (score, id) keys,
// so merging segments in any order, alone or beside any other requests,
// gives exactly the result of a single full scan.  Two ticks are kept in
// flight so the GPU never waits for the host.  All GPU work of a server runs
// on its own stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "tq_batched.h"
#include "tq_runtime.h"

using namespace tqr;

namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return static_cast<uint64_t>(ts.tv_sec) * 1000000000ull + static_cast<uint64_t>(ts.tv_nsec);
}

enum class RState { Pending, Active, Finishing, Done, Cancelled };

struct Request {
  uint64_t ticket = 0;
  int nq = 0, k = 0;
  std::vector<uint32_t> qcodes;  // canonical, host copy
  std::vector<int32_t> ids, scores;
  RState state = RState::Pending;
  bool cancel = false;
  uint64_t submit_ns = 0, admit_ns = 0, complete_ns = 0;
  int slot0 = -1;
  int ticks_done = 0;
  size_t bytes = 0;
  hipEvent_t done = nullptr;  // results are on the host once it fires
  uint64_t last_tick_ns = 0;  // when its last tick was queued (watchdog)
};

// Pinned, host-to-device staged parameters of one tick: BatchParams followed
// by the active slot list and the retiring slot list.
struct TickStage {
  char *host = nullptr;
  hipEvent_t consumed = nullptr;  // the copy out of `host` has executed
  hipEvent_t done = nullptr;      // all of the tick's device work has executed
  bool used = false;
  uint64_t queued_ns = 0;         // when the tick was queued (watchdog)
};

constexpr int kStages = 4;

}  // namespace

struct tq_server {
  const tq_db *db = nullptr;
  int device = 0;
  tq_serve_cfg cfg{};
  int S = 1;              // database segments
  int64_t seg_tiles = 0;  // tiles per segment
  int k_run = 0;          // width of the running lists (= cfg.max_k)
  int qtile = 16, grid = 512;
  size_t per_query_bytes = 0;
  hipStream_t stream = nullptr;

  // device
  uint32_t *d_qcanon = nullptr;  // max_slots x 2W
  uint32_t *d_qrows = nullptr;   // max_slots x 8 nc, by slot
  uint32_t *d_qtick = nullptr;   // max_slots x 8 nc, the active rows of a tick, compact
  uint64_t *d_running = nullptr; // max_slots x k_run
  uint64_t *d_partial = nullptr; // (qtile * grid + max_slots) x k_run
  uint64_t *d_mid = nullptr;     // first-stage merge results
  uint64_t *d_bound = nullptr;   // per (query, part, wave) published keys of a tick
  char *d_tick = nullptr;        // [BatchParams][slots: max_slots ints][retire: max_slots ints]
  tqi::BatchParams *d_prm = nullptr;
  int *d_slots = nullptr;
  int *d_retire = nullptr;
  int32_t *d_ids = nullptr, *d_scores = nullptr;  // max_slots x k_run
  // pinned host
  uint32_t *h_qcanon = nullptr;
  int32_t *h_ids = nullptr, *h_scores = nullptr;
  TickStage stage[kStages];
  int next_stage = 0;
  std::vector<hipEvent_t> event_pool;

  // host state (guarded by mu)
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::vector<Request *> active;
  std::unordered_map<uint64_t, Request *> reqs;
  std::vector<char> slot_used;
  size_t bytes_in_use = 0;
  uint64_t next_ticket = 1;
  uint64_t n_submitted = 0, n_completed = 0;
  std::atomic<uint64_t> n_ticks{0};
  bool stopping = false;
  int loop_error = TQ_OK;
  char loop_msg[160] = "";  // why the loop stopped
  std::thread th;
  int64_t tick = 0;
};

namespace {

int first_fit(tq_server *s, int nq) {
  const int M = static_cast<int>(s->slot_used.size());
  int run = 0;
  for (int i = 0; i < M; ++i) {
    run = s->slot_used[i] ? 0 : run + 1;
    if (run == nq) return i - nq + 1;
  }
  return -1;
}

void set_slots(tq_server *s, int slot0, int nq, char v) {
  for (int i = 0; i < nq; ++i) s->slot_used[slot0 + i] = v;
}

hipEvent_t take_event(tq_server *s) {
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void release_request_locked(tq_server *s, Request *r) {
  if (r->slot0 >= 0) set_slots(s, r->slot0, r->nq, 0);
  r->slot0 = -1;
  s->bytes_in_use -= r->bytes;
  r->bytes = 0;
}

struct Admitted {
  Request *r;
};

struct TickPlan {
  int k = 1;                   // largest k of the active requests
  std::vector<Admitted> admitted;
  std::vector<int> slots;      // rows of every active query
  std::vector<int> retire;     // rows of queries that retire after this tick
  std::vector<Request *> retiring;
  int64_t seg = 0;
};

// Enqueue one tick on the server stream using staging slot `st`.
hipError_t enqueue_tick(tq_server *s, TickPlan &p, TickStage &st) {
  const tqi::DbDev &db = s->db->dev;
  const int W = db.W;
  hipError_t e = hipSuccess;
  // newly admitted requests: codes to the device, scan rows, cleared lists
  for (auto &a : p.admitted) {
    Request *r = a.r;
    const size_t off = static_cast<size_t>(r->slot0) * 2 * W;
    e = hipMemcpyAsync(s->d_qcanon + off, s->h_qcanon + off, static_cast<size_t>(r->nq) * 2 * W * sizeof(uint32_t),
                       hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return e;
    e = tqi::prep_rows_launch(s->d_qcanon + off, r->nq, db, s->d_qrows + static_cast<size_t>(r->slot0) * 8 * db.nc,
                              s->stream);
    if (e != hipSuccess) return e;
    e = tqi::fill_zero_launch(s->d_running + static_cast<size_t>(r->slot0) * s->k_run,
                              static_cast<int64_t>(r->nq) * s->k_run, s->stream);
    if (e != hipSuccess) return e;
  }
  // stage the tick's parameters and slot lists
  if (st.used) {
    e = hipEventSynchronize(st.consumed);
    if (e != hipSuccess) return e;
  }
  const int nq = static_cast<int>(p.slots.size());
  const int nret = static_cast<int>(p.retire.size());
  const int kt = p.k;  // the tick's k: the largest k of the active requests
  const int nq_all = static_cast<int>(p.slots.size());
  const int engine = s->cfg.engine == TQ_ENGINE_AUTO ? default_engine(kt, nq_all) : s->cfg.engine;
  const bool matrix = engine == TQ_ENGINE_MATRIX && tqi::rows_for_k(kt) <= 2;
  const int qtile = matrix ? 64 : std::min(s->qtile, tqi::batched_max_qtile(kt));
  tqi::BatchParams b;
  const int64_t lo = p.seg * s->seg_tiles;
  const int64_t hi = std::min<int64_t>(db.ntiles, lo + s->seg_tiles);
  tqi::batch_split(b, nq, qtile, s->grid, lo, hi);
  b.slots = s->d_slots;
  b.running = s->d_running;
  b.running_stride = s->k_run;
  b.ids = nullptr;
  b.scores = nullptr;
  b.bound = s->d_bound;  // (zeroed below, before the scan)
  const size_t max_slots = s->slot_used.size();
  std::memcpy(st.host, &b, sizeof b);
  std::memcpy(st.host + sizeof b, p.slots.data(), nq * sizeof(int));
  std::memcpy(st.host + sizeof b + max_slots * sizeof(int), p.retire.data(), nret * sizeof(int));
  // one copy: parameters, active slots and (up to the used part) retiring slots
  const size_t span = sizeof b + (nret ? max_slots + nret : static_cast<size_t>(nq)) * sizeof(int);
  e = hipMemcpyAsync(s->d_tick, st.host, span, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipEventRecord(st.consumed, s->stream);
  if (e != hipSuccess) return e;
  st.used = true;
  // scan the segment for every active query and fold it into the running lists
  e = tqi::gather_rows_launch(s->d_qrows, s->d_slots, nq, 8 * db.nc, s->d_qtick, s->stream);
  if (e == hipSuccess)
    e = tqi::fill_zero_launch(s->d_bound, static_cast<int64_t>(nq) * b.parts * tqi::kBoundSlotsPerPart, s->stream);
  if (e != hipSuccess) return e;
  {
    TimedLaunch t(kTimeBatched, s->stream);
    e = matrix ? tqi::scan_mfma_launch(db, s->d_qtick, s->d_prm, kt, qtile, s->grid, b.tiles_per_part, s->d_partial,
                                       s->stream)
               : tqi::scan_batched_launch(db, s->d_qtick, s->d_prm, kt, qtile, s->grid, s->d_partial, s->stream);
  }
  if (e != hipSuccess) return e;
  e = tqi::merge_batched_launch(s->d_partial, s->d_prm, nq, kt, tqi::batch_max_parts(s->grid), s->d_mid,
                                s->stream);
  if (e != hipSuccess) return e;
  // retiring requests: results to pinned host memory
  if (nret) {
    e = tqi::running_results_launch(s->d_running, s->d_retire, nret, s->k_run, s->d_ids, s->d_scores, s->stream);
    if (e != hipSuccess) return e;
    for (Request *r : p.retiring) {
      const size_t off = static_cast<size_t>(r->slot0) * s->k_run;
      const size_t bytes = static_cast<size_t>(r->nq) * s->k_run * sizeof(int32_t);
      e = hipMemcpyAsync(s->h_ids + off, s->d_ids + off, bytes, hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_scores + off, s->d_scores + off, bytes, hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess) e = hipEventRecord(r->done, s->stream);
      if (e != hipSuccess) return e;
    }
  }
  return hipEventRecord(st.done, s->stream);
}

// Finish requests whose results have landed (non-blocking unless `wait`).
void collect_finished_locked(tq_server *s, std::vector<Request *> &finishing, bool wait_all) {
  for (size_t i = 0; i < finishing.size();) {
    Request *r = finishing[i];
    hipError_t q = wait_all ? hipEventSynchronize(r->done) : hipEventQuery(r->done);
    if (q == hipErrorNotReady) {
      ++i;
      continue;
    }
    if (q != hipSuccess) {
      s->loop_error = TQ_ERR_DEVICE;
      std::snprintf(s->loop_msg, sizeof s->loop_msg, "device error: %s", hipGetErrorString(q));
    }
    const uint64_t t = now_ns();
    r->ids.resize(static_cast<size_t>(r->nq) * r->k);
    r->scores.resize(r->ids.size());
    for (int qi = 0; qi < r->nq; ++qi) {
      const size_t src = static_cast<size_t>(r->slot0 + qi) * s->k_run;
      std::memcpy(&r->ids[static_cast<size_t>(qi) * r->k], s->h_ids + src, r->k * sizeof(int32_t));
      std::memcpy(&r->scores[static_cast<size_t>(qi) * r->k], s->h_scores + src, r->k * sizeof(int32_t));
    }
    s->event_pool.push_back(r->done);
    r->done = nullptr;
    release_request_locked(s, r);
    if (r->cancel) {
      s->reqs.erase(r->ticket);
      delete r;
    } else {
      r->complete_ns = t;
      r->state = RState::Done;
      s->n_completed++;
    }
    finishing[i] = finishing.back();
    finishing.pop_back();
  }
  s->cv_done.notify_all();
}

// Waits for `ev`.  Without a watchdog this blocks in the runtime; with one it
// polls and gives up once `queued_ns` + the timeout has passed, returning
// hipErrorNotReady (the event's state at that moment).  The GPU work itself is left to finish: the caller stops the loop
// and the drain waits for the stream.
hipError_t wait_tick(const tq_server *s, hipEvent_t ev, uint64_t queued_ns) {
  if (s->cfg.tick_timeout_us <= 0) return hipEventSynchronize(ev);
  const uint64_t deadline = queued_ns + static_cast<uint64_t>(s->cfg.tick_timeout_us) * 1000ull;
  for (;;) {
    const hipError_t q = hipEventQuery(ev);
    if (q != hipErrorNotReady) return q;
    if (now_ns() > deadline) return hipErrorNotReady;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

void stop_loop_locked(tq_server *s, hipError_t e) {
  s->loop_error = TQ_ERR_DEVICE;
  if (e == hipErrorNotReady)
    std::snprintf(s->loop_msg, sizeof s->loop_msg, "tick watchdog: a tick was not done %d us after it was queued",
                  s->cfg.tick_timeout_us);
  else
    std::snprintf(s->loop_msg, sizeof s->loop_msg, "device error: %s", hipGetErrorString(e));
  s->stopping = true;
}

void serve_loop(tq_server *s) {
  (void)hipSetDevice(s->device);
  std::vector<Request *> finishing;
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // retire cancelled active requests (safe: later device work is stream ordered)
    for (size_t i = 0; i < s->active.size();) {
      Request *r = s->active[i];
      if (r->cancel) {
        release_request_locked(s, r);
        if (r->done) s->event_pool.push_back(r->done);
        s->reqs.erase(r->ticket);
        delete r;
        s->active[i] = s->active.back();
        s->active.pop_back();
      } else {
        ++i;
      }
    }
    TickPlan plan;
    // admission in arrival order
    while (!s->stopping && !s->pending.empty() && s->loop_error == TQ_OK) {
      Request *r = s->pending.front();
      if (s->bytes_in_use + r->bytes > s->cfg.budget_bytes) break;
      const int slot0 = first_fit(s, r->nq);
      if (slot0 < 0) break;
      s->pending.pop_front();
      r->slot0 = slot0;
      set_slots(s, slot0, r->nq, 1);
      s->bytes_in_use += r->bytes;
      r->state = RState::Active;
      r->admit_ns = now_ns();
      r->done = take_event(s);
      std::memcpy(s->h_qcanon + static_cast<size_t>(slot0) * 2 * s->db->dev.W, r->qcodes.data(),
                  r->qcodes.size() * sizeof(uint32_t));
      s->active.push_back(r);
      plan.admitted.push_back({r});
    }
    if (s->active.empty()) {
      if (!finishing.empty()) {
        lk.unlock();
        const hipError_t we = wait_tick(s, finishing.front()->done, finishing.front()->last_tick_ns);
        lk.lock();
        if (we != hipSuccess) {  // in-flight requests report it from poll / wait
          stop_loop_locked(s, we);
          break;
        }
        collect_finished_locked(s, finishing, false);
        continue;
      }
      if (s->stopping) break;
      s->cv_work.wait(lk);
      continue;
    }
    plan.seg = s->tick % s->S;
    for (Request *r : s->active) {
      plan.k = std::max(plan.k, r->k);
      for (int qi = 0; qi < r->nq; ++qi) plan.slots.push_back(r->slot0 + qi);
      if (r->ticks_done + 1 == s->S) {
        for (int qi = 0; qi < r->nq; ++qi) plan.retire.push_back(r->slot0 + qi);
        plan.retiring.push_back(r);
      }
    }
    const int cur = s->next_stage;
    s->next_stage = (cur + 1) % kStages;
    const uint64_t queued = now_ns();
    for (Request *r : plan.retiring) r->last_tick_ns = queued;
    lk.unlock();
    s->stage[cur].queued_ns = queued;
    hipError_t e = enqueue_tick(s, plan, s->stage[cur]);
    // at most two ticks in flight: wait for the previous one before planning
    // the next (the GPU keeps working on this one meanwhile)
    TickStage &prev = s->stage[(cur + kStages - 1) % kStages];
    if (e == hipSuccess && prev.used) e = wait_tick(s, prev.done, prev.queued_ns);
    lk.lock();
    if (e != hipSuccess) {  // requests in flight report the error from poll / wait
      stop_loop_locked(s, e);
      break;
    }
    s->tick++;
    s->n_ticks++;
    for (Request *r : s->active) r->ticks_done++;
    for (Request *r : plan.retiring) {
      r->state = RState::Finishing;
      s->active.erase(std::find(s->active.begin(), s->active.end(), r));
      finishing.push_back(r);
    }
    collect_finished_locked(s, finishing, false);
  }
  // drain
  lk.unlock();
  (void)hipStreamSynchronize(s->stream);
  lk.lock();
  if (s->loop_error == TQ_OK) collect_finished_locked(s, finishing, true);
  s->cv_done.notify_all();
}

void free_server(tq_server *s) {
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (void *p : {(void *)s->d_qcanon, (void *)s->d_qrows, (void *)s->d_qtick, (void *)s->d_running, (void *)s->d_partial,
                  (void *)s->d_mid, (void *)s->d_bound, (void *)s->d_tick, (void *)s->d_ids, (void *)s->d_scores})
    if (p) dev_free(p);
  for (void *p : {(void *)s->h_qcanon, (void *)s->h_ids, (void *)s->h_scores})
    if (p) (void)hipHostFree(p);
  for (auto &st : s->stage) {
    if (st.host) (void)hipHostFree(st.host);
    if (st.consumed) (void)hipEventDestroy(st.consumed);
    if (st.done) (void)hipEventDestroy(st.done);
  }
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  for (auto &kv : s->reqs) {
    if (kv.second->done) (void)hipEventDestroy(kv.second->done);
    delete kv.second;
  }
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // namespace

extern "C" {

int tq_serve_create(const tq_db *db, const tq_serve_cfg *cfg, tq_server **out) {
  clear_error();
  if (!out) return fail(TQ_ERR_INVALID, "null out");
  *out = nullptr;
  if (!db) return fail(TQ_ERR_INVALID, "null db");
  tq_serve_cfg c = cfg ? *cfg : tq_serve_cfg{};
  if (c.budget_bytes == 0) c.budget_bytes = uint64_t(256) << 20;
  if (c.max_slots == 0) c.max_slots = 4096;
  if (c.max_k == 0) c.max_k = 128;
  if (c.max_request_nq == 0) c.max_request_nq = 1024;
  if (c.max_slots < 1 || c.max_slots > (1 << 20)) return fail(TQ_ERR_INVALID, "max_slots=%d", c.max_slots);
  if (c.max_k < 1 || c.max_k > TQ_MAX_K || c.max_k > db->dev.n)
    return fail(TQ_ERR_INVALID, "max_k=%d outside [1, min(n, %d)]", c.max_k, TQ_MAX_K);
  if (c.max_request_nq < 1) return fail(TQ_ERR_INVALID, "max_request_nq=%d", c.max_request_nq);
  if (c.n_segments < 0) return fail(TQ_ERR_INVALID, "n_segments=%d", c.n_segments);
  if (c.tick_timeout_us < 0) return fail(TQ_ERR_INVALID, "tick_timeout_us=%d", c.tick_timeout_us);
  if (c.engine != TQ_ENGINE_AUTO && c.engine != TQ_ENGINE_POPCOUNT && c.engine != TQ_ENGINE_MATRIX)
    return fail(TQ_ERR_INVALID, "engine=%d: serving takes AUTO, POPCOUNT or MATRIX", c.engine);

  tq_server *s = new (std::nothrow) tq_server();
  if (!s) return fail(TQ_ERR_NOMEM, "host allocation");
  s->db = db;
  s->device = db->device;
  s->cfg = c;
  s->k_run = c.max_k;
  s->qtile = tqi::batched_max_qtile(s->k_run);
  s->grid = (db->num_cu > 0 ? db->num_cu : 256) * 2;
  const int64_t ntiles = db->dev.ntiles;
  int S = c.n_segments;
  // default: one segment per 16M vectors -- a full pass per tick keeps the
  // per-tick launch and merge overhead small next to the scan
  if (S == 0) S = static_cast<int>(std::min<int64_t>(64, std::max<int64_t>(1, (db->dev.n + (1 << 24) - 1) >> 24)));
  S = static_cast<int>(std::min<int64_t>(S, ntiles));
  s->seg_tiles = (ntiles + S - 1) / S;
  s->S = static_cast<int>((ntiles + s->seg_tiles - 1) / s->seg_tiles);
  s->cfg.n_segments = s->S;
  const int W = db->dev.W, nc = db->dev.nc;
  s->per_query_bytes = static_cast<size_t>(2 * W + 16 * nc) * sizeof(uint32_t) +
                       static_cast<size_t>(s->k_run) * (sizeof(uint64_t) + 2 * sizeof(int32_t));
  s->slot_used.assign(c.max_slots, 0);

  DeviceGuard g(db->device);
  const size_t M = c.max_slots;
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  auto dm = [&](void **p, size_t bytes) {
    if (e == hipSuccess) e = dev_malloc_raw(p, bytes);
  };
  auto hm = [&](void **p, size_t bytes) {
    if (e == hipSuccess) e = hipHostMalloc(p, bytes, hipHostMallocDefault);
  };
  dm((void **)&s->d_qcanon, M * 2 * W * sizeof(uint32_t));
  dm((void **)&s->d_qrows, M * 8 * nc * sizeof(uint32_t));
  dm((void **)&s->d_qtick, M * 8 * nc * sizeof(uint32_t));
  dm((void **)&s->d_running, M * s->k_run * sizeof(uint64_t));
  // query tiles of up to 64 (matrix engine) or s->qtile (popcount engine)
  const size_t lists = tqi::batch_max_lists(std::max(64, s->qtile), s->grid, static_cast<int>(M));
  dm((void **)&s->d_partial, lists * s->k_run * sizeof(uint64_t));
  dm((void **)&s->d_bound, lists * tqi::kBoundSlotsPerPart * sizeof(uint64_t));
  int64_t mid_keys = 0;
  for (int k = 1; k <= s->k_run; ++k)
    mid_keys =
        std::max(mid_keys, tqi::merge_batched_mid_keys(static_cast<int>(M), tqi::batch_max_parts(s->grid), k));
  dm((void **)&s->d_mid, static_cast<size_t>(mid_keys) * sizeof(uint64_t));
  dm((void **)&s->d_tick, sizeof(tqi::BatchParams) + 2 * M * sizeof(int));
  if (e == hipSuccess) {
    s->d_prm = reinterpret_cast<tqi::BatchParams *>(s->d_tick);
    s->d_slots = reinterpret_cast<int *>(s->d_tick + sizeof(tqi::BatchParams));
    s->d_retire = s->d_slots + M;
  }
  dm((void **)&s->d_ids, M * s->k_run * sizeof(int32_t));
  dm((void **)&s->d_scores, M * s->k_run * sizeof(int32_t));
  hm((void **)&s->h_qcanon, M * 2 * W * sizeof(uint32_t));
  hm((void **)&s->h_ids, M * s->k_run * sizeof(int32_t));
  hm((void **)&s->h_scores, M * s->k_run * sizeof(int32_t));
  for (auto &st : s->stage) {
    hm((void **)&st.host, sizeof(tqi::BatchParams) + 2 * M * sizeof(int));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st.consumed, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    int rc = hip_fail(e, "server allocation");
    free_server(s);
    return rc;
  }
  try {
    s->th = std::thread(serve_loop, s);
  } catch (...) {
    free_server(s);
    return fail(TQ_ERR_NOMEM, "could not start the serve thread");
  }
  *out = s;
  return TQ_OK;
}

int tq_serve_submit(tq_server *s, const uint32_t *qcodes_host, int nq, int k, uint64_t *ticket) {
  clear_error();
  if (!s || !qcodes_host || !ticket) return fail(TQ_ERR_INVALID, "null server, codes or ticket");
  if (nq < 1 || nq > s->cfg.max_request_nq || nq > s->cfg.max_slots)
    return fail(TQ_ERR_INVALID, "nq=%d outside [1, %d]", nq, std::min(s->cfg.max_request_nq, s->cfg.max_slots));
  if (k < 1 || k > s->k_run) return fail(TQ_ERR_INVALID, "k=%d outside [1, max_k=%d]", k, s->k_run);
  const size_t bytes = static_cast<size_t>(nq) * s->per_query_bytes;
  if (bytes > s->cfg.budget_bytes)
    return fail(TQ_ERR_INVALID, "request needs %zu device bytes, budget is %llu", bytes,
                (unsigned long long)s->cfg.budget_bytes);
  Request *r = new (std::nothrow) Request();
  if (!r) return fail(TQ_ERR_NOMEM, "host allocation");
  r->nq = nq;
  r->k = k;
  r->bytes = bytes;
  r->qcodes.assign(qcodes_host, qcodes_host + static_cast<size_t>(nq) * 2 * s->db->dev.W);
  r->submit_ns = now_ns();
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stopping) {
      delete r;
      return fail(TQ_ERR_STATE, "server is shutting down");
    }
    r->ticket = s->next_ticket++;
    s->reqs[r->ticket] = r;
    s->pending.push_back(r);
    s->n_submitted++;
    *ticket = r->ticket;
  }
  s->cv_work.notify_one();
  return TQ_OK;
}

static int collect_locked(tq_server *s, Request *r, int32_t *ids, int32_t *scores, tq_req_stats *st) {
  if (ids) std::memcpy(ids, r->ids.data(), r->ids.size() * sizeof(int32_t));
  if (scores) std::memcpy(scores, r->scores.data(), r->scores.size() * sizeof(int32_t));
  if (st) {
    st->submit_ns = r->submit_ns;
    st->admit_ns = r->admit_ns;
    st->complete_ns = r->complete_ns;
    st->nq = r->nq;
    st->k = r->k;
    st->ticks = r->ticks_done;
    st->reserved = 0;
  }
  s->reqs.erase(r->ticket);
  delete r;
  return TQ_OK;
}

int tq_serve_poll(tq_server *s, uint64_t ticket, int32_t *ids, int32_t *scores, tq_req_stats *st) {
  clear_error();
  if (!s) return fail(TQ_ERR_INVALID, "null server");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->cancel) return fail(TQ_ERR_NOTFOUND, "unknown ticket %llu",
                                                             (unsigned long long)ticket);
  Request *r = it->second;
  if (r->state != RState::Done) {
    if (s->loop_error) return fail(s->loop_error, "the serve loop stopped: %s", s->loop_msg);
    return TQ_ERR_AGAIN;
  }
  return collect_locked(s, r, ids, scores, st);
}

int tq_serve_wait(tq_server *s, uint64_t ticket, int timeout_ms, int32_t *ids, int32_t *scores, tq_req_stats *st) {
  clear_error();
  if (!s) return fail(TQ_ERR_INVALID, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
  for (;;) {
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second->cancel)
      return fail(TQ_ERR_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Request *r = it->second;
    if (r->state == RState::Done) return collect_locked(s, r, ids, scores, st);
    if (s->loop_error) return fail(s->loop_error, "the serve loop stopped: %s", s->loop_msg);
    if (timeout_ms < 0) {
      s->cv_done.wait(lk);
    } else if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
      auto it2 = s->reqs.find(ticket);
      if (it2 != s->reqs.end() && it2->second->state == RState::Done && !it2->second->cancel)
        return collect_locked(s, it2->second, ids, scores, st);
      return TQ_ERR_AGAIN;
    }
  }
}

int tq_serve_cancel(tq_server *s, uint64_t ticket) {
  clear_error();
  if (!s) return fail(TQ_ERR_INVALID, "null server");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second->cancel)
    return fail(TQ_ERR_NOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request *r = it->second;
  switch (r->state) {
    case RState::Pending:
      s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
      s->reqs.erase(ticket);
      delete r;
      break;
    case RState::Done:
      s->reqs.erase(ticket);
      delete r;
      break;
    default:  // admitted: the loop frees it at the next tick boundary / completion
      r->cancel = true;
      break;
  }
  return TQ_OK;
}

int tq_serve_stats(tq_server *s, uint64_t *submitted, uint64_t *completed, uint64_t *ticks,
                   uint64_t *bytes_in_use) {
  clear_error();
  if (!s) return fail(TQ_ERR_INVALID, "null server");
  std::lock_guard<std::mutex> g(s->mu);
  if (submitted) *submitted = s->n_submitted;
  if (completed) *completed = s->n_completed;
  if (ticks) *ticks = s->n_ticks.load();
  if (bytes_in_use) *bytes_in_use = s->bytes_in_use;
  return TQ_OK;
}

int tq_serve_destroy(tq_server *s) {
  clear_error();
  if (!s) return TQ_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
    for (Request *r : s->pending) {
      s->reqs.erase(r->ticket);
      delete r;
    }
    s->pending.clear();
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  DeviceGuard g(s->device);
  free_server(s);
  return TQ_OK;
}

}  // extern "C"
