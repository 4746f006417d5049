// Solve server: continuous batching of D^dag D solves on one GPU.
//
// Requests are admitted FIFO while a slot is free and their footprint (the
// per-request workspace) fits in the caller's device pool.  A worker thread
// runs one engine over every admitted request: each poll block is one launch
// per CG phase across all of them (uneven lattices in one grid).  Between
// blocks finished requests leave (solution exported, memory and slot freed)
// and queued ones join, so work that arrives while others run overlaps on the
// device.  Gauge stores belong to the caller's lattices and stay resident.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "wd_host.h"

using namespace wd;

namespace {

constexpr int kMaxRhsPerRequest = 16;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing.
struct Arena {
  std::map<size_t, size_t> free_;  // offset -> length
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t len, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        *off = it->first;
        const size_t rest = it->second - len;
        const size_t noff = it->first + len;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t len) {
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct wd_server_s {
  char* pool = nullptr;
  size_t pool_bytes = 0;
  size_t data_off = 0;  // allocatable region starts here
  int max_slots = 0;
  wd_solve_params p{};
  hipStream_t stream = nullptr;
  int device = 0;
  RhsState* states = nullptr;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<EItem*> queue;
  std::map<uint64_t, EItem*> tickets;  // every live ticket
  std::map<uint64_t, bool> done;
  std::vector<char> slot_used;
  Arena arena;
  uint64_t next_ticket = 1;
  bool stop = false;
  wd_status fatal = WD_OK;
  std::string fatal_msg;
  std::thread worker;
};

static void finish_item_locked(wd_server_s* S, EItem* it) {
  S->done[it->ticket] = true;
  if (it->slot >= 0) S->slot_used[it->slot] = 0;
  if (it->pool_len) S->arena.release(it->pool_off - S->data_off, it->pool_len);
  it->slot = -1;
  it->pool_len = 0;
}

static void worker_main(wd_server_s* S) {
  (void)hipSetDevice(S->device);
  Engine eng(S->p, S->stream, S->states, nullptr);
  BlockPlanner plan;
  const size_t nst = (size_t)S->max_slots * kMaxRhsPerRequest;
  RhsState* hs = nullptr;
  hipEvent_t ev = nullptr;
  wd_status err = WD_OK;
  if (hipHostMalloc((void**)&hs, nst * sizeof(RhsState), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    err = fail(WD_EDEVICE, "server: cannot allocate poll buffers");
  }
  while (err == WD_OK) {
    std::vector<EItem*> admitted;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop && S->queue.empty() && eng.items.empty()) break;
      while (!S->queue.empty()) {
        EItem* it = S->queue.front();
        int slot = -1;
        for (int k = 0; k < S->max_slots; ++k)
          if (!S->slot_used[k]) {
            slot = k;
            break;
          }
        if (slot < 0) break;
        size_t off = 0;
        if (!S->arena.alloc(it->pool_len, &off)) break;  // FIFO: the head waits for memory
        S->queue.pop_front();
        S->slot_used[slot] = 1;
        it->slot = slot;
        it->pool_off = S->data_off + off;
        it->base = S->pool + it->pool_off;
        it->state_index = slot * kMaxRhsPerRequest;
        it->st = S->states + it->state_index;
        admitted.push_back(it);
      }
      if (eng.items.empty() && admitted.empty()) {
        S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
    }
    for (EItem* it : admitted) {
      if ((err = eng.start_item(it)) != WD_OK) break;
      eng.items.push_back(it);
      eng.set_changed();
      for (int r = 0; r < it->nrhs; ++r) {  // a new occupant of the slot: forget the old history
        const size_t q = (size_t)it->state_index + r;
        if (plan.snap.size() <= q) plan.snap.resize(q + 1, BlockPlanner::Snap{-1, 0.0, -1, 0.0});
        plan.snap[q] = BlockPlanner::Snap{-1, 0.0, -1, 0.0};
      }
    }
    if (err != WD_OK) break;
    // block size: up to the next expected event of any running request; new
    // requests start with a short block so that their rate is known early
    plan.kmax = eng.max_block();
    int K = admitted.empty() ? plan.kmax : std::min(plan.kmax, 4);
    if (admitted.empty() && !eng.items.empty()) {
      std::vector<int> idx;
      for (EItem* it : eng.items)
        for (int r = 0; r < it->nrhs; ++r) idx.push_back(it->state_index + r);
      const int k = plan.next(hs, idx.size(), 0, idx.data());
      K = k > 0 ? k : 1;
    }
    if ((err = eng.enqueue_block(K)) != WD_OK) break;
    if (hipMemcpyAsync(hs, S->states, nst * sizeof(RhsState), hipMemcpyDeviceToHost, S->stream) != hipSuccess ||
        hipEventRecord(ev, S->stream) != hipSuccess || hipEventSynchronize(ev) != hipSuccess) {
      err = fail(WD_EDEVICE, "server: state poll failed");
      break;
    }
    std::vector<EItem*> fin, keep;
    for (EItem* it : eng.items) {
      bool all = true;
      for (int r = 0; r < it->nrhs; ++r) {
        const int st = hs[it->state_index + r].state;
        all = all && (st == ST_DONE || st == ST_NOTCONV || st == ST_NONFINITE);
      }
      (all ? fin : keep).push_back(it);
    }
    if (fin.empty()) continue;
    for (EItem* it : fin)
      if ((err = eng.export_item(it)) != WD_OK) break;
    if (err != WD_OK) break;
    if (hipStreamSynchronize(S->stream) != hipSuccess) {
      err = fail(WD_EDEVICE, "server: export failed");
      break;
    }
    const double t = now_s();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (EItem* it : fin) {
        it->t_done = t;
        it->stats.resize(it->nrhs);
        for (int r = 0; r < it->nrhs; ++r)
          stats_from_state(hs[it->state_index + r], t - it->t_submit, nullptr, it->stats[r]);
        finish_item_locked(S, it);
      }
    }
    eng.items = keep;
    eng.set_changed();
    S->cv_done.notify_all();
  }
  if (err != WD_OK) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->fatal = err;
    S->fatal_msg = wd_last_error();
    auto mark = [&](EItem* it) {
      it->stats.assign(it->nrhs, wd_solve_stats{});
      for (auto& s : it->stats) s.status = err;
      finish_item_locked(S, it);
    };
    for (EItem* it : eng.items) mark(it);
    for (EItem* it : S->queue) mark(it);
    S->queue.clear();
    eng.items.clear();
  }
  (void)hipStreamSynchronize(S->stream);
  if (hs) (void)hipHostFree(hs);
  if (ev) (void)hipEventDestroy(ev);
  S->cv_done.notify_all();
}

extern "C" {

wd_status wd_server_create(wd_server* out, void* pool, size_t pool_bytes, int32_t max_slots,
                           const wd_solve_params* params, void* stream) {
  if (!out || !pool || !params) return fail(WD_EINVAL, "null argument");
  *out = nullptr;
  wd_status s = check_params(*params);
  if (s != WD_OK) return s;
  if (max_slots < 1 || max_slots > 1024) return fail(WD_EINVAL, "max_slots = %d out of range [1, 1024]", max_slots);
  const size_t hdr = states_bytes((size_t)max_slots * kMaxRhsPerRequest);
  if (pool_bytes <= hdr) return fail(WD_EBUFSIZE, "pool of %zu bytes cannot hold the state table (%zu)", pool_bytes, hdr);
  wd_server_s* S = new wd_server_s();
  S->pool = (char*)pool;
  S->pool_bytes = pool_bytes;
  S->data_off = hdr;
  S->max_slots = max_slots;
  S->p = *params;
  S->p.timing = 0;
  S->stream = (hipStream_t)stream;
  S->states = (RhsState*)pool;
  S->slot_used.assign(max_slots, 0);
  S->arena.reset(pool_bytes - hdr);
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return fail(WD_EDEVICE, "hipGetDevice failed");
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return WD_OK;
}

wd_status wd_server_destroy(wd_server S) {
  if (!S) return WD_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (auto& kv : S->tickets) delete kv.second;
  delete S;
  return WD_OK;
}

size_t wd_server_footprint(wd_server S, wd_lattice lat, int32_t nrhs) {
  if (!S || !lat || nrhs < 1) return 0;
  return align_up(item_layout(lat, S->p, nrhs).total);
}

wd_status wd_server_submit(wd_server S, wd_lattice lat, void* x, const void* b, int32_t nrhs, const double* kappa,
                           uint64_t* ticket) {
  if (!S || !lat || !x || !b || !kappa || !ticket) return fail(WD_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > kMaxRhsPerRequest) return fail(WD_EINVAL, "nrhs = %d out of range [1, %d]", nrhs, kMaxRhsPerRequest);
  if (!lat->store[F64].ptr) return fail(WD_ENOGAUGE, "the FP64 gauge store is needed for the true residual");
  if (!lat->store[S->p.inner].ptr) return fail(WD_ENOGAUGE, "no gauge store of the inner precision %d", S->p.inner);
  if (S->p.recon != 0 && lat->store[S->p.inner].recon != S->p.recon)
    return fail(WD_ENOGAUGE, "inner gauge store has recon %d, %d requested", lat->store[S->p.inner].recon, S->p.recon);
  for (int r = 0; r < nrhs; ++r)
    if (!std::isfinite(kappa[r])) return fail(WD_EINVAL, "kappa[%d] not finite", r);
  const size_t need = wd_server_footprint(S, lat, nrhs);
  if (need > S->pool_bytes - S->data_off)
    return fail(WD_EBUSY, "request footprint %zu exceeds the pool (%zu)", need, S->pool_bytes - S->data_off);
  EItem* it = new EItem();
  it->lat = lat;
  it->x = x;
  it->b = b;
  it->nrhs = nrhs;
  it->kappa.assign(kappa, kappa + nrhs);
  it->lay = item_layout(lat, S->p, nrhs);
  it->pool_len = need;
  it->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal != WD_OK) {
      delete it;
      return fail(S->fatal, "server stopped after an error: %s", S->fatal_msg.c_str());
    }
    it->ticket = S->next_ticket++;
    S->tickets[it->ticket] = it;
    S->done[it->ticket] = false;
    S->queue.push_back(it);
    *ticket = it->ticket;
  }
  S->cv_work.notify_all();
  return WD_OK;
}

static int32_t take_result_locked(wd_server S, uint64_t ticket, wd_solve_stats* stats) {
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return fail(WD_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
  if (!S->done[ticket]) return 0;
  EItem* e = it->second;
  if (stats)
    for (int r = 0; r < e->nrhs; ++r) stats[r] = e->stats[r];
  S->tickets.erase(it);
  S->done.erase(ticket);
  delete e;
  return 1;
}

int32_t wd_server_poll(wd_server S, uint64_t ticket, wd_solve_stats* stats) {
  if (!S) return fail(WD_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  return take_result_locked(S, ticket, stats);
}

int32_t wd_server_wait(wd_server S, uint64_t ticket, wd_solve_stats* stats, int32_t timeout_ms) {
  if (!S) return fail(WD_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto ready = [&] {
    auto d = S->done.find(ticket);
    return d == S->done.end() || d->second;
  };
  if (timeout_ms < 0) S->cv_done.wait(lk, ready);
  else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) return 0;
  return take_result_locked(S, ticket, stats);
}

}  // extern "C"
