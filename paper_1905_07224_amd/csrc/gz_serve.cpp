// Serving loop over the two-pass path: jobs (a compressed input already in
// device memory, and an output buffer) are queued, admitted into batches
// while their footprints (input, output and workspace) fit in the HBM budget
// and their workspaces fit in the caller's device arena, and run as batched
// launch sequences on a few streams at once; a batch that finishes frees its
// arena block and its share of the budget for the jobs queued behind it.
// The library allocates no device memory here.  See include/gzgpu.h.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "../../include/gzgpu.h"

// internal to the library (gz_api.cpp): sizing without a plan object, and
// re-planning a finished plan in place (no pinned memory allocated or freed,
// which could wait for the device while other batches run)
extern "C" int gzi_plan_ws(const gz_job *jobs, int n, const gz_opts *opts, uint64_t *ws_bytes);
extern "C" int gzi_replan(gz_plan_t *plan, const gz_job *jobs, int n, const gz_opts *opts);

namespace {

constexpr uint64_t ALIGN = 256;

// First-fit allocator over [0, size) in ALIGN units, adjacent free blocks merged.
struct Arena {
  uint64_t size = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  uint64_t used = 0, peak = 0;
  void init(uint64_t n) {
    size = n / ALIGN * ALIGN;
    free_.clear();
    if (size) free_[0] = size;
    used = peak = 0;
  }
  uint64_t largest() const {
    uint64_t m = 0;
    for (auto &f : free_) m = std::max(m, f.second);
    return m;
  }
  bool alloc(uint64_t n, uint64_t *off) {
    n = (n + ALIGN - 1) / ALIGN * ALIGN;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used += n;
        peak = std::max(peak, used);
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = (n + ALIGN - 1) / ALIGN * ALIGN;
    used -= n;
    auto it = free_.emplace(off, n).first;
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

struct Job {
  const void *comp;
  uint64_t comp_len;
  void *out;
  uint64_t out_cap;
  uint64_t tag;
  uint64_t ws;       // workspace of this job planned alone (admission estimate)
  uint64_t foot() const { return comp_len + out_cap + ws; }  // device bytes while it is in flight
  uint32_t factor;   // symbol capacity factor (raised after a capacity failure)
  bool waited = false;  // its admission waited for the budget or the arena
  double t_submit;
  double t_start;
};

struct Batch {
  gz_plan_t plan = nullptr;
  std::vector<Job> jobs;
  uint64_t off = 0, bytes = 0;
  uint64_t foot = 0;  // inputs + outputs + the batch's workspace
  int slot = 0;
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct gz_server_s {
  gz_server_opts o{};
  std::chrono::steady_clock::time_point t0;
  uint8_t *base = nullptr;
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<bool> busy;
  std::vector<gz_plan_t> plans;  // one per stream, re-planned for each batch it runs
  std::deque<Job> queue;
  std::vector<Batch> running;
  std::vector<gz_done> done;  // finished, not yet returned by poll
  uint64_t n_batches = 0;
  uint64_t resident = 0, resident_peak = 0;  // footprint of the batches in flight
  uint32_t mem_waited = 0;  // jobs whose admission waited for memory
};

namespace {

int plan_ws(const Job &j, const gz_opts &base, uint64_t *ws) {
  gz_opts o = base;
  o.sym_factor = j.factor;
  o.timing = 0;
  gz_job g{};
  g.d_comp = j.comp;
  g.comp_len = j.comp_len;
  return gzi_plan_ws(&g, 1, &o, ws);
}

void finish_job(gz_server_t s, const Job &j, int status, uint64_t out_len) {
  gz_done d{};
  d.tag = j.tag;
  d.status = status;
  d.out_len = out_len;
  d.t_submit = j.t_submit;
  d.t_start = j.t_start;
  d.t_end = now_s(s->t0);
  s->done.push_back(d);
}

// Reap every batch whose stream has passed its end event.
void reap(gz_server_t s) {
  for (size_t b = 0; b < s->running.size();) {
    Batch &B = s->running[b];
    const hipError_t q = hipEventQuery(s->events[B.slot]);
    if (q == hipErrorNotReady) {
      b++;
      continue;
    }
    for (size_t i = 0; i < B.jobs.size(); i++) {
      gz_result res;
      int r = q == hipSuccess ? gz_result_get(B.plan, (int)i, &res) : GZ_E_HIP;
      Job j = B.jobs[i];
      if (r == GZ_OK && res.status == GZ_E_CAPACITY && res.ws_needed && j.factor < 4096) {
        // more symbols than planned: queued again at the front with more room
        j.factor *= 4;
        if (plan_ws(j, s->o.opts, &j.ws) == GZ_OK) {
          s->queue.push_front(j);
          continue;
        }
      }
      finish_job(s, j, r == GZ_OK ? res.status : r, r == GZ_OK ? res.out_len : 0);
    }
    // the plan stays with its stream for the next batch
    s->arena.release(B.off, B.bytes);
    s->resident -= B.foot;
    s->busy[B.slot] = false;
    s->running.erase(s->running.begin() + (long)b);
  }
}

// The job at the head of the queue cannot start for want of memory.
void mark_waited(gz_server_t s) {
  Job &j = s->queue.front();
  if (!j.waited) {
    j.waited = true;
    s->mem_waited++;
  }
}

// Admit queued jobs, FIFO, while a stream is free and their workspaces fit.
int admit(gz_server_t s) {
  for (;;) {
    if (s->queue.empty()) return GZ_OK;
    int slot = -1;
    for (size_t k = 0; k < s->busy.size(); k++)
      if (!s->busy[k]) {
        slot = (int)k;
        break;
      }
    if (slot < 0) return GZ_OK;
    const uint64_t room = s->arena.largest();
    if (s->queue.front().ws + 4096 > s->arena.size || s->queue.front().foot() + 4096 > s->o.budget_bytes) {
      // larger than the whole arena or budget: it can never run
      Job j = s->queue.front();
      s->queue.pop_front();
      j.t_start = now_s(s->t0);
      finish_job(s, j, GZ_E_CAPACITY, 0);
      continue;
    }
    // the longest FIFO prefix whose summed workspaces fit the arena and whose
    // footprints fit what the budget has left (table overhead aside)
    const uint64_t left = s->o.budget_bytes - s->resident;
    size_t n = 0;
    uint64_t sum = 0, foot = 0;
    while (n < s->queue.size() && n < s->o.max_batch && sum + s->queue[n].ws + 4096 * (n + 1) <= room &&
           foot + s->queue[n].foot() + 4096 * (n + 1) <= left) {
      sum += s->queue[n].ws;
      foot += s->queue[n].foot();
      n++;
    }
    if (n == 0) {  // wait for memory
      mark_waited(s);
      return GZ_OK;
    }
    for (; n > 0; n--) {
      std::vector<gz_job> jobs(n);
      uint32_t factor = 0;
      for (size_t i = 0; i < n; i++) factor = std::max(factor, s->queue[i].factor);
      for (size_t i = 0; i < n; i++) {
        const Job &j = s->queue[i];
        jobs[i].d_comp = j.comp;
        jobs[i].comp_len = j.comp_len;
        jobs[i].n_chunks = 0;
        jobs[i].d_out = j.out;
        jobs[i].out_cap = j.out_cap;
      }
      gz_opts o = s->o.opts;
      o.sym_factor = factor;
      o.timing = 0;
      int r = gzi_replan(&s->plans[slot], jobs.data(), (int)n, &o);
      gz_plan_t p = s->plans[slot];
      if (r != GZ_OK) {
        if (n > 1) continue;
        Job j = s->queue.front();
        s->queue.pop_front();
        j.t_start = now_s(s->t0);
        finish_job(s, j, r, 0);
        break;
      }
      gz_info inf;
      gz_plan_info(p, &inf);
      uint64_t off = 0;
      if (!s->arena.alloc(inf.ws_bytes, &off)) {
        if (n > 1) continue;
        mark_waited(s);
        return GZ_OK;  // wait for memory
      }
      Batch B;
      B.plan = p;
      B.off = off;
      B.bytes = inf.ws_bytes;
      B.foot = inf.ws_bytes;
      B.slot = slot;
      const double t = now_s(s->t0);
      for (size_t i = 0; i < n; i++) {
        B.jobs.push_back(s->queue.front());
        B.jobs.back().t_start = t;
        B.foot += s->queue.front().comp_len + s->queue.front().out_cap;
        s->queue.pop_front();
      }
      r = gz_decompress_batch(p, s->base + off, inf.ws_bytes, s->streams[slot]);
      if (r == GZ_OK && hipEventRecord(s->events[slot], s->streams[slot]) != hipSuccess) r = GZ_E_HIP;
      if (r != GZ_OK) {
        for (const Job &j : B.jobs) finish_job(s, j, r, 0);
        s->arena.release(off, inf.ws_bytes);
        return r;
      }
      s->resident += B.foot;
      s->resident_peak = std::max(s->resident_peak, s->resident);
      s->busy[slot] = true;
      s->running.push_back(std::move(B));
      s->n_batches++;
      break;
    }
  }
}

}  // namespace

extern "C" {

int gz_server_create(gz_server_t *srv, const gz_server_opts *opts) {
  if (!srv) return GZ_E_ARG;
  *srv = nullptr;
  gz_server_t s = new (std::nothrow) gz_server_s();
  if (!s) return GZ_E_ARG;
  if (!opts || !opts->arena || opts->arena_bytes < 4096 || ((uintptr_t)opts->arena & (ALIGN - 1))) {
    delete s;
    return GZ_E_ARG;
  }
  s->o = *opts;
  if (!s->o.budget_bytes) s->o.budget_bytes = s->o.arena_bytes;
  if (!s->o.max_inflight) s->o.max_inflight = 4;
  if (!s->o.max_batch) s->o.max_batch = 64;
  if (!s->o.opts.sym_factor) s->o.opts.sym_factor = 8;
  s->t0 = std::chrono::steady_clock::now();
  s->base = (uint8_t *)s->o.arena;
  s->arena.init(s->o.arena_bytes);
  for (uint32_t k = 0; k < s->o.max_inflight; k++) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    // default priority, non-blocking with respect to the null stream
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      gz_server_destroy(s);
      return GZ_E_HIP;
    }
    s->streams.push_back(st);
    s->events.push_back(ev);
    s->busy.push_back(false);
    s->plans.push_back(nullptr);
  }
  *srv = s;
  return GZ_OK;
}

int gz_server_submit(gz_server_t s, const void *d_comp, size_t comp_len, void *d_out, size_t out_cap, uint64_t tag) {
  if (!s || !d_comp || !comp_len || (!d_out && out_cap)) return GZ_E_ARG;
  Job j{};
  j.comp = d_comp;
  j.comp_len = comp_len;
  j.out = d_out;
  j.out_cap = out_cap;
  j.tag = tag;
  j.factor = s->o.opts.sym_factor;
  j.t_submit = now_s(s->t0);
  const int r = plan_ws(j, s->o.opts, &j.ws);
  if (r != GZ_OK) return r;
  s->queue.push_back(j);
  return GZ_OK;
}

int gz_server_poll(gz_server_t s, gz_done *out, int max_done) {
  if (!s || max_done < 0 || (!out && max_done)) return GZ_E_ARG;
  reap(s);
  const int r = admit(s);
  const int n = (int)std::min<size_t>((size_t)max_done, s->done.size());
  for (int i = 0; i < n; i++) out[i] = s->done[i];
  s->done.erase(s->done.begin(), s->done.begin() + n);
  return r != GZ_OK ? r : n;
}

int gz_server_stats(gz_server_t s, gz_server_info *info) {
  if (!s || !info) return GZ_E_ARG;
  memset(info, 0, sizeof(*info));
  info->queued = (uint32_t)s->queue.size();
  uint32_t run = 0;
  for (const Batch &B : s->running) run += (uint32_t)B.jobs.size();
  info->running = run;
  info->finished_unread = (uint32_t)s->done.size();
  info->batches = s->n_batches;
  info->arena_bytes = s->arena.size;
  info->arena_used = s->arena.used;
  info->arena_peak = s->arena.peak;
  info->budget_bytes = s->o.budget_bytes;
  info->mem_waited = s->mem_waited;
  info->resident = s->resident;
  info->resident_peak = s->resident_peak;
  info->now = now_s(s->t0);
  return GZ_OK;
}

void gz_server_destroy(gz_server_t s) {
  if (!s) return;
  for (size_t k = 0; k < s->streams.size(); k++) (void)hipStreamSynchronize(s->streams[k]);
  for (gz_plan_t p : s->plans) gz_plan_destroy(p);
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
}

}  // extern "C"
