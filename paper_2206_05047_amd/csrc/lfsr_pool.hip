// Serving pool of the C ABI (include/lfsr.h): admission of independent
// super-resolution jobs by device-memory budget, resident ADMM state, and one
// graph launch per tick that advances every active job by one iteration of
// sec 5 (Algorithms 1 and 2).
//
// Memory: the caller's arena is carved first-fit into 256-byte aligned job
// workspaces; freed blocks are coalesced with their neighbours.
// Scheduling: a job owns a slot (a branch stream and a pinned status record)
// from admission until it is harvested.  The per-tick graph forks from the
// pool's stream into one branch per active job (each branch is exactly the
// launch sequence of one lfsr_iterate on that job's handle) and joins back;
// it is captured again only after an admission or a retirement.
#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lfsr_handle.h"

using namespace lfsr;

namespace {

constexpr int kMaxPoolSlots = 64;
thread_local std::string g_pool_err = "no error";

size_t round256(size_t v) { return (v + 255) & ~(size_t)255; }

struct PoolJob {
  int64_t id = 0;
  int slot = -1;
  lfsr_handle* h = nullptr;
  size_t off = 0, bytes = 0;
  int ticks = 0, n_iter = 0;
  float* out = nullptr;
};

}  // namespace

struct lfsr_pool {
  char* arena = nullptr;
  size_t bytes = 0;
  int max_slots = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> size
  std::vector<PoolJob> active, retiring;
  std::vector<int> free_slots;
  hipStream_t main = nullptr;
  std::vector<hipStream_t> branch;   // per slot
  std::vector<hipEvent_t> join;      // per slot
  std::vector<hipEvent_t> done;      // per slot: result copy complete
  hipEvent_t ev_in = nullptr, ev_fork = nullptr, ev_out = nullptr;
  DevScalars* status = nullptr;      // pinned host, per slot
  hipGraphExec_t exec = nullptr;
  // replaced graphs whose launches may still run: destroyed once their event completes
  std::vector<std::pair<hipGraphExec_t, hipEvent_t>> graveyard;
  bool dirty = true;
  int64_t next_id = 1;
  std::string err = "no error";
};

namespace {

lfsr_status pool_err(lfsr_pool* p, lfsr_status st, const std::string& msg) {
  if (p) p->err = msg;
  else g_pool_err = msg;
  return st;
}

lfsr_status pool_hip(lfsr_pool* p, hipError_t e, const char* where) {
  if (e == hipSuccess) return LFSR_OK;
  return pool_err(p, LFSR_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool arena_take(lfsr_pool* p, size_t need, size_t* off) {
  for (auto it = p->free_blocks.begin(); it != p->free_blocks.end(); ++it) {
    if (it->second < need) continue;
    *off = it->first;
    const size_t rest = it->second - need;
    const size_t at = it->first + need;
    p->free_blocks.erase(it);
    if (rest > 0) p->free_blocks[at] = rest;
    return true;
  }
  return false;
}

void arena_give(lfsr_pool* p, size_t off, size_t size) {
  auto it = p->free_blocks.emplace(off, size).first;
  auto nx = std::next(it);
  if (nx != p->free_blocks.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    p->free_blocks.erase(nx);
  }
  if (it != p->free_blocks.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      p->free_blocks.erase(it);
    }
  }
}

void destroy_job(lfsr_pool* p, PoolJob& j) {
  lfsr_destroy(j.h);
  j.h = nullptr;
  arena_give(p, j.off, j.bytes);
  p->free_slots.push_back(j.slot);
}

// Destroy the replaced graphs whose last launch is known to have completed
// (all = true: wait for them).  Only a successful query or wait counts: a
// graph whose completion cannot be confirmed (not ready, or the runtime
// returned an error) is kept, and leaked at pool destruction rather than
// destroyed while a launch of it may still run.
void sweep_graveyard(lfsr_pool* p, bool all) {
  std::vector<std::pair<hipGraphExec_t, hipEvent_t>> keep;
  for (auto& ge : p->graveyard) {
    const hipError_t q = all ? hipEventSynchronize(ge.second) : hipEventQuery(ge.second);
    if (q != hipSuccess) {
      keep.push_back(ge);
      continue;
    }
    (void)hipGraphExecDestroy(ge.first);
    (void)hipEventDestroy(ge.second);
  }
  p->graveyard.swap(keep);
}

// Capture the per-tick graph: fork from the pool stream into one branch per
// active job, one ADMM iteration on each, join.  The graph it replaces may
// still be executing (ticks are not synchronised), so it is retired with an
// event recorded behind its last launch and destroyed later.
lfsr_status capture(lfsr_pool* p) {
  if (p->exec) {
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, p->main);
    if (e != hipSuccess) {
      if (ev) (void)hipEventDestroy(ev);
      return pool_hip(p, e, "lfsr_pool_tick retire graph");
    }
    p->graveyard.emplace_back(p->exec, ev);
    p->exec = nullptr;
  }
  sweep_graveyard(p, false);
  hipError_t e = hipStreamBeginCapture(p->main, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return pool_hip(p, e, "lfsr_pool_tick begin capture");
  lfsr_status st = LFSR_OK;
  e = hipEventRecord(p->ev_fork, p->main);
  for (size_t i = 0; i < p->active.size() && e == hipSuccess && st == LFSR_OK; ++i) {
    PoolJob& j = p->active[i];
    hipStream_t b = p->branch[j.slot];
    e = hipStreamWaitEvent(b, p->ev_fork, 0);
    if (e != hipSuccess) break;
    st = lfsr_iterate(j.h, 1, b);
    j.h->n_done -= 1;  // captured, not run
    if (st) {
      p->err = std::string("lfsr_pool_tick job ") + std::to_string(j.id) + ": " + j.h->err;
      break;
    }
    e = hipEventRecord(p->join[j.slot], b);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->main, p->join[j.slot], 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(p->main, &graph);
  if (st) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e == hipSuccess) e = ee;
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return pool_hip(p, e, "lfsr_pool_tick capture");
  p->dirty = false;
  return LFSR_OK;
}

}  // namespace

extern "C" {

lfsr_status lfsr_pool_create(void* d_arena, size_t bytes, int32_t max_slots, lfsr_pool** out) {
  if (!out) return pool_err(nullptr, LFSR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_arena || bytes == 0) return pool_err(nullptr, LFSR_ENOMEM, "arena is NULL or empty");
  if (((uintptr_t)d_arena & 255) != 0) return pool_err(nullptr, LFSR_EINVAL, "arena not 256-byte aligned");
  if (max_slots < 1 || max_slots > kMaxPoolSlots) return pool_err(nullptr, LFSR_EINVAL, "max_slots must be in 1..64");
  lfsr_pool* p = new (std::nothrow) lfsr_pool();
  if (!p) return pool_err(nullptr, LFSR_ENOMEM, "host allocation of the pool failed");
  p->arena = (char*)d_arena;
  p->bytes = bytes & ~(size_t)255;
  p->max_slots = max_slots;
  p->free_blocks[0] = p->bytes;
  hipError_t e = hipStreamCreateWithFlags(&p->main, hipStreamNonBlocking);
  p->branch.assign(max_slots, nullptr);
  p->join.assign(max_slots, nullptr);
  p->done.assign(max_slots, nullptr);
  for (int i = 0; i < max_slots && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&p->branch[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done[i], hipEventDisableTiming);
    p->free_slots.push_back(max_slots - 1 - i);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&p->status, sizeof(DevScalars) * max_slots, hipHostMallocDefault);
  if (e != hipSuccess) {
    const std::string msg = std::string("lfsr_pool_create: ") + hipGetErrorString(e);
    lfsr_pool_destroy(p);
    return pool_err(nullptr, LFSR_EDEVICE, msg);
  }
  *out = p;
  return LFSR_OK;
}

void lfsr_pool_destroy(lfsr_pool* p) {
  if (!p) return;
  if (p->main) (void)hipStreamSynchronize(p->main);
  sweep_graveyard(p, true);
  for (auto& j : p->active) lfsr_destroy(j.h);
  for (auto& j : p->retiring) lfsr_destroy(j.h);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  for (auto s : p->branch)
    if (s) (void)hipStreamDestroy(s);
  for (auto e : p->join)
    if (e) (void)hipEventDestroy(e);
  for (auto e : p->done)
    if (e) (void)hipEventDestroy(e);
  for (auto e : {p->ev_in, p->ev_fork, p->ev_out})
    if (e) (void)hipEventDestroy(e);
  if (p->main) (void)hipStreamDestroy(p->main);
  if (p->status) (void)hipHostFree(p->status);
  delete p;
}

const char* lfsr_pool_last_error(const lfsr_pool* p) { return p ? p->err.c_str() : g_pool_err.c_str(); }

lfsr_status lfsr_pool_submit(lfsr_pool* p, const lfsr_params* prm, const float* d_lr, const float* d_disp,
                             const float* d_occ, const float* d_x0, float* d_hr_out, void* hip_stream,
                             int64_t* job_id) {
  if (!p) return pool_err(nullptr, LFSR_EINVAL, "pool is NULL");
  if (!prm || !d_lr || !d_disp || !d_hr_out || !job_id)
    return pool_err(p, LFSR_EINVAL, "params, d_lr, d_disp, d_hr_out and job_id are required");
  const size_t need = lfsr_workspace_bytes(prm);
  if (need == 0) return pool_err(p, LFSR_EINVAL, std::string("invalid parameters: ") + lfsr_last_error(nullptr));
  const size_t take = round256(need);
  if (take > p->bytes) return pool_err(p, LFSR_ENOMEM, "job workspace larger than the whole arena");
  if (p->free_slots.empty()) return pool_err(p, LFSR_EBUSY, "no free slot");
  size_t off = 0;
  if (!arena_take(p, take, &off)) return pool_err(p, LFSR_EBUSY, "not enough free arena space");
  PoolJob j;
  j.slot = p->free_slots.back();
  j.off = off;
  j.bytes = take;
  j.n_iter = prm->admm_iters;
  j.out = d_hr_out;
  lfsr_status st = lfsr_create(prm, p->arena + off, take, &j.h);
  if (st) {
    arena_give(p, off, take);
    return pool_err(p, st, std::string("lfsr_create: ") + lfsr_last_error(nullptr));
  }
  // the job's setup runs on the pool stream, after the caller's pending work
  hipError_t e = hipEventRecord(p->ev_in, (hipStream_t)hip_stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->main, p->ev_in, 0);
  if (e != hipSuccess) {
    lfsr_destroy(j.h);
    arena_give(p, off, take);
    return pool_hip(p, e, "lfsr_pool_submit order");
  }
  st = lfsr_init(j.h, d_lr, d_disp, d_occ, d_x0, p->main);
  if (st) {
    const std::string msg = std::string("lfsr_init: ") + j.h->err;
    lfsr_destroy(j.h);
    arena_give(p, off, take);
    return pool_err(p, st, msg);
  }
  p->free_slots.pop_back();
  j.id = p->next_id++;
  *job_id = j.id;
  p->active.push_back(j);
  p->dirty = true;
  return LFSR_OK;
}

lfsr_status lfsr_pool_tick(lfsr_pool* p, void* hip_stream, int32_t* h_active) {
  if (!p) return pool_err(nullptr, LFSR_EINVAL, "pool is NULL");
  if (h_active) *h_active = (int32_t)p->active.size();
  if (p->active.empty()) return LFSR_OK;
  hipStream_t cs = (hipStream_t)hip_stream;
  hipError_t e = hipEventRecord(p->ev_in, cs);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->main, p->ev_in, 0);
  if (e != hipSuccess) return pool_hip(p, e, "lfsr_pool_tick order");
  if (p->dirty || !p->exec) {
    lfsr_status st = capture(p);
    if (st) return st;
  }
  e = hipGraphLaunch(p->exec, p->main);
  if (e != hipSuccess) return pool_hip(p, e, "lfsr_pool_tick launch");
  // retire the jobs that have run all their iterations.  A job is in exactly
  // one of active / retiring at every return, also after a failure (it then
  // stays active), so that destruction releases each handle once.
  std::vector<PoolJob> keep;
  keep.reserve(p->active.size());
  lfsr_status bad = LFSR_OK;
  for (PoolJob& j : p->active) {
    j.ticks += 1;
    j.h->n_done = j.ticks;
    if (bad || j.ticks < j.n_iter) {
      keep.push_back(j);
      continue;
    }
    lfsr_status st = lfsr_read_state(j.h, j.out, nullptr, nullptr, nullptr, p->main);
    if (st) {
      bad = pool_err(p, st, std::string("lfsr_pool_tick output: ") + j.h->err);
      keep.push_back(j);
      continue;
    }
    e = hipMemcpyAsync(&p->status[j.slot], j.h->b.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, p->main);
    if (e == hipSuccess) e = hipEventRecord(p->done[j.slot], p->main);
    if (e != hipSuccess) {
      bad = pool_hip(p, e, "lfsr_pool_tick retire");
      keep.push_back(j);
      continue;
    }
    p->retiring.push_back(j);
    p->dirty = true;
  }
  p->active.swap(keep);
  if (bad) return bad;
  e = hipEventRecord(p->ev_out, p->main);
  if (e == hipSuccess) e = hipStreamWaitEvent(cs, p->ev_out, 0);
  return pool_hip(p, e, "lfsr_pool_tick order out");
}

lfsr_status lfsr_pool_poll(lfsr_pool* p, int64_t* h_ids, int32_t* h_status, int32_t* h_iters, int32_t cap,
                           int32_t* h_count) {
  if (!p) return pool_err(nullptr, LFSR_EINVAL, "pool is NULL");
  if (!h_count || (cap > 0 && !h_ids)) return pool_err(p, LFSR_EINVAL, "h_count and h_ids are required");
  // a failed event query leaves that job (and the ones after it) retiring;
  // the jobs harvested before it are reported in h_ids / *h_count as usual
  int n = 0;
  std::vector<PoolJob> keep;
  hipError_t bad = hipSuccess;
  for (PoolJob& j : p->retiring) {
    if (bad != hipSuccess || n >= cap) {
      keep.push_back(j);
      continue;
    }
    const hipError_t q = hipEventQuery(p->done[j.slot]);
    if (q == hipErrorNotReady) {
      keep.push_back(j);
      continue;
    }
    if (q != hipSuccess) {
      bad = q;
      keep.push_back(j);
      continue;
    }
    const DevScalars& sc = p->status[j.slot];
    h_ids[n] = j.id;
    if (h_status) h_status[n] = (sc.err_flags & 1) ? LFSR_ENONFINITE : (sc.err_flags & 2) ? LFSR_EINVAL : LFSR_OK;
    if (h_iters) h_iters[n] = sc.iters_done;
    ++n;
    destroy_job(p, j);
  }
  p->retiring.swap(keep);
  *h_count = n;
  return pool_hip(p, bad, "lfsr_pool_poll");
}

lfsr_status lfsr_pool_info(const lfsr_pool* p, int32_t* h_active, int32_t* h_retiring, size_t* h_free,
                           size_t* h_largest_free) {
  if (!p) return pool_err(nullptr, LFSR_EINVAL, "pool is NULL");
  size_t tot = 0, big = 0;
  for (auto& kv : p->free_blocks) {
    tot += kv.second;
    big = std::max(big, kv.second);
  }
  if (h_active) *h_active = (int32_t)p->active.size();
  if (h_retiring) *h_retiring = (int32_t)p->retiring.size();
  if (h_free) *h_free = tot;
  if (h_largest_free) *h_largest_free = big;
  return LFSR_OK;
}

}  // extern "C"
