// Request server: many flexible GMRES solves of mixed shapes in flight on one device.
//
// Each request is a SolveRun (the host state machine of the single-solve entry point)
// whose Krylov bases and scratch live in one device arena.  Requests are spread over a
// few HIP streams ("lanes").  When a lane's previous launches have completed, every
// request on it reads its host-mapped scalars, advances its FP64 least-squares state
// and gets its next phase; requests of one context at the same kind of phase are then
// launched together, one kernel per step for the whole group, through device pointer
// tables (their Arnoldi indices may differ).  Lanes run concurrently on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "context.h"
#include "solve_run.h"

using namespace fdg;

namespace {

// First-fit allocator over [0, cap) with coalescing of freed neighbours.
class ArenaAlloc {
 public:
  void init(size_t cap) {
    free_.clear();
    if (cap) free_[0] = cap;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    auto it = free_.emplace(off, bytes).first;
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

 private:
  std::map<size_t, size_t> free_;
};

struct Slot {
  bool used = false;
  bool fresh = false;  // admitted; first phase not launched yet
  int lane = -1;
  size_t off = 0, bytes = 0;
  int64_t tag = 0;
  SolveRun run;
};

struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  int nfresh = 0;
  double load = 0.0;  // sum of N over its requests
  std::vector<int> slots;
  TableArena tab;
};

size_t table_cap(int max_slots) {
  const size_t per = 32 * sizeof(void *) + 256 * sizeof(double) + 64;
  return (size_t)std::min(max_slots, 1024) * per + 65536;
}

}  // namespace

struct fdg_server {
  int device = 0, max_slots = 0, m = 0;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  ArenaAlloc alloc;
  double *pin = nullptr, *pin_dev = nullptr;  // host-mapped, max_slots * host_doubles(m)
  std::vector<Slot> slots;
  std::vector<int> free_slots;
  std::vector<Lane> lanes;
  std::deque<fdg_done> completed;
  int pending = 0;
  int64_t services = 0, groups = 0, grouped_runs = 0, max_group = 0;
};

namespace {

void release_slot(fdg_server *s, int idx) {
  Slot &sl = s->slots[idx];
  s->alloc.release(sl.off, sl.bytes);
  Lane &ln = s->lanes[sl.lane];
  ln.load -= (double)sl.run.N;
  sl.used = false;
  sl.lane = -1;
  s->free_slots.push_back(idx);
}

void complete(fdg_server *s, int idx, int status) {
  Slot &sl = s->slots[idx];
  fdg_done d;
  std::memset(&d, 0, sizeof(d));
  d.tag = sl.tag;
  d.status = status;
  d.info = sl.run.info();
  s->completed.push_back(d);
}

// Groups of runs that can share launches: same context and step mask (context able to
// take gathered batches), at most kMaxGroupEntries each, in admission order.
void make_groups(fdg_server *s, const std::vector<int> &idx, std::vector<std::vector<SolveRun *>> &out) {
  out.clear();
  std::map<std::pair<const fdg_ctx *, unsigned>, size_t> open;
  for (int i : idx) {
    SolveRun *r = &s->slots[i].run;
    const unsigned steps = r->phase().steps;
    if (!groupable(r->ctx) || (steps & kStepZeroX)) {
      out.push_back({r});
      continue;
    }
    const auto key = std::make_pair((const fdg_ctx *)r->ctx, steps);
    auto it = open.find(key);
    if (it == open.end() || out[it->second].size() >= (size_t)kMaxGroupEntries) {
      open[key] = out.size();
      out.push_back({r});
    } else {
      out[it->second].push_back(r);
    }
  }
}

int service_lane(fdg_server *s, int li) {
  Lane &ln = s->lanes[li];
  ++s->services;
  // 1. the lane's launches completed: advance every request that was in flight
  std::vector<int> keep;
  keep.reserve(ln.slots.size());
  for (int idx : ln.slots) {
    Slot &sl = s->slots[idx];
    if (sl.fresh) {
      sl.fresh = false;
      keep.push_back(idx);
      continue;
    }
    sl.run.consume();
    if (sl.run.finished()) {
      complete(s, idx, sl.run.status());
      release_slot(s, idx);
      --s->pending;
    } else {
      keep.push_back(idx);
    }
  }
  ln.slots.swap(keep);
  ln.nfresh = 0;
  ln.busy = false;
  if (ln.slots.empty()) return FDG_OK;
  // 2. launch the next phase of every request, grouped
  std::vector<std::vector<SolveRun *>> groups;
  make_groups(s, ln.slots, groups);
  ln.tab.reset();
  const Exec ex{ln.stream, false};
  for (auto &g : groups) {
    int st = enqueue_phase(ex, g.data(), (int)g.size(), &ln.tab);
    if (st == FDG_ENOMEM && g.size() > 1) {  // table space exhausted: launch one by one
      st = FDG_OK;
      for (SolveRun *r : g)
        if ((st = enqueue_phase(ex, &r, 1, nullptr)) != FDG_OK) break;
    }
    if (st != FDG_OK) return st;
    ++s->groups;
    s->grouped_runs += (int64_t)g.size();
    s->max_group = std::max<int64_t>(s->max_group, (int64_t)g.size());
  }
  HIPCHK(hipEventRecord(ln.ev, ln.stream));
  ln.busy = true;
  return FDG_OK;
}

}  // namespace

// ------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------
extern "C" int fdg_server_destroy(fdg_server *s) {
  clear_error();
  if (!s) return FDG_OK;
  for (Lane &ln : s->lanes) {
    if (ln.stream) {
      (void)hipStreamSynchronize(ln.stream);
      (void)hipStreamDestroy(ln.stream);
    }
    if (ln.ev) (void)hipEventDestroy(ln.ev);
    if (ln.tab.host) (void)hipHostFree(ln.tab.host);
    if (ln.tab.dev) (void)hipFree(ln.tab.dev);
  }
  if (s->arena) (void)hipFree(s->arena);
  if (s->pin) (void)hipHostFree(s->pin);
  delete s;
  return FDG_OK;
}

extern "C" int fdg_server_create(fdg_server **out, int max_slots, int restart, int lanes, size_t arena_bytes) {
  clear_error();
  if (!out) return set_error(FDG_EINVAL, "server_create: NULL argument");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 4096) return set_error(FDG_EINVAL, "server_create: max_slots in [1, 4096]");
  if (restart < 1 || restart > 255) return set_error(FDG_EINVAL, "server_create: restart in [1, 255]");
  if (lanes < 1 || lanes > 16) return set_error(FDG_EINVAL, "server_create: lanes in [1, 16]");
  if (arena_bytes < 4096) return set_error(FDG_EINVAL, "server_create: arena too small");
  fdg_server *s = new fdg_server();
  int st = FDG_OK;
  auto fail = [&](int code) {
    fdg_server_destroy(s);
    return code;
  };
  if ((st = hip_check(hipGetDevice(&s->device), "hipGetDevice")) != FDG_OK) return fail(st);
  s->max_slots = max_slots;
  s->m = restart;
  s->arena_bytes = arena_bytes;
  if ((st = hip_check(hipMalloc((void **)&s->arena, arena_bytes), "server arena")) != FDG_OK) return fail(st);
  s->alloc.init(arena_bytes);
  const size_t pin_bytes = sizeof(double) * (size_t)max_slots * host_doubles(restart);
  if ((st = hip_check(hipHostMalloc((void **)&s->pin, pin_bytes, hipHostMallocMapped), "server pinned")) != FDG_OK)
    return fail(st);
  if ((st = hip_check(hipHostGetDevicePointer((void **)&s->pin_dev, s->pin, 0), "hipHostGetDevicePointer")) !=
      FDG_OK)
    return fail(st);
  s->slots.resize(max_slots);
  for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->lanes.resize(lanes);
  const size_t tcap = table_cap(max_slots);
  for (Lane &ln : s->lanes) {
    if ((st = hip_check(hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking), "hipStreamCreate")) != FDG_OK)
      return fail(st);
    if ((st = hip_check(hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming), "hipEventCreate")) != FDG_OK)
      return fail(st);
    if ((st = hip_check(hipHostMalloc((void **)&ln.tab.host, tcap, hipHostMallocDefault), "table staging")) !=
        FDG_OK)
      return fail(st);
    if ((st = hip_check(hipMalloc((void **)&ln.tab.dev, tcap), "table device")) != FDG_OK) return fail(st);
    ln.tab.cap = tcap;
  }
  *out = s;
  return FDG_OK;
}

extern "C" size_t fdg_server_run_bytes(const fdg_ctx *c, int restart) {
  if (!c || restart < 1) return 0;
  return run_bytes(c, restart);
}

extern "C" int fdg_server_admit(fdg_server *s, fdg_ctx *c, const double *b, double *x, double rtol, int maxit,
                                int flags, int64_t tag) {
  clear_error();
  if (!s || !c || !b || !x) return set_error(FDG_EINVAL, "server_admit: NULL argument");
  if (b == x) return set_error(FDG_EINVAL, "server_admit: b and x alias");
  if (c->batch != 1) return set_error(FDG_EINVAL, "server_admit: context batch must be 1");
  if (c->device != s->device) return set_error(FDG_EINVAL, "server_admit: context on another device");
  if (!(rtol >= 0.0) || maxit < 0) return set_error(FDG_EINVAL, "server_admit: bad rtol/maxit");
  int st = ctx_ready(c);
  if (st != FDG_OK) return st;
  if (s->free_slots.empty()) return set_error(FDG_EFULL, "server_admit: all %d slots in use", s->max_slots);
  const size_t bytes = run_bytes(c, s->m);
  size_t off = 0;
  if (!s->alloc.alloc(bytes, &off))
    return set_error(FDG_EFULL, "server_admit: %zu arena bytes not available", bytes);
  const int idx = s->free_slots.back();
  s->free_slots.pop_back();
  Slot &sl = s->slots[idx];
  sl.used = true;
  sl.fresh = true;
  sl.off = off;
  sl.bytes = bytes;
  sl.tag = tag;
  RunBufs rb = carve_run(s->arena + off, c, s->m);
  rb.hh = s->pin + (size_t)idx * host_doubles(s->m);
  rb.hh_dev = s->pin_dev + (size_t)idx * host_doubles(s->m);
  sl.run.init(c, rb, s->m, b, x, rtol, maxit, flags);
  // lane: one already serving this context with room in its group (shared launches),
  // else the least loaded
  int lane = -1;
  if (groupable(c))
    for (size_t li = 0; li < s->lanes.size() && lane < 0; ++li) {
      int same = 0;
      for (int j : s->lanes[li].slots) same += s->slots[j].run.ctx == c ? 1 : 0;
      if (same > 0 && same < kMaxGroupEntries) lane = (int)li;
    }
  if (lane < 0) {
    lane = 0;
    for (size_t li = 1; li < s->lanes.size(); ++li)
      if (s->lanes[li].load < s->lanes[lane].load) lane = (int)li;
  }
  sl.lane = lane;
  Lane &ln = s->lanes[lane];
  ln.slots.push_back(idx);
  ln.load += (double)c->N;
  ++ln.nfresh;
  ++s->pending;
  return FDG_OK;
}

extern "C" int fdg_server_step(fdg_server *s, int wait_us, fdg_done *done, int cap, int *ndone) {
  clear_error();
  if (!s || !ndone || (cap > 0 && !done) || cap < 0) return set_error(FDG_EINVAL, "server_step: bad argument");
  *ndone = 0;
  const auto t0 = std::chrono::steady_clock::now();
  while (true) {
    bool any = false;
    for (size_t li = 0; li < s->lanes.size(); ++li) {
      Lane &ln = s->lanes[li];
      if (ln.slots.empty()) continue;
      bool ready;
      if (ln.busy) {
        const hipError_t e = hipEventQuery(ln.ev);
        if (e == hipErrorNotReady) {
          (void)hipGetLastError();
          ready = false;
        } else {
          HIPCHK(e);
          ready = true;
        }
      } else {
        ready = ln.nfresh > 0;
      }
      if (!ready) continue;
      int st = service_lane(s, (int)li);
      if (st != FDG_OK) return st;
      any = true;
    }
    if (any || s->pending == 0 || !s->completed.empty()) break;
    const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    if (us >= wait_us) break;
  }
  while (*ndone < cap && !s->completed.empty()) {
    done[*ndone] = s->completed.front();
    s->completed.pop_front();
    ++*ndone;
  }
  return FDG_OK;
}

extern "C" int fdg_server_pending(const fdg_server *s) {
  if (!s) return 0;
  return s->pending + (int)s->completed.size();
}

extern "C" int fdg_server_stats(const fdg_server *s, int64_t *services, int64_t *groups, int64_t *grouped_runs,
                                int64_t *max_group) {
  clear_error();
  if (!s || !services || !groups || !grouped_runs || !max_group)
    return set_error(FDG_EINVAL, "server_stats: NULL argument");
  *services = s->services;
  *groups = s->groups;
  *grouped_runs = s->grouped_runs;
  *max_group = s->max_group;
  return FDG_OK;
}
