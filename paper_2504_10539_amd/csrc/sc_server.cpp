// sc_server.cpp -- continuous-batching serving loop for droplet simulations
// (lbm_server_* / lbm_submit / lbm_poll in include/lbm.h).
//
// A scheduler thread owns the GPU work.  Each tick it retires finished
// simulations, admits queued requests while the HBM pool and the slot count
// allow, initialises the new ones, and replays one HIP graph that advances
// every resident simulation by up to K steps with the batched step kernel.
// Requests that arrive while others run join at the next tick, so their work
// overlaps on the device.  Each resident simulation owns its own buffers and
// the per-cell arithmetic is the single-run kernel's, so its result is the
// same alone and in the mix.
//
// Failure detection: every run's step kernels set its status word (a pinned
// host word per slot) when they collide a cell whose density is not finite or
// not positive; the scheduler reads the words each tick and retires such runs
// at once with LBM_EUNSTABLE instead of stepping them to their last step.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <string>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sc_runtime.h"

using namespace sclbm;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) in 256-byte units.
class PoolAlloc {
 public:
  explicit PoolAlloc(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes, 256);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        in_use_ += bytes;
        high_ = std::max(high_, in_use_);
        return true;
      }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes, 256);
    in_use_ -= bytes;
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
  size_t in_use() const { return in_use_; }
  size_t high_water() const { return high_; }

 private:
  size_t in_use_ = 0, high_ = 0;
  std::map<size_t, size_t> free_;
};

struct Pending {
  uint64_t ticket;
  lbm_request req;
  std::vector<double> drops;
  double t_submit;
  size_t bytes;
  int passed = 0;  // times a later request was admitted ahead of it
};

struct Slot {
  Pending q;
  lbm_ctx* ctx = nullptr;
  size_t off = 0;
  int64_t left = 0;  // steps still to enqueue
  double t_admit = 0;
  int64_t taken = 0;      // steps enqueued (advanced, once the stream has run them)
  int flag = -1;          // index of the slot's status word
  bool unstable = false;  // retired because its status word was set
};

struct Finishing {
  Slot s;
  hipEvent_t ev = nullptr;
  double* h_res = nullptr;  // pinned, 10 doubles
};

struct Done {
  lbm_result res;
  lbm_status status;
};

constexpr int kMaxBypass = 64;  // a request may be passed at most this often

// Step variants and table capacities of the continuous policy's batch engine.
// Multi-step strip variants, valid for every request width: 256-thread strips
// suit the range of request sizes (64 .. 2048 columns) better than wider ones.
// FP32 three steps per launch on 64-byte-aligned 240-column strips (the two
// steps or the one step a tick leaves over in the two-step variant of those
// strips or a single-step tail); the FP16 forms two steps per launch on
// 250-column strips (per-cell shift with 2 rows in flight), a tail launch
// taking the odd last step of a tick; a request up to 256 columns wide is one
// periodic strip.  Moment storage takes two-step 240-column strips (its
// two-step kernel keeps four halo columns on each side).  Item capacity: every cell of the
// pool in the narrowest strips and shortest bands, plus a margin per slot.
struct EngineTables {
  int cap_items[kNumStorages], cap_titems[kNumStorages], variants[kNumStorages];
};
EngineTables engine_tables(size_t pool_bytes, int max_slots) {
  EngineTables t{};
  const int v = find_variant(256, 1, 1, 0, 2, 240);
  const int v3 = find_variant(256, 1, 1, 0, 3, 240);
  const int per = (int)std::min<size_t>(
      pool_bytes / (36ull * tile_width(v * kNumRows) * kMinRows) + 64ull * max_slots, 1u << 22);
  const int variants[kNumStorages] = {v3, find_variant(256, 1, 1, 0, 2, 250),
                                      find_variant(256, 1, 2, 0, 2, 250), v};
  for (int k = 0; k < kNumStorages; ++k) {
    t.variants[k] = variants[k];
    t.cap_items[k] = per;
    t.cap_titems[k] = step_variant(variants[k]).steps >= 2 ? per : 0;
  }
  return t;
}

size_t request_bytes(const lbm_params& p) {
  const WorkLayout w = work_layout(p.nx, p.ny);
  return 2 * align_up(pop_bytes_for(p), 256) + align_up(w.total, 256);
}

}  // namespace

struct lbm_server {
  lbm_server_opts opts{};
  char* pool = nullptr;
  size_t pool_bytes = 0;
  size_t capacity = 0;  // bytes of the pool that requests can use (the rest holds the batch tables)
  hipStream_t stream = nullptr;
  int device = 0;
  Clock::time_point t0 = Clock::now();

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> queue;
  std::unordered_map<uint64_t, Done> done;
  std::unordered_map<uint64_t, int> live;  // tickets not yet collected
  uint64_t next_ticket = 1;
  bool stop = false;
  bool broken = false;    // the scheduler stopped on an internal error
  int64_t in_flight = 0;  // admitted or queued, not finished
  lbm_server_stats st{};

  // scheduler-thread state
  PoolAlloc* alloc = nullptr;
  std::vector<Slot> active;
  std::vector<Finishing> finishing;
  BatchEngine eng;
  bool eng_ready = false;
  std::deque<hipEvent_t> tick_events;
  std::vector<double*> pinned_free;
  // Status words, one per slot that may still have work on the device
  // (resident or finishing): pinned host memory the kernels write through its
  // device address (the fake executor uses plain host memory).  A word is
  // reused only after every launch of its previous owner has completed.
  volatile int* flags = nullptr;
  int* flags_dev = nullptr;
  std::vector<int> flags_host;
  std::vector<int> free_flags;
  std::thread worker;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void run();
  void admit_locked(std::vector<Slot>& admitted);
  lbm_status start_slot(Slot& s);
  void finish_slot(Slot& s);
  void poll_finishing(bool block);
  void complete(const Slot& s, lbm_status status, const lbm_metrics& m, int64_t taken);
  void release_flag(Slot& s);
  void retire_unstable();
  void fake_tick();
  void run_guarded();
  void fail_all(lbm_status code);
};

// taken: time steps the run advanced.  Throughput counts only runs that
// completed with LBM_OK; the work of unstable runs is counted apart.
void lbm_server::complete(const Slot& s, lbm_status status, const lbm_metrics& m, int64_t taken) {
  std::lock_guard<std::mutex> lk(mu);
  Done d{};
  d.res.metrics = m;
  d.res.t_submit = s.q.t_submit;
  d.res.t_admit = s.t_admit;
  d.res.t_done = now();
  d.res.ticket = (int64_t)s.q.ticket;
  d.status = status;
  done[s.q.ticket] = d;
  st.completed += 1;
  if (status != LBM_OK) st.failed += 1;
  st.resident -= 1;
  const double upd = (double)s.q.req.params.nx * s.q.req.params.ny * (double)taken;
  if (status == LBM_OK) st.lattice_updates += upd;
  if (status == LBM_EUNSTABLE) {
    st.unstable += 1;
    st.unstable_updates += upd;
    if (taken < s.q.req.steps) st.retired_early += 1;
  }
  in_flight -= 1;
  cv_done.notify_all();
}

// Moves requests from the queue into slots.  First come first served; a
// request that does not fit yet may be passed, at most kMaxBypass times.
void lbm_server::admit_locked(std::vector<Slot>& admitted) {
  const int max_slots = opts.policy == LBM_POLICY_FIFO ? 1 : opts.max_slots;
  int resident = (int)active.size();
  for (auto it = queue.begin();
       it != queue.end() && resident < max_slots && !free_flags.empty();) {
    size_t off = 0;
    if (alloc->alloc(it->bytes, &off)) {
      Slot s;
      s.q = std::move(*it);
      s.off = off;
      s.flag = free_flags.back();
      free_flags.pop_back();
      flags[s.flag] = 0;  // the previous owner's launches have all completed
      s.t_admit = now();
      s.left = s.q.req.steps;
      for (auto jt = queue.begin(); jt != it; ++jt) jt->passed += 1;
      it = queue.erase(it);
      admitted.push_back(std::move(s));
      ++resident;
      st.admitted += 1;
      st.resident += 1;
      continue;
    }
    if (opts.policy == LBM_POLICY_FIFO || it->passed >= kMaxBypass) break;
    ++it;
  }
  st.queued = (int64_t)queue.size();
  st.pool_in_use = alloc->in_use();
  st.pool_high_water = alloc->high_water();
}

lbm_status lbm_server::start_slot(Slot& s) {
  const lbm_params& p = s.q.req.params;
  const size_t pb = align_up(pop_bytes_for(p), 256);
  const WorkLayout w = work_layout(p.nx, p.ny);
  char* base = pool + s.off;
  lbm_ctx* c = nullptr;
  // Under the continuous policy the engine drives the run, and the slot keeps
  // the droplet list until the request completes: nothing here waits for the
  // stream, so admissions do not drain the ticks queued ahead of the GPU.
  const bool fifo = opts.policy == LBM_POLICY_FIFO;
  lbm_status r = create_ctx(&p, base, base + pb, pb, base + 2 * pb, w.total, stream, fifo, &c,
                            flags_dev + s.flag);
  if (r != LBM_OK) return r;
  s.ctx = c;
  lbm_init ip = s.q.req.init;
  r = init_droplets(c, s.q.drops.empty() ? nullptr : s.q.drops.data(), s.q.req.n_drops, &ip, fifo);
  return r;
}

// Enqueues the final exports and metrics of a finished simulation.
void lbm_server::finish_slot(Slot& s) {
  Finishing f;
  f.s = std::move(s);
  lbm_ctx* c = f.s.ctx;
  lbm_status r = LBM_OK;
  if (f.s.q.req.rho_out) r = lbm_moments(c, f.s.q.req.rho_out, nullptr, nullptr);
  if (r == LBM_OK && f.s.q.req.f_out) r = lbm_get_state(c, f.s.q.req.f_out);
  void* idle = c->pop[c->parity ^ 1];
  hipError_t e = launch_diagnostics(c->p.storage, c->pop[c->parity], c->p.nx, c->p.ny,
                                    c->host_desc().rho0, reinterpret_cast<double*>(idle),
                                    c->d_partials, c->d_result, stream);
  if (pinned_free.empty()) {
    double* h = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&h), 16 * sizeof(double), hipHostMallocDefault) ==
        hipSuccess)
      pinned_free.push_back(h);
  }
  if (e == hipSuccess && !pinned_free.empty()) {
    f.h_res = pinned_free.back();
    pinned_free.pop_back();
    e = hipMemcpyAsync(f.h_res, c->d_result, 10 * sizeof(double), hipMemcpyDeviceToHost, stream);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&f.ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(f.ev, stream);
  // The pool range can be handed out again now: any later use is enqueued on
  // the same stream after these reads.
  {
    std::lock_guard<std::mutex> lk(mu);
    alloc->release(f.s.off, f.s.q.bytes);
    st.pool_in_use = alloc->in_use();
  }
  if (r != LBM_OK || e != hipSuccess || !f.h_res) {
    if (f.ev) (void)hipEventDestroy(f.ev);
    if (f.h_res) pinned_free.push_back(f.h_res);
    (void)hipStreamSynchronize(stream);
    lbm_destroy(c);
    release_flag(f.s);
    lbm_metrics m{};
    complete(f.s, r != LBM_OK ? r : LBM_EDEVICE, m, f.s.taken);
    return;
  }
  finishing.push_back(std::move(f));
}

void lbm_server::poll_finishing(bool block) {
  for (size_t i = 0; i < finishing.size();) {
    Finishing& f = finishing[i];
    hipError_t e = block ? hipEventSynchronize(f.ev) : hipEventQuery(f.ev);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    lbm_metrics m{};
    lbm_status status = LBM_OK;
    if (e != hipSuccess) {
      status = LBM_EDEVICE;
    } else {
      const double* r = f.h_res;
      const lbm_params& p = f.s.q.req.params;
      const double ncell = (double)p.nx * p.ny;
      m.mass = r[0];
      m.mom_x = r[1];
      m.mom_y = r[2];
      m.finite = r[3] == 0.0 ? 1 : 0;
      m.n_above = (int64_t)r[4];
      m.Gmax = r[5];
      m.sum_grad = r[6];
      m.E_int = r[7];
      m.rho_max = r[8];
      m.rho_min = r[9];
      m.W = r[4] / ncell;
      m.drho = r[8] - r[9];
      m.W_eff = r[5] > 0.0 ? r[6] / (r[5] * ncell) : 0.0;
      m.step = f.s.ctx->steps;
      if (!m.finite || f.s.unstable) status = LBM_EUNSTABLE;
    }
    (void)hipEventDestroy(f.ev);
    pinned_free.push_back(f.h_res);
    delete f.s.ctx;  // no pinned buffer was made for it; its work has completed
    Slot s = std::move(f.s);
    finishing.erase(finishing.begin() + i);
    release_flag(s);  // every launch that could write it has completed
    complete(s, status, m, s.taken);
  }
}

void lbm_server::release_flag(Slot& s) {
  if (s.flag >= 0) free_flags.push_back(s.flag);
  s.flag = -1;
}

// Retires the resident runs whose status word a step kernel has set: their
// final diagnostics are enqueued behind the ticks already queued, and the
// request completes with LBM_EUNSTABLE.
void lbm_server::retire_unstable() {
  for (size_t i = 0; i < active.size();) {
    if (flags[active[i].flag] == 0) {
      ++i;
      continue;
    }
    Slot s = std::move(active[i]);
    active.erase(active.begin() + i);
    s.unstable = true;
    finish_slot(s);
  }
}

// Host-only executor for tests of the scheduling logic: a tick advances each
// resident request by up to K steps and sleeps for the time that work would
// take at opts.fake_mlups.
// A request whose starting density is not positive (what the GPU path finds
// unstable) sets its status word in its first tick and is retired then, as the
// GPU path retires a run whose kernels flag it.
void lbm_server::fake_tick() {
  double work = 0;
  for (Slot& s : active) {
    const int64_t k = std::min<int64_t>(opts.steps_per_tick, s.left);
    s.left -= k;
    s.taken += k;
    work += (double)s.q.req.params.nx * s.q.req.params.ny * (double)k;
    const lbm_init& in = s.q.req.init;
    if (k > 0 && !((std::min(in.rho_g, in.rho_l) - in.noise_amp) > 0.0)) flags[s.flag] = 1;
  }
  const double secs = work / (std::max(opts.fake_mlups, 1e-6) * 1e6);
  if (secs > 0) std::this_thread::sleep_for(std::chrono::duration<double>(secs));
  for (size_t i = 0; i < active.size();) {
    const bool flagged = flags[active[i].flag] != 0;
    if (active[i].left > 0 && !flagged) {
      ++i;
      continue;
    }
    Slot s = std::move(active[i]);
    active.erase(active.begin() + i);
    {
      std::lock_guard<std::mutex> lk(mu);
      alloc->release(s.off, s.q.bytes);
      st.pool_in_use = alloc->in_use();
    }
    release_flag(s);
    const lbm_request& q = s.q.req;
    lbm_metrics m{};
    m.step = s.taken;
    m.mass = (double)q.params.nx * q.params.ny;
    m.finite = flagged ? 0 : 1;
    complete(s, flagged ? LBM_EUNSTABLE : LBM_OK, m, s.taken);
  }
}

void lbm_server::run() {
  if (!opts.fake_executor) (void)hipSetDevice(device);
  bool members_changed = true;
  while (true) {
    std::vector<Slot> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] {
        return stop || !queue.empty() || !active.empty() || !finishing.empty();
      });
      if (stop && queue.empty() && active.empty() && finishing.empty()) break;
      admit_locked(admitted);
      st.ticks += 1;
    }
    if (opts.fake_executor) {
      for (Slot& s : admitted) active.push_back(std::move(s));
      fake_tick();
      continue;
    }
    for (Slot& s : admitted) {
      const lbm_status r = start_slot(s);
      if (r != LBM_OK) {
        {
          std::lock_guard<std::mutex> lk(mu);
          alloc->release(s.off, s.q.bytes);
        }
        if (s.ctx) lbm_destroy(s.ctx);  // synchronises: nothing of it is left on the device
        release_flag(s);
        complete(s, r, lbm_metrics{}, 0);
        continue;
      }
      active.push_back(std::move(s));
      members_changed = true;
    }
    // Requests of zero steps finish at once.
    for (size_t i = 0; i < active.size();) {
      if (active[i].left > 0) {
        ++i;
        continue;
      }
      Slot s = std::move(active[i]);
      active.erase(active.begin() + i);
      finish_slot(s);
      members_changed = true;
    }
    if (!active.empty()) {
      lbm_status r = LBM_OK;
      if (opts.policy == LBM_POLICY_FIFO) {
        Slot& s = active[0];
        const int64_t k = std::min<int64_t>(opts.steps_per_tick, s.left);
        r = lbm_step_n(s.ctx, k);
        s.left -= k;
        s.taken += k;
      } else {
        if (members_changed) {
          std::vector<lbm_ctx*> m;
          std::vector<int64_t> rem;
          for (Slot& s : active) {
            m.push_back(s.ctx);
            rem.push_back(s.left);
          }
          r = eng.load(m, rem);
          members_changed = false;
        }
        if (r == LBM_OK) r = eng.replay();
        for (Slot& s : active) {
          const int64_t k = std::min<int64_t>(opts.steps_per_tick, s.left);
          s.left -= k;
          s.taken += k;
          s.ctx->steps += k;
          s.ctx->parity = (int)((s.ctx->parity + tick_flips(k, eng.per_launch(s.ctx->p.storage))) & 1);
        }
      }
      if (r != LBM_OK) {
        // A device failure poisons every resident simulation.
        for (Slot& s : active) {
          {
            std::lock_guard<std::mutex> lk(mu);
            alloc->release(s.off, s.q.bytes);
          }
          release_flag(s);
          complete(s, LBM_EDEVICE, lbm_metrics{}, 0);
        }
        active.clear();
        members_changed = true;
      }
      // Runs that went unstable in the ticks already run leave now.
      {
        const size_t before = active.size();
        retire_unstable();
        if (active.size() != before) members_changed = true;
      }
      for (size_t i = 0; i < active.size();) {
        if (active[i].left > 0) {
          ++i;
          continue;
        }
        Slot s = std::move(active[i]);
        active.erase(active.begin() + i);
        finish_slot(s);
        members_changed = true;
      }
      // Keep at most two ticks queued ahead of the GPU.
      hipEvent_t ev = nullptr;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
        (void)hipEventRecord(ev, stream);
        tick_events.push_back(ev);
      }
      while (tick_events.size() > 2) {
        (void)hipEventSynchronize(tick_events.front());
        (void)hipEventDestroy(tick_events.front());
        tick_events.pop_front();
      }
    }
    poll_finishing(active.empty());
  }
  for (hipEvent_t e : tick_events) (void)hipEventDestroy(e);
  tick_events.clear();
}

// The scheduler thread: an exception out of the loop (host memory exhausted,
// or an internal error) stops the scheduler, fails every request it holds
// with LBM_EDEVICE and makes later submissions fail, instead of ending the
// process.
void lbm_server::run_guarded() {
  try {
    run();
    return;
  } catch (...) {
  }
  try {
    if (!opts.fake_executor) (void)hipStreamSynchronize(stream);
    fail_all(LBM_EDEVICE);
  } catch (...) {
  }
}

void lbm_server::fail_all(lbm_status code) {
  std::lock_guard<std::mutex> lk(mu);
  broken = true;
  auto fail_one = [&](uint64_t ticket, double t_submit, double t_admit, bool resident) {
    Done d{};
    d.res.t_submit = t_submit;
    d.res.t_admit = t_admit;
    d.res.t_done = now();
    d.res.ticket = (int64_t)ticket;
    d.status = code;
    done[ticket] = d;
    st.completed += 1;
    st.failed += 1;
    if (resident) st.resident -= 1;
    in_flight -= 1;
  };
  for (const Pending& q : queue) fail_one(q.ticket, q.t_submit, 0.0, false);
  queue.clear();
  for (Slot& s : active) {
    fail_one(s.q.ticket, s.q.t_submit, s.t_admit, true);
    delete s.ctx;  // the stream was drained before
  }
  active.clear();
  for (Finishing& f : finishing) {
    fail_one(f.s.q.ticket, f.s.q.t_submit, f.s.t_admit, true);
    if (f.ev) (void)hipEventDestroy(f.ev);
    if (f.h_res) pinned_free.push_back(f.h_res);
    delete f.s.ctx;
  }
  finishing.clear();
  st.queued = 0;
  set_error("serving loop stopped on an internal error");
  cv_done.notify_all();
}

extern "C" {

lbm_status lbm_server_create(void* pool, size_t pool_bytes, void* hip_stream,
                             const lbm_server_opts* opts, lbm_server** out) {
  return guarded("lbm_server_create", [&]() -> lbm_status {
    if (!out || !opts) return fail(LBM_EINVAL, "out or opts is NULL");
    *out = nullptr;
    if (opts->policy != LBM_POLICY_CONTINUOUS && opts->policy != LBM_POLICY_FIFO)
      return fail(LBM_EINVAL, "unknown policy");
    if (opts->steps_per_tick < 1 || opts->steps_per_tick > 4096)
      return fail(LBM_EINVAL, "steps_per_tick must be in [1, 4096]");
    if (opts->max_slots < 1 || opts->max_slots > 4096)
      return fail(LBM_EINVAL, "max_slots must be in [1, 4096]");
    if (!opts->fake_executor && (!pool || ((uintptr_t)pool & 255)))
      return fail(LBM_EINVAL, "pool must be a 256-byte aligned device buffer");
    if (opts->fake_executor && !(opts->fake_mlups > 0.0))
      return fail(LBM_EINVAL, "fake_mlups must be > 0");
    if (pool_bytes < 4096) return fail(LBM_EINVAL, "pool too small");
    lbm_server* s = new (std::nothrow) lbm_server();
    if (!s) return fail(LBM_ENOMEM, "host allocation failed");
    s->opts = *opts;
    s->pool = reinterpret_cast<char*>(pool);
    s->pool_bytes = pool_bytes;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->st.pool_bytes = pool_bytes;
    if (!opts->fake_executor) {
      if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(LBM_EDEVICE, "hipGetDevice failed");
      }
    }
    // Engine workspace lives at the top of the pool; requests share the rest
    // (the fake executor keeps the same split, so its budget is the GPU
    // path's).
    size_t eng_bytes = 0;
    EngineTables tab{};
    if (opts->policy == LBM_POLICY_CONTINUOUS) {
      tab = engine_tables(pool_bytes, opts->max_slots);
      eng_bytes = align_up(BatchEngine::work_bytes(opts->max_slots, tab.cap_items, tab.cap_titems,
                                                   opts->steps_per_tick),
                           256);
      if (eng_bytes >= pool_bytes / 2) {
        delete s;
        return fail(LBM_ENOMEM, "pool too small for the batch tables");
      }
    }
    if (eng_bytes > 0 && !opts->fake_executor) {
      s->eng.persistent = true;
      s->eng.lazy_storages = true;  // no empty launches for storage types not yet served
      // One band height for every request: the persistent grid hands items out
      // round-robin, which balances only items of similar size.  32 rows: on a
      // saturated FP32 trace with three steps per launch 8, 16 and 32 rows
      // served 121k, 140k and 145k MLUPS.
      s->eng.row_override = row_choice(32);
      lbm_status r = s->eng.init(s->stream, opts->steps_per_tick, opts->max_slots, tab.cap_items,
                                 tab.cap_titems, tab.variants, s->pool + pool_bytes - eng_bytes,
                                 eng_bytes);
      if (r != LBM_OK) {
        s->eng.destroy();
        delete s;
        return r;
      }
      s->eng_ready = true;
    }
    s->capacity = pool_bytes - eng_bytes;
    s->st.pool_bytes = s->capacity;
    // Status words: every resident slot and every slot still finishing holds
    // one; admission waits for a free word.
    const int nflags = 2 * opts->max_slots + 8;
    for (int k = nflags - 1; k >= 0; --k) s->free_flags.push_back(k);
    if (opts->fake_executor) {
      s->flags_host.assign(nflags, 0);
      s->flags = s->flags_host.data();
    } else {
      void* h = nullptr;
      void* d = nullptr;
      hipError_t e = hipHostMalloc(&h, nflags * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent);
      if (e == hipSuccess) e = hipHostGetDevicePointer(&d, h, 0);
      if (e != hipSuccess) {
        if (h) (void)hipHostFree(h);
        if (s->eng_ready) s->eng.destroy();
        delete s;
        return hip_fail(e, "status words (hipHostMalloc)");
      }
      std::memset(h, 0, nflags * sizeof(int));
      s->flags = reinterpret_cast<volatile int*>(h);
      s->flags_dev = reinterpret_cast<int*>(d);
    }
    try {
      s->alloc = new PoolAlloc(s->capacity);
      s->worker = std::thread([s] { s->run_guarded(); });
    } catch (...) {
      if (!opts->fake_executor) (void)hipHostFree(const_cast<int*>(s->flags));
      if (s->eng_ready) s->eng.destroy();
      delete s->alloc;
      delete s;
      throw;
    }
    *out = s;
    return LBM_OK;
  });
}

lbm_status lbm_submit(lbm_server* s, const lbm_request* r, uint64_t* ticket) {
  return guarded("lbm_submit", [&]() -> lbm_status {
    if (!s || !r || !ticket) return fail(LBM_EINVAL, "server, request or ticket is NULL");
    lbm_status v = validate_params(&r->params);
    if (v != LBM_OK) return v;
    if (r->steps < 0) return fail(LBM_EINVAL, "steps must be >= 0");
    if (r->n_drops < 0 || (r->n_drops > 0 && !r->drops)) return fail(LBM_EINVAL, "bad droplet array");
    if (!(r->init.width > 0.0) || r->init.noise_amp < 0.0 || !std::isfinite(r->init.rho_l) ||
        !std::isfinite(r->init.rho_g))
      return fail(LBM_EINVAL, "bad init fields");
    // The droplet list goes into the run's idle buffer after its FP64 density
    // scratch (lbm_init_droplets): checked before anything is copied.
    const size_t ncell = (size_t)r->params.nx * r->params.ny;
    if ((size_t)r->n_drops * 24 + align_up(ncell * 8, 256) > align_up(pop_bytes_for(r->params), 256))
      return fail(LBM_EINVAL, "too many droplets for this grid");
    const size_t bytes = request_bytes(r->params);
    if (bytes > s->capacity)
      return fail(LBM_ENOMEM, "request needs " + std::to_string(bytes) +
                                  " bytes; the pool's capacity for requests is " +
                                  std::to_string(s->capacity));
    Pending q;
    q.req = *r;
    q.drops.assign(r->drops, r->drops + 3 * (size_t)r->n_drops);
    q.req.drops = nullptr;
    q.bytes = bytes;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(LBM_EBUSY, "server is stopping");
    if (s->broken) return fail(LBM_EDEVICE, "serving loop stopped on an internal error");
    q.ticket = s->next_ticket++;
    q.t_submit = s->now();
    *ticket = q.ticket;
    s->live[q.ticket] = 1;
    s->queue.push_back(std::move(q));
    s->st.submitted += 1;
    s->st.queued = (int64_t)s->queue.size();
    s->in_flight += 1;
    s->cv_work.notify_one();
    return LBM_OK;
  });
}

lbm_status lbm_poll(lbm_server* s, uint64_t ticket, lbm_result* out) {
  return guarded("lbm_poll", [&]() -> lbm_status {
    if (!s || !out) return fail(LBM_EINVAL, "server or out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(ticket);
    if (it == s->done.end()) {
      if (s->live.count(ticket)) return LBM_PENDING;
      return fail(LBM_ENOTFOUND, "unknown or already collected ticket");
    }
    *out = it->second.res;
    const lbm_status st = it->second.status;
    s->done.erase(it);
    s->live.erase(ticket);
    if (st != LBM_OK) set_error("request did not complete cleanly");
    return st;
  });
}

lbm_status lbm_server_drain(lbm_server* s) {
  return guarded("lbm_server_drain", [&]() -> lbm_status {
    if (!s) return fail(LBM_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->in_flight == 0; });
    return LBM_OK;
  });
}

lbm_status lbm_server_get_stats(lbm_server* s, lbm_server_stats* out) {
  return guarded("lbm_server_get_stats", [&]() -> lbm_status {
    if (!s || !out) return fail(LBM_EINVAL, "server or out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return LBM_OK;
  });
}

double lbm_server_clock(const lbm_server* s) { return s ? s->now() : -1.0; }

lbm_status lbm_server_destroy(lbm_server* s) {
  return guarded("lbm_server_destroy", [&]() -> lbm_status {
    if (!s) return LBM_OK;
    lbm_server_drain(s);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
      s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    if (!s->opts.fake_executor) {
      (void)hipStreamSynchronize(s->stream);
      for (double* h : s->pinned_free) (void)hipHostFree(h);
      if (s->flags) (void)hipHostFree(const_cast<int*>(s->flags));
      if (s->eng_ready) s->eng.destroy();
    }
    delete s->alloc;
    delete s;
    return LBM_OK;
  });
}

}  // extern "C"
