// Serving loop: continuous batching of LP solves under a device-memory
// budget.
//
// Submitted LPs are copied, then prepared (validation, rescaling, CSR
// transpose, tiling) by worker threads that take them in submission order. The scheduler
// thread admits prepared LPs in submission order while the budget, the
// launch-table capacity and the slot limit allow; it uploads each into its
// own block of the arena and computes its initial A x on the upload stream
// while the resident LPs keep iterating on the compute stream. Between
// launch sequences it rewrites the shared launch tables (fixed addresses,
// so one captured launch sequence serves every mix), reads every resident
// LP's control block with one copy, and retires LPs that finished: their
// iterates are downloaded, unscaled and handed to poll / wait, and their
// block returns to the arena.
//
// Each LP's arithmetic depends only on its own data: rows are reduced
// inside one tile and every cross-tile sum is exact (double-double), so a
// result does not depend on what else shares the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "opdhg.h"
#include "opdhg_host.h"
#include "opdhg_internal.h"

namespace opdhg {
namespace {

using Clock = std::chrono::steady_clock;

double seconds_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// First-fit allocator over [0, size) in 256-byte units; freed blocks merge
// with free neighbours.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, noff = it->first + bytes;
      free_.erase(it);
      if (rest) free_[noff] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
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
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

enum class JobState { kQueued, kPrepared, kAdmitted, kActive, kFinished, kDone };

struct Job {
  uint64_t ticket = 0;
  opdhg_params p{};
  // owned copy of the LP until it is prepared
  int64_t m = 0, n = 0, nnz = 0;
  double c0 = 0.0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> va, b, c, l, u;
  std::vector<int8_t> sense;
  // prepared form and placement
  Prepared P;
  SlotLayout L;
  size_t own_tables = 0;  // bytes of the LP's own launch tables (initial products)
  size_t need = 0;        // arena bytes: slot + own tables
  size_t off = 0;
  bool placed = false;
  LpDev lpd{};
  hipEvent_t ready = nullptr;  // upload and initial products done (upload stream)
  bool stop_sent = false;
  Ctl last{};                  // control block at retirement
  JobState state = JobState::kQueued;
  bool cancel = false;
  int err = OPDHG_OK;  // error delivered by poll (OPDHG_OK: a result)
  std::string errmsg;
  std::vector<double> x, y;
  opdhg_result res{};
  Clock::time_point t_submit, t_admit, t_done;
};

// Shared launch tables at fixed offsets of the arena's table region.
struct SharedTables {
  uint8_t* base = nullptr;
  size_t o_lps = 0, o_board = 0, o_cn = 0, o_wt = 0, o_wa = 0, end = 0;
  int64_t cap_lps = 0, cap_wt = 0, cap_wa = 0;

  bool layout(uint8_t* b, size_t bytes, int64_t max_active) {
    base = b;
    o_lps = 0;
    o_board = align256(sizeof(LpDev) * max_active);
    o_cn = o_board + align256(sizeof(Ctl) * max_active);
    o_wt = o_cn + align256(sizeof(Counts));
    if (bytes < o_wt + 2 * 256 * sizeof(WorkItem)) return false;
    const size_t half = ((bytes - o_wt) / 2) & ~size_t(255);
    o_wa = o_wt + half;
    end = bytes;
    cap_lps = max_active;
    cap_wt = (int64_t)(half / sizeof(WorkItem));
    cap_wa = (int64_t)((bytes - o_wa) / sizeof(WorkItem));
    return true;
  }
};

}  // namespace

struct ServerImpl {
  opdhg_server_cfg cfg{};
  uint8_t* arena_base = nullptr;
  size_t arena_bytes = 0;
  size_t table_bytes = 0;
  size_t budget = 0;
  hipStream_t s_comp = nullptr, s_h2d = nullptr, s_d2h = nullptr;
  SharedTables tab;
  Group grp;
  int64_t wg_cap = kGridCap;
  Ctl* pinned_board = nullptr;

  std::mutex mu;
  std::condition_variable cv_prep, cv_sched, cv_done;
  bool stopping = false;
  bool failed = false;
  std::string fail_msg;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;  // not yet released
  std::deque<std::shared_ptr<Job>> to_prepare;              // submission order
  std::deque<std::shared_ptr<Job>> waiting;                 // submission order (queued or prepared)
  std::unordered_map<uint64_t, double> latency;
  Arena arena;
  size_t peak = 0;
  int64_t n_submitted = 0, n_completed = 0, n_cancelled = 0, n_failed = 0, n_replays = 0;
  int64_t n_active = 0;

  // scheduler-thread state
  std::vector<std::shared_ptr<Job>> active;  // resident, in table order
  int64_t items_t = 0, items_a = 0;          // tiles of the resident LPs

  std::vector<std::thread> th_prep;
  std::thread th_sched;

  // FP64 fallback of FP32 requests that end short of their tolerance
  bool fallback_on = false;
  int device = 0;
  hipStream_t s_fb = nullptr;
  std::deque<std::shared_ptr<Job>> to_fallback;
  std::condition_variable cv_fb;
  std::thread th_fb;
  size_t fb_wait = 0;  // arena bytes a fallback waits for (admissions pause meanwhile)
  int64_t n_fallback = 0;
  std::unordered_set<uint64_t> fell_back;  // tickets whose result is the FP64 solve's

  void prep_loop();
  void sched_loop();
  void fallback_loop();
  bool fits_tables(int64_t nlps, int64_t it, int64_t ia) const;
  int admit(Job& j);
  int write_shared();
  int retire(Job& j, bool cancelled);
  void finish_job(Job& j, int err, const std::string& msg);
  void fail_all(const std::string& msg);
};

namespace {

// Padded work-list length of a side with n items under the workgroup cap.
int64_t padded_items(int64_t n, int64_t cap) {
  int g, c;
  chunking(n, cap, &g, &c);
  return (int64_t)g * c;
}

opdhg_lp lp_view(const Job& j) {
  opdhg_lp v;
  v.m = j.m;
  v.n = j.n;
  v.nnz = j.nnz;
  v.row_ptr = j.rp.data();
  v.col_idx = j.ci.data();
  v.val = j.va.data();
  v.b = j.b.data();
  v.row_sense = j.sense.data();
  v.c = j.c.data();
  v.l = j.l.data();
  v.u = j.u.data();
  v.obj_offset = j.c0;
  return v;
}

template <typename T>
void release_vec(std::vector<T>& v) {
  std::vector<T>().swap(v);
}

}  // namespace

bool ServerImpl::fits_tables(int64_t nlps, int64_t it, int64_t ia) const {
  return nlps <= tab.cap_lps && padded_items(it, wg_cap) <= tab.cap_wt &&
         padded_items(ia, wg_cap) <= tab.cap_wa;
}

void ServerImpl::finish_job(Job& j, int err, const std::string& msg) {
  if (fallback_on) {  // the copy of the LP kept for a fallback
    release_vec(j.rp);
    release_vec(j.ci);
    release_vec(j.va);
    release_vec(j.b);
    release_vec(j.c);
    release_vec(j.l);
    release_vec(j.u);
    release_vec(j.sense);
  }
  j.err = err;
  j.errmsg = msg;
  j.state = JobState::kDone;
  j.t_done = Clock::now();
  if (err == OPDHG_ERR_CANCELLED) ++n_cancelled;
  else if (err != OPDHG_OK) ++n_failed;
  else ++n_completed;
  latency[j.ticket] = seconds_between(j.t_submit, j.t_done);
  cv_done.notify_all();
}

void ServerImpl::fail_all(const std::string& msg) {
  std::lock_guard<std::mutex> lk(mu);
  failed = true;
  fail_msg = msg;
  for (auto& kv : jobs)
    if (kv.second->state != JobState::kDone) finish_job(*kv.second, OPDHG_ERR_DEVICE, msg);
  waiting.clear();
  to_prepare.clear();
  cv_done.notify_all();
}

// Worker (one of several): takes submitted LPs in submission order and
// prepares them; admission still follows submission order.
void ServerImpl::prep_loop() {
  for (;;) {
    std::shared_ptr<Job> j;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_prep.wait(lk, [&] { return stopping || !to_prepare.empty(); });
      if (stopping) return;
      j = to_prepare.front();
      to_prepare.pop_front();
      if (j->cancel || j->state != JobState::kQueued) continue;
    }
    const opdhg_lp v = lp_view(*j);
    int rc = prepare(&v, &j->p, j->P, false);
    std::string msg = rc ? std::string(opdhg_last_error()) : std::string();
    if (!rc) {
      j->L = slot_layout(j->P, cfg.precision);
      j->own_tables = tables_bytes({&j->P}, wg_cap);
      j->need = align256(j->L.total) + align256(j->own_tables);
      if (j->need > budget) {
        rc = OPDHG_ERR_OVER_BUDGET;
        msg = "LP needs " + std::to_string(j->need) + " bytes; budget is " +
              std::to_string(budget);
      } else if (!fits_tables(1, j->P.tiles_t.size(), j->P.tiles_a.size())) {
        rc = OPDHG_ERR_OVER_BUDGET;
        msg = "LP has more tiles than the launch tables hold";
      }
    }
    if (!fallback_on) {  // else a fallback solves the LP again from its copy
      if (!j->P.dstruct) {  // else the device builds the structure from them at admission
        release_vec(j->rp);
        release_vec(j->ci);
        release_vec(j->va);
      }
      release_vec(j->b);
      release_vec(j->c);
      release_vec(j->l);
      release_vec(j->u);
      release_vec(j->sense);
    }
    std::lock_guard<std::mutex> lk(mu);
    if (j->state != JobState::kQueued) continue;  // cancelled meanwhile
    if (rc) {
      auto it = std::find(waiting.begin(), waiting.end(), j);
      if (it != waiting.end()) waiting.erase(it);
      finish_job(*j, rc, msg);
    } else {
      j->state = JobState::kPrepared;
      cv_sched.notify_all();
    }
  }
}

// Uploads a placed LP into its arena block and computes A x of its start
// point on the upload stream; records j.ready.
int ServerImpl::admit(Job& j) {
  uint8_t* base = arena_base + table_bytes + j.off;
  SlotImage img;
  int rc = upload_slot(base, j.L, j.P, cfg.precision, s_h2d, img);
  if (rc) return rc;
  j.lpd = slot_pointers(base, j.L, j.P);
  // the staging image (and the LP's own arrays) must outlive the copy
  HIP_TRY(hipStreamSynchronize(s_h2d));
  if (j.P.dstruct) {
    if (!fallback_on) {
      release_vec(j.rp);
      release_vec(j.ci);
      release_vec(j.va);
    }
    j.P.h_rp = nullptr;
    j.P.h_ci = nullptr;
    j.P.h_val = nullptr;
  }
  LaunchCfg own{};
  std::vector<uint8_t> staging;
  int64_t nwt = 0, nwa = 0;
  if ((rc = write_tables(base + align256(j.L.total), {j.lpd}, {&j.P}, wg_cap, s_h2d, staging,
                         &own, &nwt, &nwa)))
    return rc;
  rc = cfg.precision == OPDHG_FP32 ? Kernels<float>::init_products(own, s_h2d)
                                   : Kernels<double>::init_products(own, s_h2d);
  if (rc) return fail(OPDHG_ERR_DEVICE, device_error_string());
  HIP_TRY(hipEventCreateWithFlags(&j.ready, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(j.ready, s_h2d));
  // the table staging vector is pageable and goes away here
  HIP_TRY(hipStreamSynchronize(s_h2d));
  return OPDHG_OK;
}

// Rewrites the shared launch tables for the resident set (compute stream,
// between launch sequences).
int ServerImpl::write_shared() {
  std::vector<LpDev> lps;
  std::vector<const Prepared*> preps;
  for (auto& j : active) {
    lps.push_back(j->lpd);
    preps.push_back(&j->P);
  }
  std::vector<WorkItem> wt, wa;
  int gt = 1, ct = 1, ga = 1, ca = 1;
  side_items(lps, preps, true, wg_cap, &gt, &ct, wt);
  side_items(lps, preps, false, wg_cap, &ga, &ca, wa);
  // the step kernels run the evaluation lists, one partial slot per tile
  for (size_t i = 0; i < lps.size(); ++i) {
    lps[i].nslot_st = (int32_t)preps[i]->tiles_t.size();
    lps[i].nslot_sa = (int32_t)preps[i]->tiles_a.size();
  }
  if ((int64_t)wt.size() > tab.cap_wt || (int64_t)wa.size() > tab.cap_wa ||
      (int64_t)lps.size() > tab.cap_lps)
    return fail(OPDHG_ERR_OVER_BUDGET, "launch tables overflow");
  Counts cn{(int32_t)items_t, (int32_t)items_a, (int32_t)lps.size(), 0, gt, ct, ga, ca,
            {1, 1}, {0, 0}};  // a changed set: let the next guarded evaluations look
  if (!lps.empty())
    HIP_TRY(hipMemcpyAsync(tab.base + tab.o_lps, lps.data(), sizeof(LpDev) * lps.size(),
                           hipMemcpyHostToDevice, s_comp));
  HIP_TRY(hipMemcpyAsync(tab.base + tab.o_wt, wt.data(), sizeof(WorkItem) * wt.size(),
                         hipMemcpyHostToDevice, s_comp));
  HIP_TRY(hipMemcpyAsync(tab.base + tab.o_wa, wa.data(), sizeof(WorkItem) * wa.size(),
                         hipMemcpyHostToDevice, s_comp));
  HIP_TRY(hipMemcpyAsync(tab.base + tab.o_cn, &cn, sizeof(cn), hipMemcpyHostToDevice, s_comp));
  // pageable sources: wait before the vectors go away
  HIP_TRY(hipStreamSynchronize(s_comp));
  return OPDHG_OK;
}

// Downloads a finished LP's returned iterate, fills its result and frees
// its block (no launch references it any more).
int ServerImpl::retire(Job& j, bool cancelled) {
  int rc = OPDHG_OK;
  if (!cancelled) {
    const Ctl& c = j.last;
    std::vector<double> tmp;
    j.x.assign(j.P.n, 0.0);
    tmp.resize(j.P.n);
    rc = download_vec(j.lpd.x[c.cur], j.P.n, cfg.precision, s_d2h, tmp.data());
    if (!rc) unpermute(tmp.data(), j.P.perm_t, j.P.dc.data(), j.x.data());
    if (!rc && j.P.m) {
      j.y.assign(j.P.m, 0.0);
      tmp.resize(j.P.m);
      rc = download_vec(j.lpd.y[c.cur], j.P.m, cfg.precision, s_d2h, tmp.data());
      if (!rc) unpermute(tmp.data(), j.P.perm_a, j.P.dr.data(), j.y.data());
    }
    fill_result(c, seconds_between(j.t_admit, Clock::now()), &j.res);
  }
  const std::string msg = rc ? std::string(opdhg_last_error()) : std::string();
  if (j.ready) (void)hipEventDestroy(j.ready);
  j.ready = nullptr;
  j.P = Prepared();
  std::lock_guard<std::mutex> lk(mu);
  if (j.placed) arena.release(j.off, j.need);
  j.placed = false;
  --n_active;
  cv_fb.notify_all();  // a fallback may be waiting for the memory
  const bool short_of_tol = j.res.status == OPDHG_STATUS_ITERATION_LIMIT ||
                            j.res.status == OPDHG_STATUS_NUMERICAL_ERROR;
  if (fallback_on && !cancelled && rc == OPDHG_OK && !stopping && short_of_tol) {
    auto it = jobs.find(j.ticket);
    if (it != jobs.end()) {
      to_fallback.push_back(it->second);
      return rc;
    }
  }
  finish_job(j, cancelled ? OPDHG_ERR_CANCELLED : rc, cancelled ? "cancelled" : msg);
  return rc;
}

// Fallback worker: solves the handed-over FP32 requests again in FP64, one
// at a time, on its own stream, in arena memory taken like an admission. The
// FP32 result stands where the fallback cannot run.
void ServerImpl::fallback_loop() {
  (void)hipSetDevice(device);
  for (;;) {
    std::shared_ptr<Job> j;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_fb.wait(lk, [&] { return stopping || !to_fallback.empty(); });
      if (to_fallback.empty()) return;
      j = to_fallback.front();
      to_fallback.pop_front();
      if (j->cancel || stopping) {
        finish_job(*j, j->cancel ? OPDHG_ERR_CANCELLED : OPDHG_OK, j->cancel ? "cancelled" : "");
        continue;
      }
    }
    opdhg_params p64 = j->p;
    p64.precision = OPDHG_FP64;
    const opdhg_lp v = lp_view(*j);
    size_t need = 0;
    int rc = opdhg_workspace_bytes(&v, &p64, &need);
    need = align256(need);
    size_t off = 0;
    bool got = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (rc || need > budget) {
        finish_job(*j, OPDHG_OK, "");
        continue;
      }
      fb_wait = need;
      while (!stopping && !j->cancel && !(got = arena.alloc(need, &off)))
        cv_fb.wait_for(lk, std::chrono::duration<double>(std::max(cfg.poll_interval_s, 1e-4)));
      fb_wait = 0;
      cv_sched.notify_all();
      if (!got) {
        finish_job(*j, j->cancel ? OPDHG_ERR_CANCELLED : OPDHG_OK, j->cancel ? "cancelled" : "");
        continue;
      }
      peak = std::max(peak, arena.used());
    }
    std::vector<double> x((size_t)j->n), y((size_t)std::max<int64_t>(j->m, 1));
    opdhg_result res{};
    rc = opdhg_solve(&v, &p64, arena_base + table_bytes + off, need, s_fb, x.data(), y.data(),
                     &res);
    const std::string msg = rc ? std::string(opdhg_last_error()) : std::string();
    std::lock_guard<std::mutex> lk(mu);
    arena.release(off, need);
    cv_sched.notify_all();
    if (rc == OPDHG_OK) {
      y.resize((size_t)j->m);
      j->x.swap(x);
      j->y.swap(y);
      j->res = res;
      ++n_fallback;
      fell_back.insert(j->ticket);
      finish_job(*j, OPDHG_OK, "");
    } else {
      // a device error is the request's; otherwise the FP32 result stands
      finish_job(*j, rc == OPDHG_ERR_DEVICE ? rc : OPDHG_OK, rc == OPDHG_ERR_DEVICE ? msg : "");
    }
  }
}

void ServerImpl::sched_loop() {
  static const int32_t one = 1;
  std::vector<std::shared_ptr<Job>> finished;  // retire while the next sequence runs
  bool dirty = false;
  for (;;) {
    // 1. launch the resident set
    const bool running = !active.empty();
    if (running) {
      if (grp.replay() != OPDHG_OK ||
          hipMemcpyAsync(pinned_board, tab.base + tab.o_board, sizeof(Ctl) * active.size(),
                         hipMemcpyDeviceToHost, s_comp) != hipSuccess) {
        fail_all(std::string("launch failed: ") + opdhg_last_error());
        return;
      }
      std::lock_guard<std::mutex> lk(mu);
      ++n_replays;
    }
    // 2. while it runs: retire LPs that finished in the previous sequence
    for (auto& j : finished) {
      if (retire(*j, j->cancel) != OPDHG_OK && j->err == OPDHG_ERR_DEVICE) {
        fail_all(j->errmsg);
        return;
      }
    }
    finished.clear();
    // ... and admit waiting LPs in submission order
    std::vector<std::shared_ptr<Job>> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stopping) break;
      while (!waiting.empty()) {
        auto& j = waiting.front();
        if (j->cancel) {
          finish_job(*j, OPDHG_ERR_CANCELLED, "cancelled");
          waiting.pop_front();
          continue;
        }
        if (j->state != JobState::kPrepared) break;
        const int64_t nl = (int64_t)(active.size() + admitted.size()) + 1;
        int64_t it = items_t, ia = items_a;
        for (auto& a : admitted) {
          it += a->P.tiles_t.size();
          ia += a->P.tiles_a.size();
        }
        it += j->P.tiles_t.size();
        ia += j->P.tiles_a.size();
        if (nl > cfg.max_active || !fits_tables(nl, it, ia)) break;
        if (fb_wait > 0) break;  // a fallback takes freed memory first
        size_t off = 0;
        if (!arena.alloc(j->need, &off)) break;
        j->off = off;
        j->placed = true;
        j->state = JobState::kAdmitted;
        j->t_admit = Clock::now();
        peak = std::max(peak, arena.used());
        ++n_active;
        admitted.push_back(j);
        waiting.pop_front();
      }
    }
    for (auto& j : admitted) {
      if (admit(*j) != OPDHG_OK) {
        fail_all(std::string("admission failed: ") + opdhg_last_error());
        return;
      }
    }
    // 3. wait for the sequence; read the resident LPs' control blocks
    if (running && hipStreamSynchronize(s_comp) != hipSuccess) {
      fail_all("compute stream failed");
      return;
    }
    std::vector<std::shared_ptr<Job>> keep;
    std::unique_lock<std::mutex> lk3(mu);
    for (size_t i = 0; i < active.size(); ++i) {
      auto& j = active[i];
      const Ctl& c = pinned_board[i];
      if (c.status != kRunning || j->cancel) {
        j->last = c;
        j->state = JobState::kFinished;
        finished.push_back(j);
        items_t -= j->P.tiles_t.size();
        items_a -= j->P.tiles_a.size();
        dirty = true;
        continue;
      }
      if (!j->stop_sent && seconds_between(j->t_admit, Clock::now()) > j->p.time_limit_s) {
        // final evaluation at the start of the next sequence
        if (hipMemcpyAsync(&j->lpd.ctl->stop_request, &one, sizeof(one), hipMemcpyHostToDevice,
                           s_comp) != hipSuccess ||
            hipMemcpyAsync(&j->lpd.ctl->need_eval, &one, sizeof(one), hipMemcpyHostToDevice,
                           s_comp) != hipSuccess) {
          lk3.unlock();
          fail_all("time-limit request failed");
          return;
        }
        j->stop_sent = true;
      }
      keep.push_back(j);
    }
    active.swap(keep);
    bool wait_ok = true;
    for (auto& j : admitted) {
      wait_ok = wait_ok && hipStreamWaitEvent(s_comp, j->ready, 0) == hipSuccess;
      active.push_back(j);
      items_t += j->P.tiles_t.size();
      items_a += j->P.tiles_a.size();
      j->state = JobState::kActive;
      dirty = true;
    }
    lk3.unlock();
    if (!wait_ok) {
      fail_all("stream wait failed");
      return;
    }
    if (dirty && !active.empty()) {
      if (write_shared() != OPDHG_OK) {
        fail_all(std::string("table update failed: ") + opdhg_last_error());
        return;
      }
    }
    dirty = false;
    // 4. idle: nothing resident and nothing retiring
    if (active.empty() && finished.empty()) {
      std::unique_lock<std::mutex> lk(mu);
      if (stopping) break;
      const bool ready = !waiting.empty() && (waiting.front()->state == JobState::kPrepared ||
                                              waiting.front()->cancel);
      if (!ready)
        cv_sched.wait_for(lk, std::chrono::duration<double>(cfg.poll_interval_s));
    }
  }
  // shutdown: resident LPs are dropped
  (void)hipStreamSynchronize(s_comp);
  (void)hipStreamSynchronize(s_h2d);
  for (auto& j : finished) (void)retire(*j, true);
  for (auto& j : active) (void)retire(*j, true);
  active.clear();
}

}  // namespace opdhg

using namespace opdhg;

struct opdhg_server {
  ServerImpl impl;
};

extern "C" {

void opdhg_server_default_cfg(opdhg_server_cfg* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->budget_bytes = 0;
  cfg->max_active = 256;
  cfg->attempts_per_replay = 64;
  cfg->precision = OPDHG_FP32;
  cfg->workgroups = 0;
  cfg->prep_threads = 0;
  cfg->fallback = OPDHG_FALLBACK_NONE;
  cfg->poll_interval_s = 1e-3;
}

opdhg_server* opdhg_server_create(const opdhg_server_cfg* cfg, void* d_arena, size_t arena_bytes,
                                  void* compute_stream, void* h2d_stream, void* d2h_stream) {
  if (!cfg || !d_arena) {
    fail(OPDHG_ERR_INVALID_ARGUMENT, "cfg and arena are required");
    return nullptr;
  }
  if (cfg->max_active < 1 || cfg->max_active > 65535 || cfg->attempts_per_replay < 1 ||
      cfg->attempts_per_replay > kPowRing ||
      (cfg->precision != OPDHG_FP32 && cfg->precision != OPDHG_FP64) || cfg->workgroups < 0 ||
      cfg->prep_threads < 0 || cfg->prep_threads > 64 ||
      (cfg->fallback != OPDHG_FALLBACK_NONE && cfg->fallback != OPDHG_FALLBACK_FP64) ||
      cfg->workgroups > kMaxGrid || !(cfg->poll_interval_s >= 0.0)) {
    fail(OPDHG_ERR_INVALID_ARGUMENT, "bad server configuration");
    return nullptr;
  }
  if (reinterpret_cast<uintptr_t>(d_arena) % 256) {
    fail(OPDHG_ERR_INVALID_ARGUMENT, "arena must be 256-byte aligned");
    return nullptr;
  }
  auto s = std::make_unique<opdhg_server>();
  ServerImpl& S = s->impl;
  S.cfg = *cfg;
  S.arena_base = static_cast<uint8_t*>(d_arena);
  S.arena_bytes = arena_bytes;
  S.table_bytes = align256(std::min<size_t>(std::max<size_t>(arena_bytes / 64, 4u << 20), 1u << 30));
  if (arena_bytes <= S.table_bytes) {
    fail(OPDHG_ERR_OVER_BUDGET, "arena too small for the launch tables");
    return nullptr;
  }
  const size_t room = (arena_bytes - S.table_bytes) & ~size_t(255);
  S.budget = cfg->budget_bytes ? std::min(cfg->budget_bytes, room) : room;
  S.wg_cap = cfg->workgroups > 0 ? cfg->workgroups : kGridCap;
  if (!S.tab.layout(S.arena_base, S.table_bytes, cfg->max_active)) {
    fail(OPDHG_ERR_OVER_BUDGET, "launch tables do not fit");
    return nullptr;
  }
  S.arena.reset(S.budget);
  S.s_comp = (hipStream_t)compute_stream;
  S.s_h2d = h2d_stream ? (hipStream_t)h2d_stream : S.s_comp;
  S.s_d2h = d2h_stream ? (hipStream_t)d2h_stream : S.s_comp;
  if (S.grp.init(compute_stream, cfg->precision)) return nullptr;
  LaunchCfg& L = S.grp.cfg;
  L.lps = reinterpret_cast<const LpDev*>(S.tab.base + S.tab.o_lps);
  L.work_t = reinterpret_cast<const WorkItem*>(S.tab.base + S.tab.o_wt);
  L.work_a = reinterpret_cast<const WorkItem*>(S.tab.base + S.tab.o_wa);
  L.counts = reinterpret_cast<const Counts*>(S.tab.base + S.tab.o_cn);
  L.board = reinterpret_cast<Ctl*>(S.tab.base + S.tab.o_board);
  // the step kernels run the same lists with the device-side chunking; no
  // request has windowed chunks (windows are off for every submission)
  L.step_t = L.work_t;
  L.step_a = L.work_a;
  L.step_fixed = 0;
  L.win_t = L.win_a = nullptr;
  L.nwin_t = L.nwin_a = 0;
  L.seg_t = L.seg_a = nullptr;
  L.nseg_t = L.nseg_a = 0;
  const int g8 = (int)((S.wg_cap + 7) / 8 * 8);
  L.launch_t = L.launch_a = L.launch_ta = g8;
  L.launch_lp = std::min(cfg->max_active, kGridCap);
  // an empty set until the first admission
  const Counts cn{0, 0, 0, 0, 0, 1, 0, 1, {0, 0}, {0, 0}};
  if (hipMemcpyAsync((void*)L.counts, &cn, sizeof(cn), hipMemcpyHostToDevice, S.s_comp) !=
          hipSuccess ||
      hipStreamSynchronize(S.s_comp) != hipSuccess) {
    fail(OPDHG_ERR_DEVICE, "initializing the launch tables failed");
    S.grp.release();
    return nullptr;
  }
  // the server's mix holds several LPs at once (or will)
  S.grp.mid_every = cfg->max_active > 1 ? kMidEvalEveryShared : kMidEvalEvery;
  if (S.grp.capture(cfg->attempts_per_replay)) {
    S.grp.release();
    return nullptr;
  }
  if (hipHostMalloc((void**)&S.pinned_board, sizeof(Ctl) * cfg->max_active,
                    hipHostMallocDefault) != hipSuccess) {
    fail(OPDHG_ERR_DEVICE, "pinned host allocation failed");
    S.grp.release();
    return nullptr;
  }
  S.fallback_on = cfg->fallback == OPDHG_FALLBACK_FP64 && cfg->precision == OPDHG_FP32;
  if (S.fallback_on &&
      (hipGetDevice(&S.device) != hipSuccess ||
       hipStreamCreateWithFlags(&S.s_fb, hipStreamNonBlocking) != hipSuccess)) {
    fail(OPDHG_ERR_DEVICE, "creating the fallback stream failed");
    (void)hipHostFree(S.pinned_board);
    S.grp.release();
    return nullptr;
  }
  const int nprep = cfg->prep_threads > 0 ? cfg->prep_threads
                                          : std::max(1, std::min(host_threads() / 2, 8));
  for (int t = 0; t < nprep; ++t) S.th_prep.emplace_back([&S] { S.prep_loop(); });
  S.th_sched = std::thread([&S] { S.sched_loop(); });
  if (S.fallback_on) S.th_fb = std::thread([&S] { S.fallback_loop(); });
  return s.release();
}

int opdhg_server_submit(opdhg_server* s, const opdhg_lp* lp, const opdhg_params* p,
                        uint64_t* ticket) {
  if (!s || !ticket) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  ServerImpl& S = s->impl;
  int rc = validate_lp(lp);
  if (rc) return rc;
  if ((rc = validate_params(p))) return rc;
  if (p->precision != S.cfg.precision)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "request precision differs from the server's");
  auto j = std::make_shared<Job>();
  j->p = *p;
  // one captured launch sequence serves every mix of requests: tiles only
  j->p.windows = OPDHG_WINDOWS_OFF;
  j->m = lp->m;
  j->n = lp->n;
  j->nnz = lp->nnz;
  j->c0 = lp->obj_offset;
  j->rp.assign(lp->row_ptr, lp->row_ptr + lp->m + 1);
  j->ci.assign(lp->col_idx, lp->col_idx + lp->nnz);
  j->va.assign(lp->val, lp->val + lp->nnz);
  j->b.assign(lp->b, lp->b + lp->m);
  j->sense.assign(lp->row_sense, lp->row_sense + lp->m);
  j->c.assign(lp->c, lp->c + lp->n);
  j->l.assign(lp->l, lp->l + lp->n);
  j->u.assign(lp->u, lp->u + lp->n);
  j->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(S.mu);
  if (S.failed) return fail(OPDHG_ERR_DEVICE, "server failed: " + S.fail_msg);
  if (S.stopping) return fail(OPDHG_ERR_INVALID_ARGUMENT, "server is shutting down");
  j->ticket = S.next_ticket++;
  S.jobs[j->ticket] = j;
  S.to_prepare.push_back(j);
  S.waiting.push_back(j);
  ++S.n_submitted;
  *ticket = j->ticket;
  S.cv_prep.notify_one();
  return OPDHG_OK;
}

static int deliver(ServerImpl& S, std::shared_ptr<Job> j, double* x, double* y,
                   opdhg_result* res) {
  // called with S.mu held and j done; releases the ticket
  S.jobs.erase(j->ticket);
  if (j->err != OPDHG_OK) return fail(j->err, j->errmsg);
  if (x) std::copy(j->x.begin(), j->x.end(), x);
  if (y) std::copy(j->y.begin(), j->y.end(), y);
  if (res) *res = j->res;
  return OPDHG_OK;
}

int opdhg_server_poll(opdhg_server* s, uint64_t ticket, double* x, double* y,
                      opdhg_result* res) {
  if (!s) return fail(OPDHG_ERR_INVALID_ARGUMENT, "server is NULL");
  ServerImpl& S = s->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.jobs.find(ticket);
  if (it == S.jobs.end()) return fail(OPDHG_ERR_UNKNOWN_TICKET, "unknown or released ticket");
  if (it->second->state != JobState::kDone) return fail(OPDHG_ERR_NOT_READY, "not ready");
  return deliver(S, it->second, x, y, res);
}

int opdhg_server_wait(opdhg_server* s, uint64_t ticket, double timeout_s, double* x, double* y,
                      opdhg_result* res) {
  if (!s) return fail(OPDHG_ERR_INVALID_ARGUMENT, "server is NULL");
  ServerImpl& S = s->impl;
  std::unique_lock<std::mutex> lk(S.mu);
  auto it = S.jobs.find(ticket);
  if (it == S.jobs.end()) return fail(OPDHG_ERR_UNKNOWN_TICKET, "unknown or released ticket");
  std::shared_ptr<Job> j = it->second;
  const auto done = [&] { return j->state == JobState::kDone; };
  if (timeout_s < 0) S.cv_done.wait(lk, done);
  else if (!S.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done))
    return fail(OPDHG_ERR_NOT_READY, "not ready");
  return deliver(S, j, x, y, res);
}

int opdhg_server_cancel(opdhg_server* s, uint64_t ticket) {
  if (!s) return fail(OPDHG_ERR_INVALID_ARGUMENT, "server is NULL");
  ServerImpl& S = s->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.jobs.find(ticket);
  if (it == S.jobs.end()) return fail(OPDHG_ERR_UNKNOWN_TICKET, "unknown or released ticket");
  Job& j = *it->second;
  if (j.state == JobState::kDone) return OPDHG_OK;
  j.cancel = true;
  if (j.state == JobState::kQueued || j.state == JobState::kPrepared) {
    auto w = std::find(S.waiting.begin(), S.waiting.end(), it->second);
    if (w != S.waiting.end()) S.waiting.erase(w);
    S.finish_job(j, OPDHG_ERR_CANCELLED, "cancelled");
  }
  // resident LPs are dropped at the next sequence boundary
  S.cv_sched.notify_all();
  return OPDHG_OK;
}

int opdhg_server_get_stats(opdhg_server* s, opdhg_server_stats* out) {
  if (!s || !out) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  ServerImpl& S = s->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  out->submitted = S.n_submitted;
  out->completed = S.n_completed;
  out->cancelled = S.n_cancelled;
  out->failed = S.n_failed;
  out->active = S.n_active;
  out->queued = (int64_t)S.waiting.size();
  out->replays = S.n_replays;
  out->bytes_in_use = S.arena.used();
  out->peak_bytes = S.peak;
  out->fallbacks = S.n_fallback;
  return OPDHG_OK;
}

int opdhg_server_latency(opdhg_server* s, uint64_t ticket, double* seconds) {
  if (!s || !seconds) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  ServerImpl& S = s->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.latency.find(ticket);
  if (it == S.latency.end()) return fail(OPDHG_ERR_NOT_READY, "no latency for this ticket yet");
  *seconds = it->second;
  return OPDHG_OK;
}

int opdhg_server_precision(opdhg_server* s, uint64_t ticket, int32_t* precision) {
  if (!s || !precision) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  ServerImpl& S = s->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  if (S.latency.find(ticket) == S.latency.end())
    return fail(OPDHG_ERR_NOT_READY, "no result for this ticket yet");
  *precision = S.fell_back.count(ticket) ? OPDHG_FP64 : S.cfg.precision;
  return OPDHG_OK;
}

void opdhg_server_destroy(opdhg_server* s) {
  if (!s) return;
  ServerImpl& S = s->impl;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stopping = true;
  }
  S.cv_prep.notify_all();
  S.cv_sched.notify_all();
  S.cv_fb.notify_all();
  for (auto& t : S.th_prep)
    if (t.joinable()) t.join();
  if (S.th_sched.joinable()) S.th_sched.join();
  if (S.th_fb.joinable()) S.th_fb.join();  // a solve in progress finishes first
  if (S.s_fb) (void)hipStreamDestroy(S.s_fb);
  if (S.pinned_board) (void)hipHostFree(S.pinned_board);
  S.grp.release();
  delete s;
}

}  // extern "C"
