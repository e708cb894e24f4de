// Autotuner of the sparse-product tiling for a set of LPs.
//
// The LPs are prepared once (validation, rescaling, transposes); each
// candidate tiling then re-tiles both CSR sides, uploads the set, captures
// the launch sequence and times replays of it on the device. The candidate
// with the most step attempts per second, summed over the set, wins. In
// FP64 every tiling gives the same result bit for bit (exact sums); in FP32
// the tiling moves results only by rounding (a row's products are summed by
// its tile's lane group).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <limits>
#include <string>
#include <thread>
#include <vector>

#include "opdhg.h"
#include "opdhg_host.h"
#include "opdhg_internal.h"

namespace opdhg {
namespace {

struct Candidate {
  int tile_nnz, lanes, workgroups;
};

constexpr int kSlots = 64;  // step-attempt slots per timed launch sequence

// tile sizes x workgroup counts; lanes per row are picked per tile
constexpr Candidate kCandidates[] = {
    {256, 0, 256},  {256, 0, 512},  {256, 0, 1024},  {256, 0, 2048},
    {512, 0, 256},  {512, 0, 512},  {512, 0, 1024},  {512, 0, 2048},
    {1024, 0, 256}, {1024, 0, 512}, {1024, 0, 1024}, {1024, 0, kGridCap},
};

void retile(Prepared& P, int64_t cap, int lanes) {
  P.tiles_a = build_tiles(P.rp_a.data(), P.m, cap, lanes);
  P.tiles_t = build_tiles(P.rp_t.data(), P.n, cap, lanes);
  step_tiles(P, cap, lanes);  // windowed chunks do not depend on the tiling
}

// Workspace bytes of the set under one candidate (tiles already built).
size_t set_bytes(const std::vector<Prepared>& P, int prec, int64_t wg_cap) {
  size_t total = 0;
  std::vector<const Prepared*> preps;
  for (const Prepared& q : P) {
    total += slot_layout(q, prec).total;
    preps.push_back(&q);
  }
  return total + tables_bytes(preps, wg_cap);
}

// Whether the windowed candidate is tried: FP32 with automatic windows.
bool try_windows(const opdhg_params* p) {
  return p->precision == OPDHG_FP32 && p->windows == OPDHG_WINDOWS_AUTO;
}

// The parameters of the windowed candidate.
opdhg_params windowed(const opdhg_params* p) {
  opdhg_params q = *p;
  q.windows = OPDHG_WINDOWS_ALWAYS;
  q.window_rows = kWinRows;
  return q;
}

// Prepares every LP with parameters that keep it running while timed.
int prepare_set(int count, const opdhg_lp* lps, const opdhg_params* p, std::vector<Prepared>& P) {
  opdhg_params q = *p;
  q.tol = 0.0;
  q.max_iter = std::numeric_limits<int64_t>::max() / 4;
  q.time_limit_s = 1e30;
  P.assign(count, Prepared());
  // the LPs are independent: up to 16 host threads take them in turn
  std::vector<int> rcs(count, OPDHG_OK);
  std::vector<std::string> msgs(count);
  std::atomic<int> next{0};
  auto work = [&] {
    for (int i = next++; i < count; i = next++) {
      int rc = validate_lp(&lps[i]);
      if (!rc) rc = prepare(&lps[i], &q, P[i], false);
      if (rc) {
        rcs[i] = rc;
        msgs[i] = opdhg_last_error();
      }
    }
  };
  const int nth = std::max(1, std::min({count, host_threads(), 16}));
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  for (int i = 0; i < count; ++i)
    if (rcs[i]) return fail(rcs[i], "LP " + std::to_string(i) + ": " + msgs[i]);
  return OPDHG_OK;
}

size_t max_bytes(std::vector<Prepared>& P, int prec) {
  size_t need = 0;
  for (const Candidate& c : kCandidates) {
    for (Prepared& q : P) retile(q, c.tile_nnz, c.lanes);
    need = std::max(need, set_bytes(P, prec, c.workgroups));
  }
  return need;
}

// Attempts per second of the set under one candidate: upload, capture,
// one warm-up replay, then `replays` timed replays.
int time_candidate(std::vector<Prepared>& P, int prec, int mid_every, const Candidate& cand,
                   uint8_t* ws, void* stream, int replays, double* rate, double* executed) {
  const int count = (int)P.size();
  for (Prepared& q : P) retile(q, cand.tile_nnz, cand.lanes);
  Group grp;
  int rc = grp.init(stream, prec);
  if (rc) return rc;
  grp.mid_every = mid_every;
  std::vector<LpDev> lpd(count);
  std::vector<const Prepared*> preps(count);
  SlotImage img;
  std::vector<uint8_t> staging;
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    const SlotLayout L = slot_layout(P[i], prec);
    if ((rc = upload_slot(ws + off, L, P[i], prec, grp.stream, img))) break;
    lpd[i] = slot_pointers(ws + off, L, P[i]);
    preps[i] = &P[i];
    off += L.total;
    if (hipStreamSynchronize(grp.stream) != hipSuccess) rc = fail(OPDHG_ERR_DEVICE, "upload");
    if (rc) break;
  }
  int64_t nwt = 0, nwa = 0;
  if (!rc) rc = write_tables(ws + off, lpd, preps, cand.workgroups, grp.stream, staging, &grp.cfg,
                            &nwt, &nwa);
  if (!rc && grp.launch_init()) rc = fail(OPDHG_ERR_DEVICE, device_error_string());
  if (!rc && hipStreamSynchronize(grp.stream) != hipSuccess) rc = fail(OPDHG_ERR_DEVICE, "init");
  if (!rc) rc = grp.capture(kSlots);
  std::vector<Ctl> b0(count), b1(count);
  auto board = [&](std::vector<Ctl>& out) {
    if (hipMemcpyAsync(out.data(), grp.cfg.board, sizeof(Ctl) * count, hipMemcpyDeviceToHost,
                       grp.stream) != hipSuccess ||
        hipStreamSynchronize(grp.stream) != hipSuccess)
      return fail(OPDHG_ERR_DEVICE, "board readback");
    return OPDHG_OK;
  };
  if (!rc) rc = grp.replay();
  if (!rc) rc = board(b0);
  auto t0 = std::chrono::steady_clock::now();
  for (int r = 0; r < replays && !rc; ++r) rc = grp.replay();
  if (!rc) rc = board(b1);
  const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  grp.release();
  if (rc) return rc;
  int64_t att = 0;
  for (int i = 0; i < count; ++i) att += b1[i].attempts - b0[i].attempts;
  *rate = dt > 0.0 ? (double)att / dt : 0.0;
  // the LPs never stop here, so every slot of every replay could hold an attempt
  *executed = (double)att / ((double)replays * kSlots * count);
  return OPDHG_OK;
}

}  // namespace
}  // namespace opdhg

using namespace opdhg;

extern "C" {

int opdhg_autotune_workspace_bytes(int count, const opdhg_lp* lps, const opdhg_params* p,
                                   size_t* bytes) {
  if (count < 1 || !lps || !bytes) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  int rc = validate_params(p);
  if (rc) return rc;
  std::vector<Prepared> P(count);
  for (int i = 0; i < count; ++i) {
    if ((rc = validate_lp(&lps[i]))) return rc;
    prepare(&lps[i], p, P[i], true);
  }
  *bytes = max_bytes(P, p->precision);
  if (try_windows(p)) {
    const opdhg_params q = windowed(p);
    for (int i = 0; i < count; ++i) prepare(&lps[i], &q, P[i], true);
    *bytes = std::max(*bytes, max_bytes(P, p->precision));
  }
  return OPDHG_OK;
}

int opdhg_autotune(int count, const opdhg_lp* lps, const opdhg_params* p, void* d_workspace,
                   size_t workspace_bytes, void* hip_stream, int replays, opdhg_tuning* out) {
  if (count < 1 || !lps || !d_workspace || !out || replays < 1)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  int rc = validate_params(p);
  if (rc) return rc;
  std::vector<Prepared> P, PW;
  if ((rc = prepare_set(count, lps, p, P))) return rc;
  size_t need = max_bytes(P, p->precision);
  const opdhg_params pw = windowed(p);
  if (try_windows(p)) {
    if ((rc = prepare_set(count, lps, &pw, PW))) return rc;
    need = std::max(need, max_bytes(PW, p->precision));
  }
  if (workspace_bytes < need)
    return fail(OPDHG_ERR_WORKSPACE_TOO_SMALL, "workspace needs " + std::to_string(need) + " bytes");
  std::memset(out, 0, sizeof(*out));
  out->windows = p->windows;
  out->window_rows = p->window_rows;
  double best = -1.0;
  for (const Candidate& c : kCandidates) {
    double rate = 0.0, executed = 0.0;
    if ((rc = time_candidate(P, p->precision, mid_eval_every(p, count), c,
                             static_cast<uint8_t*>(d_workspace), hip_stream, replays, &rate,
                             &executed)))
      return rc;
    if (c.tile_nnz == kTileCap && c.lanes == 0 && c.workgroups == kGridCap)
      out->default_attempts_per_s = rate;
    if (rate > best) {
      best = rate;
      out->tile_nnz = c.tile_nnz;
      out->lanes = c.lanes;
      out->workgroups = c.workgroups;
      out->attempts_per_s = rate;
      out->executed_fraction = executed;
    }
    ++out->candidates;
  }
  if (try_windows(p)) {
    // the best tiling once more, with windowed chunks wherever they pay
    const Candidate c{out->tile_nnz, out->lanes, out->workgroups};
    double rate = 0.0, executed = 0.0;
    if ((rc = time_candidate(PW, p->precision, mid_eval_every(&pw, count), c,
                             static_cast<uint8_t*>(d_workspace), hip_stream, replays, &rate,
                             &executed)))
      return rc;
    if (rate > best) {
      out->attempts_per_s = rate;
      out->executed_fraction = executed;
      out->windows = pw.windows;
      out->window_rows = pw.window_rows;
    }
    ++out->candidates;
  }
  return OPDHG_OK;
}

}  // extern "C"
