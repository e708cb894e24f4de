// Host side of the opdhg library: validation, rescaling, CSR transpose,
// tiling, workspace layout, upload, graph capture and the replay loop for
// single solves, sessions and packed batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "crmath.h"
#include "opdhg.h"
#include "opdhg_host.h"
#include "opdhg_internal.h"

namespace opdhg {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int host_threads() {
  const unsigned hw = std::thread::hardware_concurrency();
  return hw ? (int)hw : 1;
}

// f(b, lo, hi) for blocks b = 0..nb-1 of [0, items) (equal sizes), on up
// to 16 host threads. The blocks depend only on items and nb, never on the
// thread count, so work split this way gives the same result on any host.
template <typename F>
static void for_blocks(int64_t items, int nb, F&& f) {
  const int nth = std::max(1, std::min({host_threads(), 16, nb}));
  std::atomic<int> next{0};
  auto work = [&] {
    for (int b = next++; b < nb; b = next++) f(b, items * b / nb, items * (b + 1) / nb);
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
}

// Blocks for for_blocks: about 64k items each, at most 64.
static int item_blocks(int64_t items) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, items / 65536));
}

int fail_hip(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return OPDHG_ERR_DEVICE;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------

// f(r0, r1) on row ranges of about equal nonzeros, on up to 16 host threads
template <typename F>
static void parallel_rows(const int64_t* ptr, int64_t rows, F&& f);

int validate_lp(const opdhg_lp* lp) {
  if (!lp) return fail(OPDHG_ERR_INVALID_ARGUMENT, "lp is NULL");
  const int64_t m = lp->m, n = lp->n, nnz = lp->nnz;
  if (n < 1) return fail(OPDHG_ERR_INVALID_ARGUMENT, "n must be at least 1");
  if (m < 0) return fail(OPDHG_ERR_INVALID_ARGUMENT, "m must be nonnegative");
  if (nnz < 0 || nnz >= (int64_t(1) << 31))
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "nnz must be in [0, 2^31)");
  if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31))
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "m and n must be below 2^31");
  if (!lp->row_ptr || !lp->c || !lp->l || !lp->u)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "NULL array");
  if (m > 0 && (!lp->b || !lp->row_sense))
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "NULL array");
  if (nnz > 0 && (!lp->col_idx || !lp->val))
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "NULL array");
  if (lp->row_ptr[0] != 0) return fail(OPDHG_ERR_INVALID_ARGUMENT, "row_ptr[0] must be 0");
  for (int64_t i = 0; i < m; ++i)
    if (lp->row_ptr[i + 1] < lp->row_ptr[i])
      return fail(OPDHG_ERR_INVALID_ARGUMENT, "row_ptr must be nondecreasing");
  if (lp->row_ptr[m] != nnz) return fail(OPDHG_ERR_INVALID_ARGUMENT, "row_ptr[m] must equal nnz");
  // The entries, by row ranges on up to 16 threads. A row whose columns
  // ascend has no duplicate; another row's columns are sorted in a copy.
  // Each range reports its first bad row; the first over all ranges wins,
  // so the message is the one a serial pass would give.
  static const char* const kWhy[] = {"", "column index out of range",
                                     "duplicate (row, column) entry",
                                     "A has a non-finite entry", "b must be finite",
                                     "row sense must be 0 or 1"};
  std::mutex mu;
  int64_t bad_row = m;
  int bad_why = 0;
  parallel_rows(lp->row_ptr, m, [&](int64_t r0, int64_t r1) {
    std::vector<int32_t> cols;
    for (int64_t i = r0; i < r1; ++i) {
      int why = 0;
      bool ascending = true;
      for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1] && !why; ++k) {
        const int32_t j = lp->col_idx[k];
        if (j < 0 || j >= n) why = 1;
        else if (!std::isfinite(lp->val[k])) why = 3;
        else if (k > lp->row_ptr[i] && j <= lp->col_idx[k - 1]) ascending = false;
      }
      if (!why && !ascending) {
        cols.assign(lp->col_idx + lp->row_ptr[i], lp->col_idx + lp->row_ptr[i + 1]);
        std::sort(cols.begin(), cols.end());
        if (std::adjacent_find(cols.begin(), cols.end()) != cols.end()) why = 2;
      }
      if (!why && !std::isfinite(lp->b[i])) why = 4;
      if (!why && lp->row_sense[i] != 0 && lp->row_sense[i] != 1) why = 5;
      if (why) {
        std::lock_guard<std::mutex> lock(mu);
        if (i < bad_row) {
          bad_row = i;
          bad_why = why;
        }
        return;
      }
    }
  });
  if (bad_why) return fail(OPDHG_ERR_INVALID_ARGUMENT, kWhy[bad_why]);
  for (int64_t j = 0; j < n; ++j) {
    if (!std::isfinite(lp->c[j])) return fail(OPDHG_ERR_INVALID_ARGUMENT, "c must be finite");
    const double l = lp->l[j], u = lp->u[j];
    if (std::isnan(l) || std::isnan(u))
      return fail(OPDHG_ERR_INVALID_ARGUMENT, "bounds must not be NaN");
    if (l == INFINITY || u == -INFINITY)
      return fail(OPDHG_ERR_INVALID_ARGUMENT, "l must be below +inf and u above -inf");
    if (l > u) return fail(OPDHG_ERR_INVALID_ARGUMENT, "l must not exceed u");
  }
  if (!std::isfinite(lp->obj_offset))
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "objective offset must be finite");
  return OPDHG_OK;
}

int validate_params(const opdhg_params* p) {
  if (!p) return fail(OPDHG_ERR_INVALID_ARGUMENT, "params is NULL");
  if (!(p->tol >= 0.0)) return fail(OPDHG_ERR_INVALID_ARGUMENT, "tol must be >= 0");
  if (p->max_iter < 0) return fail(OPDHG_ERR_INVALID_ARGUMENT, "max_iter must be >= 0");
  if (!(p->time_limit_s >= 0.0)) return fail(OPDHG_ERR_INVALID_ARGUMENT, "time limit must be >= 0");
  if (p->precision != OPDHG_FP64 && p->precision != OPDHG_FP32)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "unknown precision");
  if (p->schedule < 0 || p->schedule > 2) return fail(OPDHG_ERR_INVALID_ARGUMENT, "unknown schedule");
  if (!(p->lr >= 0.0) || !std::isfinite(p->lr))
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "lr must be finite and >= 0");
  if (p->phi < 1) return fail(OPDHG_ERR_INVALID_ARGUMENT, "phi must be >= 1");
  if (!(p->precond_floor >= 0.0) || !std::isfinite(p->precond_floor))
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "precond_floor must be finite and >= 0");
  if (p->ruiz_iters < 0) return fail(OPDHG_ERR_INVALID_ARGUMENT, "ruiz_iters must be >= 0");
  if (!std::isfinite(p->pc_beta) || p->pc_beta > 2.0)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "pc_beta must be <= 2 (negative skips the pass)");
  if (p->eval_every < 1) return fail(OPDHG_ERR_INVALID_ARGUMENT, "eval_every must be >= 1");
  if (p->max_step_retries < 0)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "max_step_retries must be >= 0");
  if (p->tile_nnz < 0) return fail(OPDHG_ERR_INVALID_ARGUMENT, "tile_nnz must be >= 0");
  if (p->lanes < 0 || p->lanes > 64 || (p->lanes & (p->lanes - 1)) != 0)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "lanes must be 0 or a power of two <= 64");
  if (p->workgroups < 0 || p->workgroups > kMaxGrid)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "workgroups must be in [0, 65536]");
  if (p->step_rule != OPDHG_STEP_ADAPTIVE && p->step_rule != OPDHG_STEP_CONSTANT)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "unknown step rule");
  if (p->restart_scheme != OPDHG_RESTART_ADAPTIVE && p->restart_scheme != OPDHG_RESTART_NONE)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "unknown restart scheme");
  if (p->l2_rescale != 0 && p->l2_rescale != 1)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "l2_rescale must be 0 or 1");
  if (p->power_iters < 1) return fail(OPDHG_ERR_INVALID_ARGUMENT, "power_iters must be >= 1");
  if (!(p->step_scale > 0.0) || !std::isfinite(p->step_scale))
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "step_scale must be finite and > 0");
  if (!(p->power_tol >= 0.0) || !std::isfinite(p->power_tol))
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "power_tol must be finite and >= 0");
  if (p->step_norm != OPDHG_STEP_NORM_PLAIN && p->step_norm != OPDHG_STEP_NORM_PRECOND)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "unknown step norm");
  if (p->windows < OPDHG_WINDOWS_AUTO || p->windows > OPDHG_WINDOWS_ALWAYS)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "windows must be OPDHG_WINDOWS_AUTO, _OFF or _ALWAYS");
  constexpr int kMaxParam = kWinCap / kWinParamBucket;
  if (p->window_buckets < 0 || p->window_buckets > kMaxParam)
    return fail(OPDHG_ERR_INVALID_ARGUMENT,
                "window_buckets must be in [0, " + std::to_string(kMaxParam) + "]");
  if (p->window_rows < 0 || p->window_rows > kWinRows)
    return fail(OPDHG_ERR_INVALID_ARGUMENT,
                "window_rows must be in [0, " + std::to_string(kWinRows) + "]");
  if (p->prep < OPDHG_PREP_AUTO || p->prep > OPDHG_PREP_DEVICE)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "prep must be OPDHG_PREP_AUTO, _HOST or _DEVICE");
  return OPDHG_OK;
}

// ---------------------------------------------------------------------------
// double-double accumulation on the host: sums rounded once at the end,
// so they agree with any other correctly rounded evaluation of the same sum
// except in near-tie cases
// ---------------------------------------------------------------------------

struct HostDD {
  double hi = 0.0, lo = 0.0;
  void add(double x) {
    const double s = hi + x;
    const double bb = s - hi;
    lo += (hi - (s - bb)) + (x - bb);
    hi = s;
  }
  void add_prod(double a, double b) {
    const double p = a * b;
    add(p);
    lo += std::fma(a, b, -p);
  }
  double value() const { return hi + lo; }
};

// Euclidean norm, the squares summed in double-double: per block of
// for_blocks (one block below 2^17 entries), then the blocks in order, so the
// result depends on n only, not on the host's threads.
static double dd_norm(const double* v, int64_t n) {
  const int nb = item_blocks(n);
  std::vector<HostDD> part(nb);
  for_blocks(n, nb, [&](int b, int64_t i0, int64_t i1) {
    HostDD a;
    for (int64_t i = i0; i < i1; ++i) a.add_prod(v[i], v[i]);
    part[b] = a;
  });
  HostDD acc = part[0];
  for (int b = 1; b < nb; ++b) {
    acc.add(part[b].hi);
    acc.lo += part[b].lo;
  }
  return std::sqrt(acc.value());
}

// ---------------------------------------------------------------------------
// rescaling: Ruiz infinity-norm passes then one Pock-Chambolle pass
// (Section 2 of the paper), square-root split between rows and columns
// ---------------------------------------------------------------------------

// ---- host parallelism for the preparation (results do not depend on it) ----

// Runs f(begin, end) over [0, rows) cut into pieces of about equal nonzero
// counts (ptr: rows + 1 offsets), one host thread per piece.
template <typename F>
static void parallel_rows(const int64_t* ptr, int64_t rows, F&& f) {
  const int64_t total = rows ? ptr[rows] : 0;
  const int nth = (int)std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)std::min(host_threads(), 16), rows, total / 65536 + 1}));
  if (nth == 1) {
    f((int64_t)0, rows);
    return;
  }
  std::vector<int64_t> cut(nth + 1, rows);
  cut[0] = 0;
  for (int t = 1; t < nth; ++t) {
    const int64_t target = total * t / nth;
    cut[t] = std::lower_bound(ptr, ptr + rows + 1, target) - ptr;
    cut[t] = std::max(cut[t], cut[t - 1]);
  }
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) pool.emplace_back([&, t] { f(cut[t], cut[t + 1]); });
  f(cut[0], cut[1]);
  for (auto& th : pool) th.join();
}

// Runs the tasks on their own threads (the calling thread takes the first).
static void run_tasks(std::vector<std::function<void()>> tasks) {
  std::vector<std::thread> pool;
  for (size_t t = 1; t < tasks.size(); ++t) pool.emplace_back(tasks[t]);
  if (!tasks.empty()) tasks[0]();
  for (auto& th : pool) th.join();
}

// Calls f(a, b) on consecutive pieces [a, b) of [0, n) on up to 16 host
// threads, in pieces of at least `min_piece`.
template <typename F>
static void parallel_pieces(size_t n, size_t min_piece, F&& f) {
  const size_t nth = std::max<size_t>(
      1, std::min<size_t>({(size_t)std::min(host_threads(), 16), n / std::max<size_t>(min_piece, 1)}));
  if (nth == 1) {
    f((size_t)0, n);
    return;
  }
  std::vector<std::thread> pool;
  for (size_t t = 1; t < nth; ++t) pool.emplace_back([&, t] { f(n * t / nth, n * (t + 1) / nth); });
  f((size_t)0, n / nth);
  for (auto& th : pool) th.join();
}

// Column-major index of a CSR matrix: for column j, entries
// cstart[j] .. cstart[j+1]-1 of cpos hold the CSR positions of its
// nonzeros in ascending row order, and crow their rows.
// An array left uninitialised on allocation, so that the threads that fill
// it are the first to touch its pages.
template <typename T>
struct RawArray {
  std::unique_ptr<T[]> p;
  void reset(int64_t count) { p.reset(new T[std::max<int64_t>(count, 1)]); }
  T& operator[](int64_t i) { return p[i]; }
  const T& operator[](int64_t i) const { return p[i]; }
};

struct ColIndex {
  std::vector<int64_t> cstart;
  RawArray<int64_t> cpos;
  RawArray<int32_t> crow;
  RawArray<double> cabs;  // |value| in the same order, read sequentially by column passes
};

static void build_col_index(const opdhg_lp* lp, ColIndex& C, bool with_abs = true) {
  const int64_t m = lp->m, n = lp->n, nnz = lp->nnz;
  C.cstart.assign(n + 1, 0);
  C.cpos.reset(nnz);
  C.crow.reset(nnz);
  if (with_abs) C.cabs.reset(nnz);
  // a counting sort by column in parallel: thread t takes a range of rows
  // (in row order), counts its columns, and scatters its entries to the
  // positions after those of threads t' < t, so rows stay ascending within
  // every column exactly as a serial pass would leave them
  int nth = (int)std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)std::min(host_threads(), 16), m, nnz / 262144 + 1}));
  nth = (int)std::max<int64_t>(1, std::min<int64_t>(nth, (int64_t)(1ll << 29) / (4 * (n + 1))));
  std::vector<int64_t> cut(nth + 1, m);
  cut[0] = 0;
  for (int t = 1; t < nth; ++t)
    cut[t] = std::max(cut[t - 1],
                      (int64_t)(std::lower_bound(lp->row_ptr, lp->row_ptr + m + 1, nnz * t / nth) -
                                lp->row_ptr));
  // each thread zeroes (and first touches) its own counts
  std::vector<std::vector<int32_t>> cnt(nth);
  auto run = [&](auto&& f) {
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t) pool.emplace_back([&, t] { f(t); });
    f(0);
    for (auto& th : pool) th.join();
  };
  run([&](int t) {
    cnt[t].assign(n, 0);
    for (int64_t k = lp->row_ptr[cut[t]]; k < lp->row_ptr[cut[t + 1]]; ++k) cnt[t][lp->col_idx[k]]++;
  });
  // column starts, then each thread's first position in every column
  for (int64_t j = 0; j < n; ++j) {
    int64_t c = 0;
    for (int t = 0; t < nth; ++t) c += cnt[t][j];
    C.cstart[j + 1] = C.cstart[j] + c;
  }
  run([&](int t) {
    // this thread's columns in [n * t / nth, n * (t + 1) / nth): turn counts into positions
    for (int64_t j = n * t / nth; j < n * (t + 1) / nth; ++j) {
      int64_t pos = C.cstart[j];
      for (int u = 0; u < nth; ++u) {
        const int32_t c = cnt[u][j];
        cnt[u][j] = (int32_t)(pos - C.cstart[j]);  // offset of thread u inside column j
        pos += c;
      }
    }
  });
  run([&](int t) {
    std::vector<int32_t>& off = cnt[t];
    for (int64_t i = cut[t]; i < cut[t + 1]; ++i)
      for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k) {
        const int32_t j = lp->col_idx[k];
        const int64_t q = C.cstart[j] + off[j]++;
        C.cpos[q] = k;
        C.crow[q] = (int32_t)i;
        if (with_abs) C.cabs[q] = std::fabs(lp->val[k]);
      }
  });
}

// Entries per column (= row lengths of A^T), counted by row ranges in
// parallel and added per column.
static void column_counts(const opdhg_lp* lp, std::vector<int64_t>& len) {
  const int64_t m = lp->m, n = lp->n;
  // one shared count per column, incremented atomically by blocks of rows
  // (integer counts: the order of the increments does not matter)
  std::vector<int32_t> cnt(n, 0);
  int32_t* c = cnt.data();
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(64, lp->nnz / 131072));
  for_blocks(m, nb, [&](int, int64_t i0, int64_t i1) {
    for (int64_t k = lp->row_ptr[i0]; k < lp->row_ptr[i1]; ++k)
      __atomic_fetch_add(c + lp->col_idx[k], 1, __ATOMIC_RELAXED);
  });
  len.resize(n);
  for_blocks(n, item_blocks(n), [&](int, int64_t j0, int64_t j1) {
    for (int64_t j = j0; j < j1; ++j) len[j] = cnt[j];
  });
}

// Ruiz passes then one Pock-Chambolle pass (Section 2): per pass, each row
// and column statistic of |A~| (the infinity norm for Ruiz; for
// Pock-Chambolle the sum of |a|^beta over a row and of |a|^(2 - beta) over
// a column; the L2 norm for the optional L2 pass) divides
// its diagonal by its square root, a zero statistic read as 1. Maxima do not
// depend on order and the sums are double-double, so the threads change no
// bit of the result.
static void rescale_with(const opdhg_lp* lp, const ColIndex& C, int ruiz_iters, bool l2,
                         double beta, std::vector<double>& sval, std::vector<double>& dr,
                         std::vector<double>& dc) {
  const int64_t m = lp->m, n = lp->n;
  dr.assign(m, 1.0);
  dc.assign(n, 1.0);
  std::vector<double> rs(m), cs(n);
  auto apply = [&]() {
    for (int64_t i = 0; i < m; ++i) dr[i] = dr[i] / std::sqrt(rs[i] == 0.0 ? 1.0 : rs[i]);
    for (int64_t j = 0; j < n; ++j) dc[j] = dc[j] / std::sqrt(cs[j] == 0.0 ? 1.0 : cs[j]);
  };
  for (int it = 0; it < ruiz_iters; ++it) {
    parallel_rows(lp->row_ptr, m, [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) {
        double rmax = 0.0;
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k)
          rmax = std::max(rmax, std::fabs(lp->val[k]) * dr[i] * dc[lp->col_idx[k]]);
        rs[i] = rmax;
      }
    });
    parallel_rows(C.cstart.data(), n, [&](int64_t j0, int64_t j1) {
      for (int64_t j = j0; j < j1; ++j) {
        double cmax = 0.0;
        for (int64_t q = C.cstart[j]; q < C.cstart[j + 1]; ++q)
          cmax = std::max(cmax, C.cabs[q] * dr[C.crow[q]] * dc[j]);
        cs[j] = cmax;
      }
    });
    apply();
  }
  if (l2) {  // divide by the square roots of the rows' and columns' L2 norms
    parallel_rows(lp->row_ptr, m, [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) {
        HostDD racc;
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k) {
          const double a = std::fabs(lp->val[k]) * dr[i] * dc[lp->col_idx[k]];
          racc.add(a * a);
        }
        rs[i] = std::sqrt(racc.value());
      }
    });
    parallel_rows(C.cstart.data(), n, [&](int64_t j0, int64_t j1) {
      for (int64_t j = j0; j < j1; ++j) {
        HostDD cacc;
        for (int64_t q = C.cstart[j]; q < C.cstart[j + 1]; ++q) {
          const double a = C.cabs[q] * dr[C.crow[q]] * dc[j];
          cacc.add(a * a);
        }
        cs[j] = std::sqrt(cacc.value());
      }
    });
    apply();
  }
  if (beta >= 0.0) {
    parallel_rows(lp->row_ptr, m, [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) {
        HostDD racc;
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k) {
          const double a = std::fabs(lp->val[k]) * dr[i] * dc[lp->col_idx[k]];
          racc.add(beta == 1.0 ? a : std::pow(a, beta));
        }
        rs[i] = racc.value();
      }
    });
    parallel_rows(C.cstart.data(), n, [&](int64_t j0, int64_t j1) {
      for (int64_t j = j0; j < j1; ++j) {
        HostDD cacc;
        for (int64_t q = C.cstart[j]; q < C.cstart[j + 1]; ++q) {
          const double a = C.cabs[q] * dr[C.crow[q]] * dc[j];
          cacc.add(beta == 1.0 ? a : std::pow(a, 2.0 - beta));
        }
        cs[j] = cacc.value();
      }
    });
    apply();
  }
  sval.resize(lp->nnz);
  parallel_rows(lp->row_ptr, m, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i)
      for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k)
        sval[k] = lp->val[k] * dr[i] * dc[lp->col_idx[k]];
  });
}

void rescale_host(const opdhg_lp* lp, const opdhg_params* p, std::vector<double>& sval,
                  std::vector<double>& dr, std::vector<double>& dc) {
  ColIndex C;
  build_col_index(lp, C);
  rescale_with(lp, C, p->ruiz_iters, p->l2_rescale != 0, p->pc_beta, sval, dr, dc);
}

// Power iteration on A~^T A~ for |A~|_2 (the constant step of vanilla PDHG,
// Section 2): v = 1 / |1|, then per round w = A~^T (A~ v), lam = |w|,
// v = w / lam; stop after `iters` rounds, when lam moves by at most
// tol * lam, or when w = 0 (returns 0). For a unit v, lam <= |A~|_2^2.
static double spectral_norm_with(const opdhg_lp* lp, const ColIndex& C,
                                 const std::vector<double>& sval, int iters, double tol) {
  const int64_t m = lp->m, n = lp->n;
  std::vector<double> v(n, 1.0), av(m), w(n);
  const double n1 = dd_norm(v.data(), n);
  for (int64_t j = 0; j < n; ++j) v[j] = v[j] / n1;
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    parallel_rows(lp->row_ptr, m, [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) {
        HostDD acc;
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k)
          acc.add_prod(sval[k], v[lp->col_idx[k]]);
        av[i] = acc.value();
      }
    });
    parallel_rows(C.cstart.data(), n, [&](int64_t j0, int64_t j1) {
      for (int64_t j = j0; j < j1; ++j) {
        HostDD acc;
        for (int64_t q = C.cstart[j]; q < C.cstart[j + 1]; ++q)
          acc.add_prod(sval[C.cpos[q]], av[C.crow[q]]);
        w[j] = acc.value();
      }
    });
    const double lam_new = dd_norm(w.data(), n);
    if (lam_new == 0.0) return 0.0;
    for (int64_t j = 0; j < n; ++j) v[j] = w[j] / lam_new;
    const bool done = std::fabs(lam_new - lam) <= tol * lam_new;
    lam = lam_new;
    if (done) break;
  }
  return std::sqrt(lam);
}

// ---------------------------------------------------------------------------
// row classes and tiling
//
// On the device the rows of each side are relabelled so that rows of like
// length sit together: long rows (more than 256 nonzeros) first, then
// medium (33 to 256), then short, keeping the original order inside each
// class. Variables follow the order of the A^T rows and constraints the
// order of the A rows. The relabelling is a permutation of the LP, and
// every FP64 sum is rounded once from its exact value, so results do not
// depend on it; it only keeps one long row from holding up a workgroup of
// short ones.
// ---------------------------------------------------------------------------

static int row_class(int64_t len) { return len > 256 ? 0 : (len > 32 ? 1 : 2); }

// perm[new] = old, stable within each class; class_end[c] = end of class c.
// Blocks of rows count their classes, then each block writes its rows of
// each class at that class's offset for the block (a stable partition).
static void class_order(const std::vector<int64_t>& len, std::vector<int32_t>& perm,
                        int64_t class_end[3]) {
  const int64_t rows = (int64_t)len.size();
  const int nb = item_blocks(rows);
  std::vector<std::array<int64_t, 3>> cnt(nb, {0, 0, 0});
  for_blocks(rows, nb, [&](int b, int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) cnt[b][row_class(len[i])]++;
  });
  int64_t tot[3] = {0, 0, 0};
  for (int b = 0; b < nb; ++b)
    for (int c = 0; c < 3; ++c) tot[c] += cnt[b][c];
  class_end[0] = tot[0];
  class_end[1] = tot[0] + tot[1];
  class_end[2] = rows;
  std::vector<std::array<int64_t, 3>> at(nb);
  int64_t run[3] = {0, tot[0], tot[0] + tot[1]};
  for (int b = 0; b < nb; ++b)
    for (int c = 0; c < 3; ++c) {
      at[b][c] = run[c];
      run[c] += cnt[b][c];
    }
  perm.resize(rows);
  for_blocks(rows, nb, [&](int b, int64_t i0, int64_t i1) {
    std::array<int64_t, 3> w = at[b];
    for (int64_t i = i0; i < i1; ++i) perm[w[row_class(len[i])]++] = (int32_t)i;
  });
}

// rp[0] = 0, rp[i + 1] = rp[i] + len[perm[i]] (row pointers in device
// order), as a two-pass blocked scan.
static void device_row_ptr(const std::vector<int64_t>& len, const std::vector<int32_t>& perm,
                           std::vector<int32_t>& rp) {
  const int64_t rows = (int64_t)perm.size();
  rp.assign(rows + 1, 0);
  const int nb = item_blocks(rows);
  std::vector<int64_t> sum(nb + 1, 0);
  for_blocks(rows, nb, [&](int b, int64_t i0, int64_t i1) {
    int64_t t = 0;
    for (int64_t i = i0; i < i1; ++i) t += len[perm[i]];
    sum[b + 1] = t;
  });
  for (int b = 0; b < nb; ++b) sum[b + 1] += sum[b];
  for_blocks(rows, nb, [&](int b, int64_t i0, int64_t i1) {
    int64_t t = sum[b];
    for (int64_t i = i0; i < i1; ++i) {
      t += len[perm[i]];
      rp[i + 1] = (int32_t)t;
    }
  });
}

// Lanes per row for a stream tile whose longest row has max_len nonzeros:
// enough that each lane sums at most 16 products, at most 64.
static int lanes_for(int64_t max_len) {
  int L = 1;
  while (L < 64 && max_len > 16 * L) L <<= 1;
  return L;
}

// Rows of one CSR side into tiles. A row with more than `cap` nonzeros is a
// tile of its own (lanes 0); other rows are packed greedily into stream
// tiles of at most `cap` nonzeros and kBlock / lanes rows.
std::vector<Tile> build_tiles(const int32_t* rp, int64_t rows, int64_t cap, int lanes_fixed) {
  std::vector<Tile> tiles;
  int64_t i = 0;
  while (i < rows) {
    const int64_t len = rp[i + 1] - rp[i];
    if (len > cap) {
      tiles.push_back(Tile{(int32_t)i, (int32_t)(i + 1), rp[i], rp[i + 1], 0, 0});
      ++i;
      continue;
    }
    const int64_t start = i;
    int64_t nz = 0, max_len = 0;
    int L = 1;
    while (i < rows) {
      const int64_t l = rp[i + 1] - rp[i];
      if (l > cap) break;
      const int64_t ml = std::max(max_len, l);
      const int Ln = lanes_fixed > 0 ? lanes_fixed : lanes_for(ml);
      if (i > start && (nz + l > cap || i - start + 1 > kBlock / Ln)) break;
      nz += l;
      max_len = ml;
      L = Ln;
      ++i;
    }
    tiles.push_back(Tile{(int32_t)start, (int32_t)i, rp[start], rp[i], L, 0});
  }
  if (tiles.empty()) tiles.push_back(Tile{0, 0, 0, 0, 1, 0});
  return tiles;
}

// ---------------------------------------------------------------------------
// windowed chunks (FP32 step kernels)
//
// Rows [lo, hi) of one side are cut into chunks of `chunk_rows` rows. A
// chunk is windowed when the vector entries its nonzeros gather lie in a few
// runs of kWinBucket-entry buckets: the runs are packed into at most kWinMaxPass
// passes of `per_pass` buckets, and the staged entries (4 bytes each) must
// cost at most half the chunk's matrix bytes (8 per nonzero), so the window
// copies stay small against the stream of the matrix. Other chunks stay
// in tiles.
// ---------------------------------------------------------------------------

constexpr int64_t kWinMinNnz = 8192;  // smaller chunks are not worth a workgroup of kWinBlock

// Chunk rows of a windowed side: the parameter, or the side's windowable
// rows spread evenly over whole rounds of kWinRound chunks (one chunk per
// compute unit at a time, so no round is left half empty), at least 1024.
constexpr int64_t kWinRound = 256;
constexpr int64_t kWinMinChunks = 128;  // fewer chunks than this leave most CUs idle

static int64_t window_chunk_rows(const opdhg_params* p, int64_t rows) {
  if (p->window_rows > 0) {
    // as few chunks as the cap allows, of equal size: a short last chunk
    // would stage the whole window for few rows and fall back to tiles
    const int64_t nch = std::max<int64_t>(1, (rows + p->window_rows - 1) / p->window_rows);
    return std::max<int64_t>(1, (rows + nch - 1) / nch);
  }
  const int64_t rounds = std::max<int64_t>(1, (rows + kWinRound * kWinRows - 1) / (kWinRound * kWinRows));
  const int64_t per = (rows + rounds * kWinRound - 1) / (rounds * kWinRound);
  return std::min<int64_t>(kWinRows, std::max<int64_t>(1024, per));
}

// Buckets per pass of a chunk of several passes, and the most buckets a
// chunk of one pass stages (the parameter sets both, in units of
// kWinParamBucket entries).
static int window_per_pass(const opdhg_params* p) {
  return p->window_buckets > 0 ? p->window_buckets * (kWinParamBucket / kWinBucket) : kWinBuckets;
}
static int window_one_pass(const opdhg_params* p) {
  return p->window_buckets > 0 ? window_per_pass(p) : kWinOneBuckets;
}

static void plan_windows(const std::vector<int32_t>& rp, const HostArray<int32_t>& ci,
                         int64_t ncols, int64_t lo, int64_t hi, int64_t long_end,
                         int64_t chunk_rows, int per_pass, int one_cap, WinPlan& W) {
  if (hi <= lo || ncols <= 0) return;
  const int64_t nb = (ncols + kWinBucket - 1) / kWinBucket;
  const int64_t max_buckets = (int64_t)per_pass * kWinMaxPass;
  std::vector<int32_t> stamp(nb, -1), rstamp(nb, -1);
  std::vector<int64_t> touched;
  // a chunk's staged buckets: (bucket, pass, offset in the pass's window)
  struct Slot {
    int64_t bucket;
    int32_t pass, off;
  };
  std::vector<std::vector<Slot>> slots;
  int32_t id = 0;
  for (int64_t a = lo, b = lo; a < hi; a = b, ++id) {
    // grow the chunk row by row. It ends at chunk_rows rows, before a row
    // that would need more than kWinMaxPass passes, or (past a quarter of
    // chunk_rows) before a row most of whose buckets are new: a new block
    // of columns begins there, and a chunk that crossed into it would stage
    // both blocks.
    touched.clear();
    for (b = a; b < hi && b - a < chunk_rows; ++b) {
      int64_t row_b = 0, row_new = 0;
      for (int64_t k = rp[b]; k < rp[b + 1]; ++k) {
        const int64_t bk = ci[k] / kWinBucket;
        if (rstamp[bk] == (int32_t)b) continue;
        rstamp[bk] = (int32_t)b;
        ++row_b;
        if (stamp[bk] != id) ++row_new;
      }
      if (b > a && ((int64_t)touched.size() + row_new > max_buckets ||
                    (4 * (b - a) >= chunk_rows && 2 * row_new > row_b)))
        break;
      for (int64_t k = rp[b]; k < rp[b + 1]; ++k) {
        const int64_t bk = ci[k] / kWinBucket;
        if (stamp[bk] != id) {
          stamp[bk] = id;
          touched.push_back(bk);
        }
      }
    }
    const int64_t nz = (int64_t)rp[b] - rp[a];
    if (nz < kWinMinNnz) continue;
    const int64_t nbk = (int64_t)touched.size();
    // a chunk whose buckets fit one_cap takes one pass over them all
    const int64_t step = nbk <= one_cap ? std::max<int64_t>(nbk, 1) : per_pass;
    if ((nbk + step - 1) / step > kWinMaxPass) continue;
    if (nbk * kWinBucket * 4 > nz * 4) continue;  // staged bytes <= half the matrix bytes
    std::sort(touched.begin(), touched.end());
    // buckets to passes in order; runs of consecutive buckets become one range
    const int32_t pass0 = (int32_t)W.passes.size();
    int npass = 0;
    std::vector<Slot> sl;
    for (int64_t q = 0; q < nbk; q += step) {
      WinPass ps{0, 0, (int32_t)W.ranges.size(), 0};
      int32_t off = 0;
      for (int64_t u = q; u < std::min(nbk, q + step); ++u) {
        const int64_t bk = touched[u];
        const int32_t src = (int32_t)(bk * kWinBucket);
        const int32_t len = (int32_t)std::min<int64_t>(kWinBucket, ncols - src);
        if (ps.nrange > 0 && u > q && touched[u - 1] == bk - 1) {
          W.ranges.back().len += len;  // extends the previous range
        } else {
          W.ranges.push_back(WinRange{src, len});
          ps.nrange++;
        }
        sl.push_back(Slot{bk, npass, off});
        off += len;
      }
      W.passes.push_back(ps);
      ++npass;
    }
    W.r0.push_back((int32_t)a);
    W.r1.push_back((int32_t)b);
    W.pass0.push_back(pass0);
    W.npass.push_back(npass);
    slots.push_back(std::move(sl));
  }
  const int64_t nch = (int64_t)W.chunks();
  W.nseg.assign(nch, 0);
  W.seg0.assign(nch, 0);
  if (nch == 0) return;

  // Row segments. A long row (rows [0, long_end)), or a row of [lo, hi)
  // that no chunk took, whose every entry falls in some chunk's window is
  // split by chunk: the entries of a bucket go to one of the chunks that
  // stage it (chosen by the row, so that the long rows spread over those
  // chunks), and each (row, chunk) pair becomes an extra row of that chunk,
  // after its own rows. Its pass sums go to a partial of its own; a
  // finishing kernel adds a row's partials in chunk order. The row then
  // leaves the tiles (a side whose rows all leave them needs no tile launch
  // beside its windowed one).
  std::vector<std::vector<int32_t>> cover(nb);  // chunks staging each bucket
  for (int64_t c = 0; c < nch; ++c)
    for (const Slot& x : slots[c]) cover[x.bucket].push_back((int32_t)c);
  auto chunk_of = [&](int64_t r, int64_t bk) -> int32_t {
    const std::vector<int32_t>& cv = cover[bk];
    return cv.empty() ? -1 : cv[(size_t)(r % (int64_t)cv.size())];
  };
  std::vector<std::vector<int64_t>> seg_rows(nch);  // per chunk: its segment rows, in order
  std::vector<int32_t> used;
  std::vector<int32_t> cstamp(nch, -1);
  // candidate rows in ascending order: the long rows, then the rows of
  // [lo, hi) outside every chunk (the chunks are in row order)
  std::vector<int64_t> cand;
  for (int64_t r = 0; r < std::min(long_end, hi); ++r) cand.push_back(r);
  {
    int64_t r = std::max(lo, std::min(long_end, hi));
    for (int64_t c = 0; c <= nch; ++c) {
      const int64_t stop = c < nch ? (int64_t)W.r0[c] : hi;
      for (; r < stop; ++r) cand.push_back(r);
      if (c < nch) r = std::max<int64_t>(r, W.r1[c]);
    }
  }
  for (int64_t r : cand) {
    if (rp[r + 1] == rp[r]) continue;
    used.clear();
    bool ok = true;
    for (int64_t k = rp[r]; k < rp[r + 1] && ok; ++k) {
      const int32_t c = chunk_of(r, ci[k] / kWinBucket);
      if (c < 0) ok = false;
      else if (cstamp[c] != (int32_t)r) {
        cstamp[c] = (int32_t)r;
        used.push_back(c);
      }
    }
    if (!ok) continue;
    for (int32_t c : used)
      if ((int64_t)W.r1[c] - W.r0[c] + W.nseg[c] + 1 > kWinRows) ok = false;
    if (!ok) continue;
    std::sort(used.begin(), used.end());
    W.srow.push_back((int32_t)r);
    for (int32_t c : used) {
      seg_rows[c].push_back(r);
      W.nseg[c]++;
    }
  }
  // global segment ids: chunk by chunk
  int32_t sid = 0;
  for (int64_t c = 0; c < nch; ++c) {
    W.seg0[c] = sid;
    sid += W.nseg[c];
  }
  W.nsegs = sid;
  // each segmented row's partials, in chunk order
  {
    std::vector<int32_t> next(nch, 0);
    std::vector<std::vector<std::pair<int32_t, int32_t>>> per_row(W.srow.size());
    std::vector<int32_t> row_index((size_t)hi, -1);
    for (size_t q = 0; q < W.srow.size(); ++q) row_index[W.srow[q]] = (int32_t)q;
    for (int64_t c = 0; c < nch; ++c)
      for (int64_t r : seg_rows[c]) per_row[row_index[r]].push_back({(int32_t)c, W.seg0[c] + next[c]++});
    W.sptr.assign(1, 0);
    for (auto& v : per_row) {
      std::sort(v.begin(), v.end());
      for (auto& pr : v) W.sids.push_back(pr.second);
      W.sptr.push_back((int32_t)W.sids.size());
    }
  }

  // each chunk's segment entries (CSR position, chunk-local row), in
  // segment order: one pass over the segmented rows (ascending, the order in
  // which the chunks took them)
  std::vector<std::vector<std::pair<int64_t, int32_t>>> seg_entries(nch);
  {
    std::vector<int32_t> taken(nch, 0), local(nch, -1), at(nch, -1);
    for (int32_t r : W.srow)
      for (int64_t k = rp[r]; k < rp[r + 1]; ++k) {
        const int32_t c = chunk_of(r, ci[k] / kWinBucket);
        if (at[c] != r) {
          at[c] = r;
          local[c] = (W.r1[c] - W.r0[c]) + taken[c]++;
        }
        seg_entries[c].push_back({k, local[c]});
      }
  }
  // Each pass of each chunk: the rows with entries in it (own rows, then
  // segments), longest first (equal counts in row order), cut into slices of
  // kWinSlice rows. A slice's entries go k-major, each row's in CSR order,
  // padded to the slice's longest row with zero entries of window column 0.
  // The chunks are independent, so they are spread over up to 16 host
  // threads: each chunk first counts its slices and entries per pass, the
  // passes' ranges follow in chunk order, and then every chunk writes its
  // own ranges.
  auto for_chunks = [&](auto&& f) {
    std::atomic<int64_t> next{0};
    auto work = [&] {
      std::vector<int32_t> bpass(nb, -1), boff(nb, 0);
      for (int64_t c = next++; c < nch; c = next++) {
        for (const Slot& x : slots[c]) {
          bpass[x.bucket] = x.pass;
          boff[x.bucket] = x.off;
        }
        f(c, bpass, boff);
        for (const Slot& x : slots[c]) bpass[x.bucket] = -1;
      }
    };
    const int nth = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(host_threads(), 16), nch));
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
  };
  // a chunk's rows per pass: entry counts (pass-major) and the order
  struct PassRows {
    int32_t nrows = 0;
    std::vector<int32_t> cnt, order;
    int32_t nact[kWinMaxPass] = {};
  };
  auto pass_rows = [&](int64_t c, const std::vector<int32_t>& bpass, PassRows& R) {
    const int64_t a = W.r0[c], b = W.r1[c];
    const int np = W.npass[c];
    const int32_t nr = (int32_t)(b - a + W.nseg[c]);
    R.nrows = nr;
    R.cnt.assign((size_t)np * nr, 0);
    for (int64_t r = a; r < b; ++r)
      for (int64_t k = rp[r]; k < rp[r + 1]; ++k)
        ++R.cnt[(size_t)bpass[ci[k] / kWinBucket] * nr + (r - a)];
    for (const auto& e : seg_entries[c])
      ++R.cnt[(size_t)bpass[ci[e.first] / kWinBucket] * nr + e.second];
    R.order.resize((size_t)np * nr);
    std::vector<int32_t> at;
    for (int q = 0; q < np; ++q) {
      // counting sort by count, descending; rows ascending within a count
      const int32_t* cq = R.cnt.data() + (size_t)q * nr;
      int32_t* oq = R.order.data() + (size_t)q * nr;
      int32_t mx = 0;
      for (int32_t r = 0; r < nr; ++r) mx = std::max(mx, cq[r]);
      at.assign((size_t)mx + 1, 0);
      for (int32_t r = 0; r < nr; ++r)
        if (cq[r] > 0) ++at[mx - cq[r]];
      int32_t s = 0;
      for (int32_t v = 0; v <= mx; ++v) {
        const int32_t k = at[v];
        at[v] = s;
        s += k;
      }
      for (int32_t r = 0; r < nr; ++r)
        if (cq[r] > 0) oq[at[mx - cq[r]]++] = r;
      R.nact[q] = s;
    }
  };
  std::vector<int64_t> pass_slices(W.passes.size(), 0), pass_entries(W.passes.size(), 0);
  for_chunks([&](int64_t c, const std::vector<int32_t>& bpass, const std::vector<int32_t>&) {
    PassRows R;
    pass_rows(c, bpass, R);
    for (int q = 0; q < W.npass[c]; ++q) {
      const int32_t* cq = R.cnt.data() + (size_t)q * R.nrows;
      const int32_t* oq = R.order.data() + (size_t)q * R.nrows;
      int64_t ns = 0, ne = 0;
      for (int32_t i = 0; i < R.nact[q]; i += kWinSlice, ++ns) ne += (int64_t)kWinSlice * cq[oq[i]];
      pass_slices[W.pass0[c] + q] = ns;
      pass_entries[W.pass0[c] + q] = ne;
    }
  });
  std::vector<int64_t> pass_e0(W.passes.size(), 0);
  int64_t nslice = 0, total = 0;
  for (size_t q = 0; q < W.passes.size(); ++q) {
    W.passes[q].s0 = (int32_t)nslice;
    nslice += pass_slices[q];
    W.passes[q].s1 = (int32_t)nslice;
    pass_e0[q] = total;
    total += pass_entries[q];
  }
  if (total > (int64_t)INT32_MAX || nslice * kWinSlice > (int64_t)INT32_MAX) {
    W = WinPlan();  // beyond 32-bit entry offsets: no windows
    return;
  }
  W.slices.resize(nslice);
  W.lane.resize(nslice * kWinSlice);
  W.col.resize(total);
  W.src.resize(total);
  for_chunks([&](int64_t c, const std::vector<int32_t>& bpass, const std::vector<int32_t>& boff) {
    PassRows R;
    pass_rows(c, bpass, R);
    const int np = W.npass[c];
    const int32_t nr = R.nrows;
    // each row's slice and lane in every pass, and its next entry there
    std::vector<int32_t> place((size_t)np * nr, -1), fill((size_t)np * nr, 0);
    for (int q = 0; q < np; ++q) {
      const int64_t gq = W.pass0[c] + q;
      const int32_t* cq = R.cnt.data() + (size_t)q * nr;
      const int32_t* oq = R.order.data() + (size_t)q * nr;
      int64_t e = pass_e0[gq];
      for (int32_t i = 0, j = 0; i < R.nact[q]; i += kWinSlice, ++j) {
        const int32_t S = W.passes[gq].s0 + j;
        const int32_t len = cq[oq[i]];
        W.slices[S] = WinSlice{(int32_t)e, len};
        for (int l = 0; l < kWinSlice; ++l) {
          const bool on = i + l < R.nact[q];
          W.lane[(size_t)S * kWinSlice + l] = on ? (uint16_t)oq[i + l] : kWinNoRow;
          if (on) place[(size_t)q * nr + oq[i + l]] = S * kWinSlice + l;
        }
        for (int64_t p = e; p < e + (int64_t)kWinSlice * len; ++p) {  // padding first
          W.col[p] = 0;
          W.src[p] = -1;
        }
        e += (int64_t)kWinSlice * len;
      }
    }
    auto emit = [&](int64_t k, int32_t local) {
      const int64_t bk = ci[k] / kWinBucket;
      const int q = bpass[bk];
      const int32_t pl = place[(size_t)q * nr + local];
      const WinSlice& sl = W.slices[pl / kWinSlice];
      const int64_t p = sl.e0 + (int64_t)fill[(size_t)q * nr + local]++ * kWinSlice + pl % kWinSlice;
      W.col[p] = (uint16_t)(boff[bk] + (ci[k] - bk * kWinBucket));
      W.src[p] = k;
    };
    const int64_t a = W.r0[c], b = W.r1[c];
    for (int64_t r = a; r < b; ++r)
      for (int64_t k = rp[r]; k < rp[r + 1]; ++k) emit(k, (int32_t)(r - a));
    for (const auto& e : seg_entries[c]) emit(e.first, e.second);
  });
}

// Every index a windowed kernel derives from the plan stays in its
// buffers: LDS columns inside their pass's staged length, lane rows below
// the chunk's rows, slice entries inside the entry arrays, staged ranges
// inside the vector.
static bool plan_ok(const WinPlan& W, int64_t rows, int64_t ncols) {
  for (size_t c = 0; c < W.chunks(); ++c) {
    const int64_t nrow = (int64_t)W.r1[c] - W.r0[c] + W.nseg[c];
    if (W.r0[c] < 0 || W.r1[c] > rows || W.r1[c] <= W.r0[c] || nrow > kWinRows) return false;
    // one pass: the window may take the row sums' LDS too
    const int64_t cap = W.npass[c] == 1 ? kWinOneCap : kWinCap;
    if (W.seg0[c] < 0 || W.seg0[c] + W.nseg[c] > W.nsegs) return false;
    if (W.npass[c] < 1 || W.npass[c] > kWinMaxPass) return false;
    for (int32_t q = W.pass0[c]; q < W.pass0[c] + W.npass[c]; ++q) {
      if (q < 0 || (size_t)q >= W.passes.size()) return false;
      const WinPass& ps = W.passes[q];
      if (ps.s0 < 0 || ps.s1 < ps.s0 || (size_t)ps.s1 > W.slices.size() ||
          ps.s1 - ps.s0 > kWinRows / kWinSlice)
        return false;
      if (ps.range0 < 0 || ps.nrange < 1 || (size_t)(ps.range0 + ps.nrange) > W.ranges.size())
        return false;
      int64_t len = 0;
      for (int32_t g = ps.range0; g < ps.range0 + ps.nrange; ++g) {
        const WinRange& rg = W.ranges[g];
        if (rg.src < 0 || rg.len <= 0 || (int64_t)rg.src + rg.len > ncols) return false;
        len += rg.len;
      }
      if (len > cap) return false;
      for (int32_t sj = ps.s0; sj < ps.s1; ++sj) {
        const WinSlice& sl = W.slices[sj];
        if (sl.e0 < 0 || sl.e0 % kWinSlice || sl.len < 1 ||
            (int64_t)sl.e0 + (int64_t)kWinSlice * sl.len > (int64_t)W.col.size())
          return false;
        for (int l = 0; l < kWinSlice; ++l) {
          const uint16_t r = W.lane[(size_t)sj * kWinSlice + l];
          if (r != kWinNoRow && r >= nrow) return false;
        }
        for (int64_t e = sl.e0; e < sl.e0 + (int64_t)kWinSlice * sl.len; ++e)
          if (W.col[e] >= len) return false;
      }
    }
  }
  if (!W.srow.empty() &&
      (W.sptr.size() != W.srow.size() + 1 || (size_t)W.sptr.back() != W.sids.size()))
    return false;
  for (int32_t r : W.srow)
    if (r < 0 || r >= rows) return false;
  for (int32_t q : W.sids)
    if (q < 0 || q >= W.nsegs) return false;
  return W.col.size() == W.src.size() && W.lane.size() == W.slices.size() * kWinSlice;
}

// Whether automatic windows are worth planning: enough nonzeros for
// kWinMinChunks chunks, and at least half of 8 chunks sampled evenly over
// the windowable rows of A (device order, columns relabelled through inv_t)
// would be windowed. A cheap test on the original CSR, so LPs without
// column locality skip the device-order indices and the planning.
static bool windows_worth_planning(const opdhg_lp* lp, const Prepared& out,
                                   const std::vector<int32_t>& inv_t, int64_t chunk_rows,
                                   int per_pass, int one_cap) {
  if (lp->nnz < kWinMinChunks * kWinMinNnz) return false;
  const int64_t lo = out.cend_a[0], hi = lp->m;
  if (hi - lo < 8 * chunk_rows) return false;
  const int64_t nb = (lp->n + kWinBucket - 1) / kWinBucket;
  std::vector<int32_t> stamp(nb, -1);
  int ok = 0;
  for (int s = 0; s < 8; ++s) {
    const int64_t a = lo + (hi - lo - chunk_rows) * s / 7, b = a + chunk_rows;
    int64_t nz = 0, nbk = 0;
    for (int64_t r = a; r < b; ++r) {
      const int64_t i = out.perm_a[r];
      for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k) {
        const int64_t bk = inv_t[lp->col_idx[k]] / kWinBucket;
        ++nz;
        if (stamp[bk] != s) {
          stamp[bk] = s;
          ++nbk;
        }
      }
    }
    const bool passes_ok = nbk <= one_cap || (nbk + per_pass - 1) / per_pass <= kWinMaxPass;
    if (passes_ok && nbk * kWinBucket <= nz) ++ok;
  }
  return ok >= 4;
}

// Tiles over the rows of a side that no windowed chunk takes.
static std::vector<Tile> tiles_outside(const std::vector<int32_t>& rp, int64_t rows,
                                       const WinPlan& W, int64_t cap, int lanes) {
  std::vector<Tile> out;
  auto add = [&](int64_t a, int64_t b) {
    if (b <= a) return;
    for (Tile t : build_tiles(rp.data() + a, b - a, cap, lanes)) {
      t.rb += (int32_t)a;
      t.re += (int32_t)a;
      out.push_back(t);
    }
  };
  // rows taken elsewhere: the chunks' ranges and the segmented rows
  std::vector<std::pair<int64_t, int64_t>> taken;
  for (size_t c = 0; c < W.chunks(); ++c) taken.push_back({W.r0[c], W.r1[c]});
  for (int32_t r : W.srow) taken.push_back({r, r + 1});
  std::sort(taken.begin(), taken.end());
  int64_t cur = 0;
  for (auto& t : taken) {
    add(cur, t.first);
    cur = std::max(cur, t.second);
  }
  add(cur, rows);
  return out;
}

// Long-row tiles of a step list longer than kSplitNnz become pieces of
// kPieceNnz nonzeros (see Tile); their rows join the side's segments after
// the windowed plan's, which are kept as planned.
static void split_long_tiles(std::vector<Tile>& tiles, WinPlan& W) {
  W.srow.resize(W.nsrow_win);
  W.sids.resize(W.nsrow_win ? (size_t)W.sptr[W.nsrow_win] : 0);
  W.sptr.resize(W.nsrow_win ? W.nsrow_win + 1 : 0);
  W.nsegs = W.nsegs_win;
  std::vector<Tile> out;
  out.reserve(tiles.size());
  for (const Tile& t : tiles) {
    if (t.lanes != 0 || t.e - t.s <= kSplitNnz) {
      out.push_back(t);
      continue;
    }
    if (W.sptr.empty()) W.sptr.push_back(0);
    W.srow.push_back(t.rb);
    for (int32_t a = t.s; a < t.e; a += kPieceNnz) {
      const int32_t id = W.nsegs++;
      out.push_back(Tile{t.rb, t.re, a, std::min(t.e, a + kPieceNnz), -1, id});
      W.sids.push_back(id);
    }
    W.sptr.push_back((int32_t)W.sids.size());
  }
  tiles.swap(out);
}

void step_tiles(Prepared& P, int64_t cap, int lanes) {
  P.stiles_t = P.win_t.chunks() ? tiles_outside(P.rp_t, P.n, P.win_t, cap, lanes) : P.tiles_t;
  P.stiles_a = P.win_a.chunks() ? tiles_outside(P.rp_a, P.m, P.win_a, cap, lanes) : P.tiles_a;
  split_long_tiles(P.stiles_t, P.win_t);
  split_long_tiles(P.stiles_a, P.win_a);
}


// ---------------------------------------------------------------------------
// preparation: everything the device needs, computed on the host in FP64
// ---------------------------------------------------------------------------

// The step rule's factors (j+1)^-reduction and (j+1)^-growth for
// j = 1..kPowTab, correctly rounded (crmath.h; about 25 ms per table), kept
// per pair of exponents for the life of the process: every LP with the same
// exponents shares one table.
static std::vector<double> step_factor_table(double reduction, double growth) {
  static std::mutex mu;
  static std::map<std::pair<uint64_t, uint64_t>, std::vector<double>> cache;
  uint64_t kr = 0, kg = 0;
  std::memcpy(&kr, &reduction, 8);
  std::memcpy(&kg, &growth, 8);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({kr, kg});
  if (it != cache.end()) return it->second;
  std::vector<double> t(2 * kPowTab);
  for (int j = 1; j <= kPowTab; ++j) {
    t[j - 1] = crm::cr_pow((double)(j + 1), -reduction);
    t[kPowTab + j - 1] = crm::cr_pow((double)(j + 1), -growth);
  }
  if (cache.size() >= 64) cache.clear();  // a bound on what odd exponent sweeps keep
  return cache.emplace(std::make_pair(kr, kg), std::move(t)).first->second;
}

// The rest of a full preparation, after the structure: the vectors in
// device order (unscaled for the device-side preparation, scaled here
// otherwise), the first step size and primal weight (host side), and the
// per-LP constants. sval: the scaled values (host side); spec: the
// estimate of |A~|_2 for the constant step (host side).
static int prepare_finish(const opdhg_lp* lp, const opdhg_params* p, Prepared& out, double spec,
                          const std::vector<double>* sval_p) {
  const int64_t m = out.m, n = out.n, nnz = out.nnz;
  static const std::vector<double> kNone;
  const std::vector<double>& sval = sval_p ? *sval_p : kNone;
  if (out.dprep) {
    // unscaled vectors in device order; the device scales them
    out.raw_b.resize(m);
    out.sense.resize(m);
    for_blocks(m, item_blocks(m), [&](int, int64_t i0, int64_t i1) {
      for (int64_t i2 = i0; i2 < i1; ++i2) {
        const int64_t i = out.perm_a[i2];
        out.raw_b[i2] = lp->b[i];
        out.sense[i2] = lp->row_sense[i];
      }
    });
    out.raw_c.resize(n);
    out.raw_l.resize(n);
    out.raw_u.resize(n);
    out.bfin.resize(n);
    for_blocks(n, item_blocks(n), [&](int, int64_t j0, int64_t j1) {
      for (int64_t j2 = j0; j2 < j1; ++j2) {
        const int64_t j = out.perm_t[j2];
        out.raw_c[j2] = lp->c[j];
        out.raw_l[j2] = lp->l[j];
        out.raw_u[j2] = lp->u[j];
        out.bfin[j2] =
            (int8_t)((std::isfinite(lp->l[j]) ? 1 : 0) | (std::isfinite(lp->u[j]) ? 2 : 0));
      }
    });
  }
  out.b.resize(out.dprep ? 0 : m);
  out.sense.resize(m);
  out.dr_dev.resize(out.dprep ? 0 : m);

  for (int64_t i2 = 0; i2 < m && !out.dprep; ++i2) {
    const int64_t i = out.perm_a[i2];
    out.b[i2] = out.dr[i] * lp->b[i];
    out.sense[i2] = lp->row_sense[i];
    out.dr_dev[i2] = out.dr[i];
  }
  const int64_t nh = out.dprep ? 0 : n;
  out.c.resize(nh);
  out.l.resize(nh);
  out.u.resize(nh);
  if (!out.dprep) out.bfin.resize(n);
  out.x0.resize(nh);
  out.dc_dev.resize(nh);
  for (int64_t j2 = 0; j2 < nh; ++j2) {
    const int64_t j = out.perm_t[j2];
    out.c[j2] = out.dc[j] * lp->c[j];
    out.l[j2] = lp->l[j] / out.dc[j];
    out.u[j2] = lp->u[j] / out.dc[j];
    out.bfin[j2] = (int8_t)((std::isfinite(lp->l[j]) ? 1 : 0) | (std::isfinite(lp->u[j]) ? 2 : 0));
    const double z = 0.0;
    out.x0[j2] = std::min(std::max(z, out.l[j2]), out.u[j2]);
    out.dc_dev[j2] = out.dc[j];
  }
  if (!out.dprep) {
    double amax = 0.0;
    for (int64_t k = 0; k < nnz; ++k) amax = std::max(amax, std::fabs(sval[k]));
    const double bsn = dd_norm(out.b.data(), m);
    const double csn = dd_norm(out.c.data(), n);
    out.omega0 = (csn > 1e-10 && bsn > 1e-10) ? csn / bsn : 1.0;
    if (p->step_rule == OPDHG_STEP_CONSTANT)
      out.eta0 = spec > 0.0 ? p->step_scale / spec : p->step_scale;
    else
      out.eta0 = amax > 0.0 ? 1.0 / amax : 1.0;
  }
  DevParams& d = out.prm;
  std::memset(&d, 0, sizeof(d));
  d.tol = p->tol;
  d.lr = p->lr;
  d.floor = p->precond_floor;
  d.beta_suff = p->beta_suff;
  d.beta_nec = p->beta_nec;
  d.beta_art = p->beta_art;
  d.pw_smoothing = p->pw_smoothing;
  d.step_growth = p->step_growth;
  d.step_reduction = p->step_reduction;
  d.b_norm = dd_norm(lp->b, m);
  d.c_norm = dd_norm(lp->c, n);
  out.pow_tab = step_factor_table(p->step_reduction, p->step_growth);
  d.c0 = lp->obj_offset;
  d.max_iter = p->max_iter;
  d.phi = p->phi;
  d.normalize = p->normalize ? 1 : 0;
  d.schedule = p->schedule;
  d.eval_every = p->eval_every;
  d.max_retries = p->max_step_retries;
  bool lower_zero = true, no_upper = true;
  for (int64_t j = 0; j < n && (lower_zero || no_upper); ++j) {
    lower_zero = lower_zero && lp->l[j] == 0.0;
    no_upper = no_upper && lp->u[j] == std::numeric_limits<double>::infinity();
  }
  d.flags = (p->step_rule == OPDHG_STEP_CONSTANT ? kConstantStep : 0) |
            (p->restart_scheme == OPDHG_RESTART_NONE ? kNoRestart : 0) |
            (p->step_norm == OPDHG_STEP_NORM_PRECOND ? kWeightedStep : 0) |
            (lower_zero ? kLowerZero : 0) | (no_upper ? kNoUpper : 0);
  return OPDHG_OK;
}

int prepare(const opdhg_lp* lp, const opdhg_params* p, Prepared& out, bool structure_only) {
  out.m = lp->m;
  out.n = lp->n;
  out.nnz = lp->nnz;
  const int64_t m = lp->m, n = lp->n, nnz = lp->nnz;
  // device-side preparation: the rescaling and the scaled data on the GPU
  out.dprep =
      p->prep == OPDHG_PREP_DEVICE || (p->prep == OPDHG_PREP_AUTO && nnz >= kDevicePrepNnz);
  // A full host preparation needs the column index anyway: it is built
  // first and gives the column counts; sizing alone, and the device-side
  // preparation (which may build the structure on the device), count the
  // columns.
  ColIndex C;
  bool have_index = false;
  if (!structure_only && !out.dprep) {
    build_col_index(lp, C, true);
    have_index = true;
  }
  // row lengths of A and of A^T (= column counts), device order by class
  std::vector<int64_t> len_a(m), len_t(n, 0);
  for_blocks(m, item_blocks(m), [&](int, int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) len_a[i] = lp->row_ptr[i + 1] - lp->row_ptr[i];
  });
  if (have_index) {
    for (int64_t j = 0; j < n; ++j) len_t[j] = C.cstart[j + 1] - C.cstart[j];
  } else {
    column_counts(lp, len_t);
  }
  class_order(len_a, out.perm_a, out.cend_a);
  class_order(len_t, out.perm_t, out.cend_t);
  device_row_ptr(len_a, out.perm_a, out.rp_a);
  device_row_ptr(len_t, out.perm_t, out.rp_t);
  const int64_t cap = p->tile_nnz > 0 ? std::min<int64_t>(p->tile_nnz, kTileCap) : kTileCap;
  out.tiles_a = build_tiles(out.rp_a.data(), m, cap, p->lanes);
  out.tiles_t = build_tiles(out.rp_t.data(), n, cap, p->lanes);
  // windowed chunks need the device-order column indices, also for sizing;
  // automatic windows only where a sample of chunks shows column locality
  bool windows = p->precision == OPDHG_FP32 && p->windows != OPDHG_WINDOWS_OFF;
  const int per_pass = window_per_pass(p), one_cap = window_one_pass(p);
  if (windows && p->windows == OPDHG_WINDOWS_AUTO) {
    std::vector<int32_t> inv(n);
    for (int64_t j = 0; j < n; ++j) inv[out.perm_t[j]] = (int32_t)j;
    windows = windows_worth_planning(lp, out, inv, window_chunk_rows(p, m - out.cend_a[0]),
                                     per_pass, one_cap);
  }
  out.prep_ruiz = p->ruiz_iters;
  out.prep_l2 = p->l2_rescale != 0;
  out.prep_beta = p->pc_beta;
  out.prep_power = p->step_rule == OPDHG_STEP_CONSTANT;
  out.prep_power_iters = p->power_iters;
  out.prep_power_tol = p->power_tol;
  out.prep_step_scale = p->step_scale;
  // device-side structure: with the device preparation and no windowed
  // chunks (whose planning needs the structure on the host), when every
  // column fits the device's per-column ordering
  int64_t max_col = 0;
  for (int64_t j = 0; j < n; ++j) max_col = std::max(max_col, len_t[j]);
  out.dstruct = out.dprep && !windows && nnz > 0 && max_col <= kStructMaxCol;
  if (structure_only && !windows) {
    step_tiles(out, cap, p->lanes);
    return OPDHG_OK;
  }

  std::vector<int32_t> inv_a(m), inv_t(n);
  for (int64_t i = 0; i < m; ++i) inv_a[out.perm_a[i]] = (int32_t)i;
  for (int64_t j = 0; j < n; ++j) inv_t[out.perm_t[j]] = (int32_t)j;
  if (out.dstruct) {
    // the device builds both CSR copies from the caller's arrays
    out.h_rp = lp->row_ptr;
    out.h_ci = lp->col_idx;
    out.h_val = lp->val;
    out.inv_a = std::move(inv_a);
    out.inv_t = std::move(inv_t);
    out.win_t = WinPlan();
    out.win_a = WinPlan();
    step_tiles(out, cap, p->lanes);
    if (structure_only) return OPDHG_OK;
    return prepare_finish(lp, p, out, 0.0, nullptr);
  }
  std::vector<double> sval;
  if (!have_index) build_col_index(lp, C, !out.dprep);
  double spec = -1.0;
  if (!structure_only && !out.dprep) {
    rescale_with(lp, C, p->ruiz_iters, p->l2_rescale != 0, p->pc_beta, sval, out.dr, out.dc);
    if (p->step_rule == OPDHG_STEP_CONSTANT)
      spec = spectral_norm_with(lp, C, sval, p->power_iters, p->power_tol);
  }
  // values go to the device order: scaled on the host, or unscaled (raw)
  // for the device-side preparation
  const bool vals = !structure_only;
  const double* vsrc = out.dprep ? lp->val : sval.data();
  // A in device order: row i' is original row perm_a[i'], columns relabelled
  out.ci_a.resize(nnz);
  HostArray<double>& dst_a = out.dprep ? out.raw_a : out.va_a;
  HostArray<double>& dst_t = out.dprep ? out.raw_t : out.va_t;
  if (vals) dst_a.resize(nnz);
  {
    std::vector<int64_t> dptr(m + 1);  // nonzero offsets in device order, for balancing
    for (int64_t i2 = 0; i2 <= m; ++i2) dptr[i2] = out.rp_a[i2];
    parallel_rows(dptr.data(), m, [&](int64_t r0, int64_t r1) {
      for (int64_t i2 = r0; i2 < r1; ++i2) {
        const int64_t i = out.perm_a[i2];
        int64_t pos = out.rp_a[i2];
        for (int64_t k = lp->row_ptr[i]; k < lp->row_ptr[i + 1]; ++k, ++pos) {
          out.ci_a[pos] = inv_t[lp->col_idx[k]];
          if (vals) dst_a[pos] = vsrc[k];
        }
      }
    });
  }
  // A^T in device order: row j' is original column perm_t[j']; entries in
  // ascending original row, labelled with device row indices
  out.ci_t.resize(nnz);
  if (vals) dst_t.resize(nnz);
  {
    std::vector<int64_t> dptr(n + 1);
    for (int64_t j2 = 0; j2 <= n; ++j2) dptr[j2] = out.rp_t[j2];
    parallel_rows(dptr.data(), n, [&](int64_t r0, int64_t r1) {
      for (int64_t j2 = r0; j2 < r1; ++j2) {
        const int64_t j = out.perm_t[j2];
        int64_t pos = out.rp_t[j2];
        for (int64_t q = C.cstart[j]; q < C.cstart[j + 1]; ++q, ++pos) {
          out.ci_t[pos] = inv_a[C.crow[q]];
          if (vals) dst_t[pos] = vsrc[C.cpos[q]];
        }
      }
    });
  }
  // windowed chunks of both sides (rows of the long class stay in tiles):
  // A^T rows gather y (m entries), A rows gather x' (n entries)
  out.win_t = WinPlan();
  out.win_a = WinPlan();
  if (windows) {
    plan_windows(out.rp_t, out.ci_t, m, out.cend_t[0], n, out.cend_t[0],
                 window_chunk_rows(p, n - out.cend_t[0]), per_pass, one_cap, out.win_t);
    plan_windows(out.rp_a, out.ci_a, n, out.cend_a[0], m, out.cend_a[0],
                 window_chunk_rows(p, m - out.cend_a[0]), per_pass, one_cap, out.win_a);
    if (!plan_ok(out.win_t, n, m) || !plan_ok(out.win_a, m, n))
      return fail(OPDHG_ERR_DEVICE, "internal error: inconsistent window plan");
    if (p->windows == OPDHG_WINDOWS_AUTO) {
      if ((int64_t)out.win_t.chunks() < kWinMinChunks) out.win_t = WinPlan();
      if ((int64_t)out.win_a.chunks() < kWinMinChunks) out.win_a = WinPlan();
    }
  }
  for (WinPlan* W : {&out.win_t, &out.win_a}) {
    W->nsrow_win = W->srow.size();
    W->nsegs_win = W->nsegs;
  }
  step_tiles(out, cap, p->lanes);
  if (structure_only) return OPDHG_OK;
  return prepare_finish(lp, p, out, spec, &sval);
}

// Device-order vector back to the caller's order, scaled by `scale`
// (the unscaling diagonal) when given.
void unpermute(const double* dev, const std::vector<int32_t>& perm, const double* scale,
               double* out) {
  const size_t n = perm.size();
  for (size_t i = 0; i < n; ++i) {
    const int32_t o = perm[i];
    out[o] = scale ? dev[i] * scale[o] : dev[i];
  }
}

// ---------------------------------------------------------------------------
// workspace layout of one LP slot
// ---------------------------------------------------------------------------

static size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

SlotLayout slot_layout(const Prepared& P, int prec) {
  const int64_t m = P.m, n = P.n, nnz = P.nnz;
  const int64_t ntiles_t = (int64_t)P.tiles_t.size(), ntiles_a = (int64_t)P.tiles_a.size();
  SlotLayout L;
  const size_t V = prec == OPDHG_FP32 ? 4 : 8;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  L.ctl = take(sizeof(Ctl));
  L.prm = take(sizeof(DevParams));
  L.tiles_a = take(sizeof(Tile) * ntiles_a);
  L.tiles_t = take(sizeof(Tile) * ntiles_t);
  L.part_a = take(sizeof(double) * kPartStride * P.part_stride_a());
  L.part_t = take(sizeof(double) * kPartStride * P.part_stride_t());
  L.pow_tab = take(sizeof(double) * 2 * kPowTab);
  L.pow_ring = take(sizeof(double) * 2 * kPowRing);
  L.rp_a = take(4 * (m + 1));
  L.ci_a = take(4 * nnz);
  L.va_a = take(V * nnz);
  L.rp_t = take(4 * (n + 1));
  L.ci_t = take(4 * nnz);
  L.va_t = take(V * nnz);
  for (int q = 0; q < SlotLayout::kNVecN; ++q) L.vn[q] = take(V * n);
  L.dc = take(8 * n);
  L.bfin = take(n);
  for (int q = 0; q < SlotLayout::kNVecM; ++q) L.vm[q] = take(V * m);
  L.dr = take(8 * m);
  L.sense = take(m);
  if (P.win_t.chunks()) {
    const size_t e = P.win_t.col.size();
    L.wcol_t = take(2 * e);
    L.wlane_t = take(2 * P.win_t.lane.size());
    L.wslice_t = take(sizeof(WinSlice) * P.win_t.slices.size());
    L.wval_t = take(V * e);
    L.wpass_t = take(sizeof(WinPass) * P.win_t.passes.size());
    L.wrange_t = take(sizeof(WinRange) * P.win_t.ranges.size());
  }
  if (!P.win_t.srow.empty()) {  // segmented rows (windowed chunks or split tiles)
    L.segp_t = take((V == 8 ? 16 : 4) * (size_t)P.win_t.nsegs);
    L.srow_t = take(4 * P.win_t.srow.size());
    L.sptr_t = take(4 * P.win_t.sptr.size());
    L.sids_t = take(4 * P.win_t.sids.size());
  }
  if (P.win_a.chunks()) {
    const size_t e = P.win_a.col.size();
    L.wcol_a = take(2 * e);
    L.wlane_a = take(2 * P.win_a.lane.size());
    L.wslice_a = take(sizeof(WinSlice) * P.win_a.slices.size());
    L.wval_a = take(V * e);
    L.wpass_a = take(sizeof(WinPass) * P.win_a.passes.size());
    L.wrange_a = take(sizeof(WinRange) * P.win_a.ranges.size());
  }
  if (!P.win_a.srow.empty()) {  // segmented rows (windowed chunks or split tiles)
    L.segp_a = take((V == 8 ? 16 : 4) * (size_t)P.win_a.nsegs);
    L.srow_a = take(4 * P.win_a.srow.size());
    L.sptr_a = take(4 * P.win_a.sptr.size());
    L.sids_a = take(4 * P.win_a.sids.size());
  }
  if (prec == OPDHG_FP32 && (P.win_t.chunks() || P.win_a.chunks())) {
    L.has_evp = true;
    L.evp_t0 = take(4 * n);
    L.evp_t1 = take(4 * n);
    L.evp_a = take(4 * m);
  }
  if (P.dprep) {
    L.raw_a = take(8 * nnz);
    L.raw_t = take(8 * nnz);
    L.raw_b = take(8 * m);
    L.raw_c = take(8 * n);
    L.raw_l = take(8 * n);
    L.raw_u = take(8 * n);
    L.sr = take(8 * m);
    L.sc = take(8 * n);
    L.pscr = take(8 * kPrepScr);
    if (P.win_t.chunks()) L.wsrc_t = take(4 * P.win_t.src.size());
    if (P.win_a.chunks()) L.wsrc_a = take(4 * P.win_a.src.size());
  }
  if (P.dstruct) {
    L.st_perm_a = take(4 * m);
    L.st_inv_a = take(4 * m);
    L.st_inv_t = take(4 * n);
    L.st_cur = take(4 * n);
    // the caller's arrays and the entries' places last: the host image
    // skips them (and the CSR copies the device builds)
    L.st_rp = take(8 * (m + 1));
    L.st_ci = take(4 * nnz);
    L.st_val = take(8 * nnz);
    L.st_ti = take(4 * nnz);
    L.st_tk = take(4 * nnz);
  }
  L.total = off;
  return L;
}

// n-vector slots: c l u T Hp Gp x0 x1 xs0 xs1 xa
// m-vector slots: b S Hd Gd y0 y1 ys0 ys1 ya Ax0 Ax1 Axa
LpDev slot_pointers(uint8_t* base, const SlotLayout& L, const Prepared& P) {
  LpDev d;
  std::memset(&d, 0, sizeof(d));
  d.m = (int32_t)P.m;
  d.n = (int32_t)P.n;
  d.ntiles_t = (int32_t)P.part_stride_t();
  d.ntiles_a = (int32_t)P.part_stride_a();
  d.rp_a = reinterpret_cast<const int32_t*>(base + L.rp_a);
  d.ci_a = reinterpret_cast<const int32_t*>(base + L.ci_a);
  d.va_a = base + L.va_a;
  d.rp_t = reinterpret_cast<const int32_t*>(base + L.rp_t);
  d.ci_t = reinterpret_cast<const int32_t*>(base + L.ci_t);
  d.va_t = base + L.va_t;
  d.tiles_a = reinterpret_cast<const Tile*>(base + L.tiles_a);
  d.tiles_t = reinterpret_cast<const Tile*>(base + L.tiles_t);
  void** vn[SlotLayout::kNVecN] = {&d.c,     &d.l,     &d.u,     &d.T,      &d.Hp,  &d.Gp,
                                   &d.x[0],  &d.x[1],  &d.xs[0], &d.xs[1],  &d.xa};
  for (int q = 0; q < SlotLayout::kNVecN; ++q) *vn[q] = base + L.vn[q];
  void** vm[SlotLayout::kNVecM] = {&d.b,      &d.S,      &d.Hd, &d.Gd,    &d.y[0],  &d.y[1],
                                   &d.ys[0],  &d.ys[1],  &d.ya, &d.Ax[0], &d.Ax[1], &d.Axa};
  for (int q = 0; q < SlotLayout::kNVecM; ++q) *vm[q] = base + L.vm[q];
  d.dr = reinterpret_cast<const double*>(base + L.dr);
  d.dc = reinterpret_cast<const double*>(base + L.dc);
  d.sense = reinterpret_cast<const int8_t*>(base + L.sense);
  d.bfin = reinterpret_cast<const int8_t*>(base + L.bfin);
  d.part_t = reinterpret_cast<double*>(base + L.part_t);
  d.part_a = reinterpret_cast<double*>(base + L.part_a);
  d.pow_tab = reinterpret_cast<const double*>(base + L.pow_tab);
  d.pow_ring = reinterpret_cast<double*>(base + L.pow_ring);
  d.ctl = reinterpret_cast<Ctl*>(base + L.ctl);
  d.prm = reinterpret_cast<const DevParams*>(base + L.prm);
  d.s_lr = P.prm.lr;
  d.s_max_iter = P.prm.max_iter;
  d.s_phi = P.prm.phi;
  d.s_schedule = P.prm.schedule;
  d.s_normalize = P.prm.normalize;
  d.s_eval_every = P.prm.eval_every;
  d.s_max_retries = P.prm.max_retries;
  d.s_flags = P.prm.flags;
  if (P.win_t.chunks()) {
    d.wcol_t = reinterpret_cast<const uint16_t*>(base + L.wcol_t);
    d.wlane_t = reinterpret_cast<const uint16_t*>(base + L.wlane_t);
    d.wslice_t = reinterpret_cast<const WinSlice*>(base + L.wslice_t);
    d.wval_t = base + L.wval_t;
    d.wpass_t = reinterpret_cast<const WinPass*>(base + L.wpass_t);
    d.wrange_t = reinterpret_cast<const WinRange*>(base + L.wrange_t);
  }
  if (!P.win_t.srow.empty()) {
    d.segp_t = base + L.segp_t;
    d.srow_t = reinterpret_cast<const int32_t*>(base + L.srow_t);
    d.sptr_t = reinterpret_cast<const int32_t*>(base + L.sptr_t);
    d.sids_t = reinterpret_cast<const int32_t*>(base + L.sids_t);
  }
  if (P.win_a.chunks()) {
    d.wcol_a = reinterpret_cast<const uint16_t*>(base + L.wcol_a);
    d.wlane_a = reinterpret_cast<const uint16_t*>(base + L.wlane_a);
    d.wslice_a = reinterpret_cast<const WinSlice*>(base + L.wslice_a);
    d.wval_a = base + L.wval_a;
    d.wpass_a = reinterpret_cast<const WinPass*>(base + L.wpass_a);
    d.wrange_a = reinterpret_cast<const WinRange*>(base + L.wrange_a);
  }
  if (L.has_evp) {
    d.evp_t0 = reinterpret_cast<float*>(base + L.evp_t0);
    d.evp_t1 = reinterpret_cast<float*>(base + L.evp_t1);
    d.evp_a = reinterpret_cast<float*>(base + L.evp_a);
  }
  if (!P.win_a.srow.empty()) {
    d.segp_a = base + L.segp_a;
    d.srow_a = reinterpret_cast<const int32_t*>(base + L.srow_a);
    d.sptr_a = reinterpret_cast<const int32_t*>(base + L.sptr_a);
    d.sids_a = reinterpret_cast<const int32_t*>(base + L.sids_a);
  }
  return d;
}

template <typename V, typename Vec>
static void put_vec(SlotImage& img, size_t off, const Vec& v) {
  V* dst = reinterpret_cast<V*>(img.data() + off);
  for (size_t i = 0; i < v.size(); ++i) dst[i] = (V)v[i];
}

template <typename V>
static void put_const(SlotImage& img, size_t off, size_t count, double value) {
  V* dst = reinterpret_cast<V*>(img.data() + off);
  for (size_t i = 0; i < count; ++i) dst[i] = (V)value;
}

Ctl initial_ctl(const Prepared& P) {
  Ctl c;
  std::memset(&c, 0, sizeof(c));
  c.eta = P.eta0;
  c.omega = P.omega0;
  c.prev_cand = INFINITY;
  c.k_limit = std::numeric_limits<int64_t>::max();
  c.status = kRunning;
  c.need_eval = 1;
  c.learn_now = P.prm.lr > 0.0 ? 1 : 0;
  c.weighted_step = (P.prm.flags & kWeightedStep) ? 1 : 0;
  return c;
}

// Byte ranges of a slot that the host image fills and uploads: the whole
// slot, or with the device-side structure everything but the CSR copies
// and their values (built on the device) and the staging of the caller's
// arrays (uploaded from them directly).
static std::vector<std::pair<size_t, size_t>> image_ranges(const SlotLayout& L, const Prepared& P) {
  if (!P.dstruct) return {{0, L.total}};
  return {{0, L.ci_a}, {L.rp_t, L.ci_t}, {L.vn[0], L.raw_a}, {L.raw_b, L.st_rp}};
}

// Host image of a slot: every byte the device needs at the start.
template <typename V>
void slot_image(const SlotLayout& L, const Prepared& P, SlotImage& img) {
  // every byte that goes up starts at zero; the threads that zero the pages
  // touch them (with the device-side structure only the ranges that go up)
  img.resize(L.total);
  for (const auto& r : image_ranges(L, P))
    parallel_pieces(r.second - r.first, size_t(1) << 22, [&](size_t a, size_t b) {
      std::memset(img.data() + r.first + a, 0, b - a);
    });
  const Ctl c = initial_ctl(P);
  std::memcpy(img.data() + L.ctl, &c, sizeof(c));
  std::memcpy(img.data() + L.prm, &P.prm, sizeof(DevParams));
  std::memcpy(img.data() + L.tiles_a, P.tiles_a.data(), sizeof(Tile) * P.tiles_a.size());
  std::memcpy(img.data() + L.tiles_t, P.tiles_t.data(), sizeof(Tile) * P.tiles_t.size());
  std::memcpy(img.data() + L.pow_tab, P.pow_tab.data(), sizeof(double) * P.pow_tab.size());
  std::memcpy(img.data() + L.rp_a, P.rp_a.data(), 4 * P.rp_a.size());
  std::memcpy(img.data() + L.rp_t, P.rp_t.data(), 4 * P.rp_t.size());
  if (P.dstruct) {
    std::memcpy(img.data() + L.st_perm_a, P.perm_a.data(), 4 * P.perm_a.size());
    std::memcpy(img.data() + L.st_inv_a, P.inv_a.data(), 4 * P.inv_a.size());
    std::memcpy(img.data() + L.st_inv_t, P.inv_t.data(), 4 * P.inv_t.size());
    std::memcpy(img.data() + L.st_cur, P.rp_t.data(), 4 * P.n);  // A^T rows fill from their starts
  }
  // the nonzero-sized arrays, one thread each (the device builds them from
  // the caller's arrays with the device-side structure)
  if (!P.dstruct)
  run_tasks({[&] { std::memcpy(img.data() + L.ci_a, P.ci_a.data(), 4 * P.ci_a.size()); },
             [&] { std::memcpy(img.data() + L.ci_t, P.ci_t.data(), 4 * P.ci_t.size()); },
             [&] { put_vec<V>(img, L.va_a, P.va_a); },
             [&] { put_vec<V>(img, L.va_t, P.va_t); },
             [&] {
               if (P.dprep && !P.raw_a.empty())
                 std::memcpy(img.data() + L.raw_a, P.raw_a.data(), 8 * P.raw_a.size());
             },
             [&] {
               if (P.dprep && !P.raw_t.empty())
                 std::memcpy(img.data() + L.raw_t, P.raw_t.data(), 8 * P.raw_t.size());
             }});
  auto put_win = [&](const WinPlan& W, const auto& va, size_t oc, size_t olane, size_t oslice,
                     size_t ov, size_t opass, size_t orange, size_t osrow, size_t osptr,
                     size_t osids, size_t owsrc) {
    if (!W.srow.empty()) {
      std::memcpy(img.data() + osrow, W.srow.data(), 4 * W.srow.size());
      std::memcpy(img.data() + osptr, W.sptr.data(), 4 * W.sptr.size());
      std::memcpy(img.data() + osids, W.sids.data(), 4 * W.sids.size());
    }
    if (!W.chunks()) return;
    if (P.dprep) {  // the device fills the values from the scaled entries they stand for
      int32_t* ws = reinterpret_cast<int32_t*>(img.data() + owsrc);
      for (size_t e = 0; e < W.src.size(); ++e) ws[e] = (int32_t)W.src[e];
    }
    std::memcpy(img.data() + oc, W.col.data(), 2 * W.col.size());
    std::memcpy(img.data() + olane, W.lane.data(), 2 * W.lane.size());
    std::memcpy(img.data() + oslice, W.slices.data(), sizeof(WinSlice) * W.slices.size());
    V* dst = reinterpret_cast<V*>(img.data() + ov);
    if (!P.dprep)
      for (size_t e = 0; e < W.src.size(); ++e) dst[e] = W.src[e] < 0 ? V(0) : (V)va[W.src[e]];
    std::memcpy(img.data() + opass, W.passes.data(), sizeof(WinPass) * W.passes.size());
    std::memcpy(img.data() + orange, W.ranges.data(), sizeof(WinRange) * W.ranges.size());
  };
  put_win(P.win_t, P.va_t, L.wcol_t, L.wlane_t, L.wslice_t, L.wval_t, L.wpass_t, L.wrange_t,
          L.srow_t, L.sptr_t, L.sids_t, L.wsrc_t);
  put_win(P.win_a, P.va_a, L.wcol_a, L.wlane_a, L.wslice_a, L.wval_a, L.wpass_a, L.wrange_a,
          L.srow_a, L.sptr_a, L.sids_a, L.wsrc_a);
  if (P.dprep) {
    auto put64 = [&](size_t o, const auto& v) {
      if (!v.empty()) std::memcpy(img.data() + o, v.data(), 8 * v.size());
    };
    put64(L.raw_b, P.raw_b);
    put64(L.raw_c, P.raw_c);
    put64(L.raw_l, P.raw_l);
    put64(L.raw_u, P.raw_u);
    // the diagonals start at 1; the device rescales them
    double* dr = reinterpret_cast<double*>(img.data() + L.dr);
    for (int64_t i = 0; i < P.m; ++i) dr[i] = 1.0;
    double* dc = reinterpret_cast<double*>(img.data() + L.dc);
    for (int64_t j = 0; j < P.n; ++j) dc[j] = 1.0;
  }
  // n-vectors: c l u T Hp Gp x0 x1 xs0 xs1 xa
  put_vec<V>(img, L.vn[0], P.c);
  put_vec<V>(img, L.vn[1], P.l);
  put_vec<V>(img, L.vn[2], P.u);
  put_const<V>(img, L.vn[3], P.n, 1.0);
  put_vec<V>(img, L.vn[6], P.x0);
  put_vec<V>(img, L.vn[10], P.x0);
  std::memcpy(img.data() + L.dc, P.dc_dev.data(), 8 * P.dc_dev.size());
  std::memcpy(img.data() + L.bfin, P.bfin.data(), P.bfin.size());
  // m-vectors: b S Hd Gd y0 y1 ys0 ys1 ya Ax0 Ax1 Axa
  put_vec<V>(img, L.vm[0], P.b);
  put_const<V>(img, L.vm[1], P.m, 1.0);
  std::memcpy(img.data() + L.dr, P.dr_dev.data(), 8 * P.dr_dev.size());
  if (P.m) std::memcpy(img.data() + L.sense, P.sense.data(), P.sense.size());
}

template void slot_image<double>(const SlotLayout&, const Prepared&, SlotImage&);
template void slot_image<float>(const SlotLayout&, const Prepared&, SlotImage&);

// ---------------------------------------------------------------------------
// a group of LPs launched together (one LP, a batch, or the server's mix)
// ---------------------------------------------------------------------------

int mid_eval_every(const opdhg_params* p, int64_t nlps) {
  if (p->eval_slots != 0) return p->eval_slots > 0 ? p->eval_slots : 0;
  return nlps > 1 ? kMidEvalEveryShared : kMidEvalEvery;
}

int Group::enqueue(hipStream_t s, int attempts) {
  int rc = 0;
  auto K = [&](auto tag) {
    using V = decltype(tag);
    auto evaluation = [&](int mid) {
      // the opening evaluation of LPs with windowed chunks takes its sparse
      // products from the windowed machinery; the guarded ones gather
      if (mid == 0) rc |= Kernels<V>::eval_products(cfg, s);
      rc |= Kernels<V>::eval_t(cfg, s, mid);
      rc |= Kernels<V>::eval_a(cfg, s, mid);
      rc |= Kernels<V>::eval_decide(cfg, s, mid);
      rc |= Kernels<V>::apply(cfg, s, mid);
    };
    evaluation(0);
    for (int a = 0, b = 0; a < attempts; ++a) {
      if (a > 0 && mid_every > 0 && a % mid_every == 0) evaluation(++b);
      rc |= launch_side(true, 0, s);
      rc |= launch_side(false, 0, s);
      rc |= Kernels<V>::decide(cfg, s);
    }
    rc |= launch_board(cfg, s);
  };
  if (prec == OPDHG_FP32) K(float{});
  else K(double{});
  return rc;
}

int Group::capture(int attempts_per_replay) {
  // the step-rule factor ring covers kPowRing attempts per launch sequence
  attempts_per_replay = std::min(std::max(1, attempts_per_replay), kPowRing);
  if (direct) {
    seq_attempts = attempts_per_replay;
    return OPDHG_OK;
  }
  if (exec) {
    (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue(cap_stream, attempts_per_replay);
  hipError_t e = hipStreamEndCapture(cap_stream, &graph);
  if (rc != 0) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(OPDHG_ERR_DEVICE, std::string("kernel launch failed: ") + device_error_string());
  }
  if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail_hip(e, "hipGraphInstantiate");
  return OPDHG_OK;
}

// One side of an attempt (primal: A^T, dual: A): the tile kernel for the
// rows in tiles, the windowed kernel for the windowed chunks. They take
// disjoint rows and partial slots, so when both run, the tile kernel goes
// to side_stream (forked from and joined back into s by events) and the
// two overlap on the device.
int Group::launch_side(bool primal, int force, hipStream_t s) {
  const bool tiles = !cfg.step_fixed || (primal ? cfg.sgrid_t : cfg.sgrid_a) > 0;
  const bool wins = (primal ? cfg.nwin_t : cfg.nwin_a) > 0;
  auto tile = [&](hipStream_t q) {
    if (prec == OPDHG_FP32)
      return primal ? Kernels<float>::primal(cfg, q, force) : Kernels<float>::dual(cfg, q, force);
    return primal ? Kernels<double>::primal(cfg, q, force) : Kernels<double>::dual(cfg, q, force);
  };
  auto win = [&](hipStream_t q) {
    if (prec == OPDHG_FP32)
      return primal ? Kernels<float>::primal_win(cfg, q, force)
                    : Kernels<float>::dual_win(cfg, q, force);
    return primal ? Kernels<double>::primal_win(cfg, q, force)
                  : Kernels<double>::dual_win(cfg, q, force);
  };
  // segmented long rows finish after the windowed chunks wrote their partials
  auto seg = [&](hipStream_t q) {
    if ((primal ? cfg.nseg_t : cfg.nseg_a) <= 0) return 0;
    if (prec == OPDHG_FP32)
      return primal ? Kernels<float>::primal_seg(cfg, q, force)
                    : Kernels<float>::dual_seg(cfg, q, force);
    return primal ? Kernels<double>::primal_seg(cfg, q, force)
                  : Kernels<double>::dual_seg(cfg, q, force);
  };
  // the finishing kernel reads partials of windowed chunks and of split
  // tiles, so it runs after both
  if (!(tiles && wins) || !side_stream)
    return (tiles ? tile(s) : 0) | (wins ? win(s) : 0) | seg(s);
  if (hipEventRecord(ev_fork, s) != hipSuccess ||
      hipStreamWaitEvent(side_stream, ev_fork, 0) != hipSuccess)
    return -1;
  int rc = tile(side_stream);
  if (hipEventRecord(ev_join, side_stream) != hipSuccess) return -1;
  rc |= win(s);
  if (hipStreamWaitEvent(s, ev_join, 0) != hipSuccess) return -1;
  rc |= seg(s);
  return rc;
}

int Group::init(void* stream_, int prec_, bool direct_) {
  stream = (hipStream_t)stream_;
  prec = prec_;
  direct = direct_;
  if (direct) {
    // outside any capture: the windowed kernels' LDS attribute (no allocation)
    if (prec == OPDHG_FP32 && window_kernels_ready())
      return fail(OPDHG_ERR_DEVICE, device_error_string());
    return OPDHG_OK;
  }
  HIP_TRY(hipStreamCreateWithFlags(&side_stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
  // outside any capture: the windowed kernels' LDS attribute
  if (prec == OPDHG_FP32 && window_kernels_ready())
    return fail(OPDHG_ERR_DEVICE, device_error_string());
  HIP_TRY(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  return OPDHG_OK;
}

void Group::release() {
  if (exec) (void)hipGraphExecDestroy(exec);
  exec = nullptr;
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  cap_stream = nullptr;
  if (side_stream) (void)hipStreamDestroy(side_stream);
  side_stream = nullptr;
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  ev_fork = ev_join = nullptr;
}

int Group::launch_learn_flush() {
  if (prec == OPDHG_FP32) return Kernels<float>::learn_flush(cfg, stream);
  return Kernels<double>::learn_flush(cfg, stream);
}

int Group::launch_init() {
  if (prec == OPDHG_FP32) return Kernels<float>::init_products(cfg, stream);
  return Kernels<double>::init_products(cfg, stream);
}

// A forced launch of a side, as in the captured sequence.
int Group::launch_primal_forced() { return launch_side(true, 1, stream); }

int Group::launch_dual_forced() { return launch_side(false, 1, stream); }

int Group::replay() {
  if (direct) {
    if (enqueue(stream, seq_attempts))
      return fail(OPDHG_ERR_DEVICE, std::string("kernel launch failed: ") + device_error_string());
    return OPDHG_OK;
  }
  HIP_TRY(hipGraphLaunch(exec, stream));
  return OPDHG_OK;
}

// ---------------------------------------------------------------------------
// single-LP session
// ---------------------------------------------------------------------------

struct SessionImpl {
  Prepared P;
  SlotLayout L;
  uint8_t* ws = nullptr;
  LpDev lpd;
  Group grp;
  uint8_t* d_tables = nullptr;  // LpDev, WorkItems and BatchDev live after the slot
  Ctl* h_ctl = nullptr;         // pinned readback (direct mode: h_ctl_local)
  Ctl h_ctl_local{};
  bool direct = false;          // no graph, streams, events or pinned memory of its own
  double time_limit = 600.0;
  double elapsed = 0.0;
  int replays = 0;
};

// Chunking of a work list of n items over at most `cap` workgroups. A grid
// of more than 8 workgroups is rounded up to a multiple of 8 (with empty
// chunks) so the kernels can give each XCD a contiguous range of chunks.
void chunking(int64_t n, int64_t cap, int* grid, int* chunk) {
  const int64_t g0 = std::max<int64_t>(1, std::min<int64_t>(n, cap));
  const int64_t c = std::max<int64_t>(1, (n + g0 - 1) / g0);
  int64_t g = std::max<int64_t>(1, (n + c - 1) / c);
  if (g > 8) g = (g + 7) / 8 * 8;
  *chunk = (int)c;
  *grid = (int)g;
}

int64_t grid_cap(const opdhg_params* p) {
  return p->workgroups > 0 ? p->workgroups : kGridCap;
}

// Work-list sizes of a fixed set: evaluation tiles, step tiles, windowed chunks.
struct ListSizes {
  int64_t nlps = 0, nt = 0, na = 0, st = 0, sa = 0, vt = 0, va = 0, gt = 0, ga = 0;
  void add(const Prepared& P) {
    gt += (int64_t)P.win_t.seg_items();
    ga += (int64_t)P.win_a.seg_items();
    ++nlps;
    nt += (int64_t)P.tiles_t.size();
    na += (int64_t)P.tiles_a.size();
    st += (int64_t)P.stiles_t.size();
    sa += (int64_t)P.stiles_a.size();
    vt += (int64_t)P.win_t.chunks();
    va += (int64_t)P.win_a.chunks();
  }
};

static size_t tables_bytes(const ListSizes& z, int64_t cap);

size_t tables_bytes(const std::vector<const Prepared*>& preps, int64_t cap) {
  ListSizes z;
  for (const Prepared* P : preps) z.add(*P);
  return tables_bytes(z, cap);
}

static size_t tables_bytes(const ListSizes& z, int64_t cap) {
  const int64_t nt = z.nt, na = z.na, st = z.st, sa = z.sa, vt = z.vt, va = z.va;
  int g, c;
  size_t extra = 0;
  chunking(st, cap, &g, &c);
  extra += align_up(sizeof(WorkItem) * (size_t)g * c);
  chunking(sa, cap, &g, &c);
  extra += align_up(sizeof(WorkItem) * (size_t)g * c);
  auto padded = [](int64_t v) { return (size_t)(v > 8 ? (v + 7) / 8 * 8 : v); };
  extra += align_up(sizeof(WinItem) * padded(vt)) + align_up(sizeof(WinItem) * padded(va));
  extra += align_up(sizeof(SegItem) * padded(z.gt)) + align_up(sizeof(SegItem) * padded(z.ga));
  return tables_bytes(z.nlps, nt, na, cap) + extra;
}

size_t tables_bytes(int64_t nlps, int64_t nwork_t, int64_t nwork_a, int64_t cap) {
  int gt, ct, ga, ca;
  chunking(nwork_t, cap, &gt, &ct);
  chunking(nwork_a, cap, &ga, &ca);
  const size_t nl = (size_t)std::max<int64_t>(nlps, 1);
  return align_up(sizeof(LpDev) * nl) + align_up(sizeof(WorkItem) * (size_t)gt * ct) +
         align_up(sizeof(WorkItem) * (size_t)ga * ca) + align_up(sizeof(Counts)) +
         align_up(sizeof(Ctl) * nl);
}

// Order in which an LP's tiles enter the work list. Long rows (tiles of
// one row, relabelled to the front of the side) are spread evenly among the
// stream tiles, which keep their row order so consecutive chunks (one XCD)
// gather from nearby rows. Every row is finished inside its tile and all
// reductions are exact, so the order does not change any result.
static std::vector<int64_t> spread_long_tiles(const std::vector<Tile>& tiles) {
  std::vector<int64_t> longs, stream, order;
  for (size_t t = 0; t < tiles.size(); ++t) (tiles[t].lanes <= 0 ? longs : stream).push_back(t);
  order.reserve(tiles.size());
  const int64_t nl = (int64_t)longs.size(), ns = (int64_t)stream.size();
  int64_t il = 0;
  for (int64_t j = 0; j < ns; ++j) {
    // long tile il goes before stream tile floor(il * ns / nl)
    while (il < nl && il * ns <= j * nl) order.push_back(longs[il++]);
    order.push_back(stream[j]);
  }
  while (il < nl) order.push_back(longs[il++]);
  return order;
}

// Items of one side for all LPs, chunked: fills slot / first and each LP's
// slot count.
void side_items(std::vector<LpDev>& lps, const std::vector<const Prepared*>& preps, bool tside,
                int64_t cap, int* grid, int* chunk, std::vector<WorkItem>& out, bool step) {
  out.clear();
  std::vector<std::pair<int64_t, int64_t>> range(lps.size());
  for (size_t i = 0; i < lps.size(); ++i) {
    const Prepared& P = *preps[i];
    const std::vector<Tile>& tiles =
        step ? (tside ? P.stiles_t : P.stiles_a) : (tside ? P.tiles_t : P.tiles_a);
    range[i].first = (int64_t)out.size();
    for (int64_t t : spread_long_tiles(tiles)) {
      const Tile& tl = tiles[t];
      out.push_back(WorkItem{lps[i].ctl, (int32_t)i, (int32_t)t, tl.rb, tl.re, tl.s, tl.e,
                             tl.lanes, 0, tl.lanes < 0 ? tl.seg : -1, 0});
    }
    range[i].second = (int64_t)out.size();
  }
  const int64_t n = (int64_t)out.size();
  chunking(n, cap, grid, chunk);
  const int64_t C = *chunk;
  // The step kernels store every tile's partial sums in the slot of its
  // index within the LP's list: an LP's step partials, and the order the
  // decision adds them in, do not depend on how the set's items are chunked
  // over workgroups, so a packed or served LP adds exactly what its solo
  // solve adds. The evaluation kernels, whose double-double sums do not
  // depend on the order, store one partial per chunk touching the LP, in
  // the slot of the chunk's ordinal among those chunks.
  for (size_t i = 0; i < lps.size(); ++i) {
    const int64_t s = range[i].first, e = range[i].second;
    for (int64_t q = s; q < e; ++q) {
      out[q].slot = out[q].tile;
      out[q].first = q == s ? 1 : 0;
    }
    if (step) {
      (tside ? lps[i].nslot_st : lps[i].nslot_sa) = (int32_t)(e - s);
    } else {
      (tside ? lps[i].nslot_t : lps[i].nslot_a) =
          e > s ? (int32_t)((e - 1) / C - s / C + 1) : 0;
      (tside ? lps[i].item0_t : lps[i].item0_a) = (int32_t)s;
    }
  }
  const WorkItem pad{nullptr, -1, 0, 0, 0, 0, 0, 1, 0, -1, 0};
  out.resize((size_t)(*grid) * (*chunk), pad);
}

// Write the tables for a list of LPs into device memory at `dst` and point
// cfg at them.
int write_tables(uint8_t* dst, const std::vector<LpDev>& lps_in,
                 const std::vector<const Prepared*>& preps, int64_t cap, hipStream_t stream,
                 std::vector<uint8_t>& staging, LaunchCfg* cfg, int64_t* nwt, int64_t* nwa,
                 size_t capacity, bool fixed_launch) {
  std::vector<LpDev> lps(lps_in);
  std::vector<WorkItem> wt, wa, st, sa;
  std::vector<WinItem> vt, va;
  std::vector<SegItem> gt, ga;
  side_items(lps, preps, true, cap, &cfg->grid_t, &cfg->chunk_t, wt);
  side_items(lps, preps, false, cap, &cfg->grid_a, &cfg->chunk_a, wa);
  if (fixed_launch) {
    // the server's changing set: its step kernels run the evaluation lists
    // with the device-side chunking (no LP there has windowed chunks)
    for (size_t i = 0; i < lps.size(); ++i) {
      if (preps[i]->win_t.chunks() || preps[i]->win_a.chunks())
        return fail(OPDHG_ERR_INVALID_ARGUMENT, "windowed chunks in a shared launch set");
      lps[i].nslot_st = (int32_t)preps[i]->tiles_t.size();
      lps[i].nslot_sa = (int32_t)preps[i]->tiles_a.size();
    }
    cfg->sgrid_t = cfg->schunk_t = cfg->sgrid_a = cfg->schunk_a = 0;
    cfg->step_fixed = 0;
    cfg->evprod = 0;
  } else {
    side_items(lps, preps, true, cap, &cfg->sgrid_t, &cfg->schunk_t, st, true);
    side_items(lps, preps, false, cap, &cfg->sgrid_a, &cfg->schunk_a, sa, true);
    cfg->step_fixed = 1;
    int64_t nst = 0, nsa = 0;
    for (const Prepared* P : preps) {
      nst += (int64_t)P->stiles_t.size();
      nsa += (int64_t)P->stiles_a.size();
    }
    if (nst == 0) cfg->sgrid_t = 0;  // every row windowed: no tile launch
    if (nsa == 0) cfg->sgrid_a = 0;
    // 1: some LP has evaluation products; 2: every LP has them
    int with = 0;
    for (const LpDev& d : lps) with += d.evp_t0 != nullptr ? 1 : 0;
    cfg->evprod = with == 0 ? 0 : (with == (int)lps.size() ? 2 : 1);
    // windowed chunks take the partial slots after the LP's step tiles
    auto wins = [&](bool tside, std::vector<WinItem>& out) {
      std::vector<double> work;  // per chunk: entries, staged buckets and rows, in entry units
      for (size_t i = 0; i < lps.size(); ++i) {
        const WinPlan& W = tside ? preps[i]->win_t : preps[i]->win_a;
        int32_t& ns = tside ? lps[i].nslot_st : lps[i].nslot_sa;
        for (size_t c = 0; c < W.chunks(); ++c) {
          out.push_back(WinItem{lps[i].ctl, (int32_t)i, ns + (int32_t)c, W.r0[c], W.r1[c],
                                W.pass0[c], W.npass[c], W.nseg[c], W.seg0[c]});
          double w = 4.0 * (W.r1[c] - W.r0[c] + W.nseg[c]);  // a row's vectors: ~4 entries
          for (int32_t q = W.pass0[c]; q < W.pass0[c] + W.npass[c]; ++q) {
            for (int32_t sj = W.passes[q].s0; sj < W.passes[q].s1; ++sj)
              w += (double)kWinSlice * W.slices[sj].len;
            for (int32_t g = W.passes[q].range0; g < W.passes[q].range0 + W.passes[q].nrange; ++g)
              w += 0.5 * W.ranges[g].len;  // a staged float: half an entry's bytes
          }
          work.push_back(w);
        }
        ns += (int32_t)W.chunks();
      }
      if (out.size() <= 8) return;
      // The kernels give chunk c of a grid of 8L to XCD floor(c / L) (see
      // chunk_index), each XCD taking its L chunks in order. The list is
      // cut into 8 contiguous runs of about equal work (a packed set's LPs
      // differ in size; contiguity keeps an LP's chunks, which stage the
      // same vector, on one XCD's L2), each run ordered by decreasing work
      // so that the small chunks fill the end of the launch, and padded to
      // the longest run.
      const double total = std::accumulate(work.begin(), work.end(), 0.0);
      std::vector<std::vector<size_t>> run(8);
      double acc = 0.0;
      for (size_t c = 0; c < out.size(); ++c) {
        const int x = std::min(7, (int)((acc + 0.5 * work[c]) * 8.0 / total));
        run[x].push_back(c);
        acc += work[c];
      }
      size_t L = 0;
      for (auto& r : run) {
        std::stable_sort(r.begin(), r.end(), [&](size_t a, size_t b) { return work[a] > work[b]; });
        L = std::max(L, r.size());
      }
      std::vector<WinItem> lay;
      lay.reserve(8 * L);
      const WinItem pad{nullptr, -1, 0, 0, 0, 0, 0, 0, 0};
      for (auto& r : run) {
        for (size_t c : r) lay.push_back(out[c]);
        for (size_t k = r.size(); k < L; ++k) lay.push_back(pad);
      }
      out.swap(lay);
    };
    wins(true, vt);
    wins(false, va);
    // segmented long rows, kSegRows per workgroup, take the slots after the chunks
    auto segs = [&](bool tside, std::vector<SegItem>& out) {
      for (size_t i = 0; i < lps.size(); ++i) {
        const WinPlan& W = tside ? preps[i]->win_t : preps[i]->win_a;
        int32_t& ns = tside ? lps[i].nslot_st : lps[i].nslot_sa;
        const int32_t nrows = (int32_t)W.srow.size();
        for (int32_t s0 = 0, g = 0; s0 < nrows; s0 += kSegRows, ++g)
          out.push_back(SegItem{lps[i].ctl, (int32_t)i, ns + g, s0, std::min(nrows, s0 + kSegRows)});
        ns += (int32_t)W.seg_items();
      }
      if (out.size() > 8)
        while (out.size() % 8) out.push_back(SegItem{nullptr, -1, 0, 0, 0});
    };
    segs(true, gt);
    segs(false, ga);
  }
  cfg->nwin_t = (int)vt.size();
  cfg->nwin_a = (int)va.size();
  cfg->nseg_t = (int)gt.size();
  cfg->nseg_a = (int)ga.size();
  int64_t n_t = 0, n_a = 0;
  for (const Prepared* P : preps) {
    n_t += (int64_t)P->tiles_t.size();
    n_a += (int64_t)P->tiles_a.size();
  }
  const size_t nl = std::max<size_t>(lps.size(), 1);
  const size_t o_lps = 0;
  const size_t o_wt = o_lps + align_up(sizeof(LpDev) * nl);
  const size_t o_wa = o_wt + align_up(sizeof(WorkItem) * wt.size());
  const size_t o_st = o_wa + align_up(sizeof(WorkItem) * wa.size());
  const size_t o_sa = o_st + align_up(sizeof(WorkItem) * st.size());
  const size_t o_vt = o_sa + align_up(sizeof(WorkItem) * sa.size());
  const size_t o_va = o_vt + align_up(sizeof(WinItem) * vt.size());
  const size_t o_gt = o_va + align_up(sizeof(WinItem) * va.size());
  const size_t o_ga = o_gt + align_up(sizeof(SegItem) * gt.size());
  const size_t o_cn = o_ga + align_up(sizeof(SegItem) * ga.size());
  const size_t o_bd = o_cn + align_up(sizeof(Counts));
  const size_t total = o_bd + align_up(sizeof(Ctl) * nl);
  if (capacity && total > capacity)
    return fail(OPDHG_ERR_OVER_BUDGET, "launch tables need " + std::to_string(total) + " bytes");
  const size_t upload = o_bd;  // the board is written by the device
  staging.assign(upload, 0);
  if (!lps.empty()) std::memcpy(staging.data() + o_lps, lps.data(), sizeof(LpDev) * lps.size());
  std::memcpy(staging.data() + o_wt, wt.data(), sizeof(WorkItem) * wt.size());
  std::memcpy(staging.data() + o_wa, wa.data(), sizeof(WorkItem) * wa.size());
  if (!st.empty()) std::memcpy(staging.data() + o_st, st.data(), sizeof(WorkItem) * st.size());
  if (!sa.empty()) std::memcpy(staging.data() + o_sa, sa.data(), sizeof(WorkItem) * sa.size());
  if (!vt.empty()) std::memcpy(staging.data() + o_vt, vt.data(), sizeof(WinItem) * vt.size());
  if (!va.empty()) std::memcpy(staging.data() + o_va, va.data(), sizeof(WinItem) * va.size());
  if (!gt.empty()) std::memcpy(staging.data() + o_gt, gt.data(), sizeof(SegItem) * gt.size());
  if (!ga.empty()) std::memcpy(staging.data() + o_ga, ga.data(), sizeof(SegItem) * ga.size());
  Counts cn{(int32_t)n_t, (int32_t)n_a, (int32_t)lps.size(), 0,
            cfg->grid_t, cfg->chunk_t, cfg->grid_a, cfg->chunk_a, {0, 0}, {0, 0}};
  std::memcpy(staging.data() + o_cn, &cn, sizeof(cn));
  HIP_TRY(hipMemcpyAsync(dst, staging.data(), upload, hipMemcpyHostToDevice, stream));
  cfg->lps = reinterpret_cast<const LpDev*>(dst + o_lps);
  cfg->work_t = reinterpret_cast<const WorkItem*>(dst + o_wt);
  cfg->work_a = reinterpret_cast<const WorkItem*>(dst + o_wa);
  cfg->counts = reinterpret_cast<const Counts*>(dst + o_cn);
  cfg->step_t = fixed_launch ? cfg->work_t : reinterpret_cast<const WorkItem*>(dst + o_st);
  cfg->step_a = fixed_launch ? cfg->work_a : reinterpret_cast<const WorkItem*>(dst + o_sa);
  cfg->win_t = reinterpret_cast<const WinItem*>(dst + o_vt);
  cfg->win_a = reinterpret_cast<const WinItem*>(dst + o_va);
  cfg->seg_t = reinterpret_cast<const SegItem*>(dst + o_gt);
  cfg->seg_a = reinterpret_cast<const SegItem*>(dst + o_ga);
  cfg->board = reinterpret_cast<Ctl*>(dst + o_bd);
  if (!fixed_launch) {
    cfg->launch_t = cfg->grid_t;
    cfg->launch_a = cfg->grid_a;
    cfg->launch_ta = std::max(cfg->grid_t, cfg->grid_a);
    cfg->launch_lp = (int)std::max<size_t>(1, std::min<size_t>(lps.size(), kGridCap));
  }
  // one LP in a set that never changes: the decision record as uploaded
  cfg->solo = !fixed_launch && lps.size() == 1 ? 1 : 0;
  cfg->solo_rec = DecideRec{};
  if (cfg->solo) {
    const LpDev& d = lps[0];
    cfg->solo_rec = DecideRec{d.ctl, d.pow_ring, d.part_t, d.part_a,
                              d.ntiles_t, d.ntiles_a, d.nslot_st, d.nslot_sa,
                              d.s_lr, d.s_max_iter, d.s_phi, d.s_schedule,
                              d.s_normalize, d.s_eval_every, d.s_max_retries, d.s_flags};
  }
  *nwt = n_t;
  *nwa = n_a;
  return OPDHG_OK;
}

// The preparation kernels of a slot prepared on the device, then the
// diagonals (for unscaling results) and the first step size and primal
// weight back to the host.
static int device_prepare(uint8_t* base, const SlotLayout& L, Prepared& P, int prec,
                          hipStream_t stream) {
  const LpDev d = slot_pointers(base, L, P);
  PrepCfg c{};
  c.rp_a = d.rp_a;
  c.ci_a = d.ci_a;
  c.rp_t = d.rp_t;
  c.ci_t = d.ci_t;
  c.raw_a = reinterpret_cast<const double*>(base + L.raw_a);
  c.raw_t = reinterpret_cast<const double*>(base + L.raw_t);
  c.raw_b = reinterpret_cast<const double*>(base + L.raw_b);
  c.raw_c = reinterpret_cast<const double*>(base + L.raw_c);
  c.raw_l = reinterpret_cast<const double*>(base + L.raw_l);
  c.raw_u = reinterpret_cast<const double*>(base + L.raw_u);
  c.dr = reinterpret_cast<double*>(base + L.dr);
  c.dc = reinterpret_cast<double*>(base + L.dc);
  c.sr = reinterpret_cast<double*>(base + L.sr);
  c.sc = reinterpret_cast<double*>(base + L.sc);
  c.scr = reinterpret_cast<double*>(base + L.pscr);
  c.va_a = const_cast<void*>(d.va_a);
  c.va_t = const_cast<void*>(d.va_t);
  c.b = d.b;
  c.c = d.c;
  c.l = d.l;
  c.u = d.u;
  c.x0 = d.x[0];
  c.xa = d.xa;
  c.wval_t = const_cast<void*>(d.wval_t);
  c.wval_a = const_cast<void*>(d.wval_a);
  c.wsrc_t = P.win_t.chunks() ? reinterpret_cast<const int32_t*>(base + L.wsrc_t) : nullptr;
  c.wsrc_a = P.win_a.chunks() ? reinterpret_cast<const int32_t*>(base + L.wsrc_a) : nullptr;
  c.went_t = P.win_t.chunks() ? (int64_t)P.win_t.src.size() : 0;
  c.went_a = P.win_a.chunks() ? (int64_t)P.win_a.src.size() : 0;
  c.ctl = d.ctl;
  c.m = (int32_t)P.m;
  c.n = (int32_t)P.n;
  c.nlong_a = (int32_t)P.cend_a[0];
  c.nlong_t = (int32_t)P.cend_t[0];
  c.step_scale = P.prep_step_scale;
  c.power_tol = P.prep_power_tol;
  c.power_iters = P.prep_power_iters;
  int rc = 0;
  // Ruiz passes, the L2 pass, the Pock-Chambolle pass (Section 2), as on the host
  for (int it = 0; it < P.prep_ruiz && !rc; ++it)
    rc = prep_stats(c, stream, false, 0, 0.0) | prep_stats(c, stream, true, 0, 0.0) |
         prep_apply(c, stream);
  if (!rc && P.prep_l2)
    rc = prep_stats(c, stream, false, 2, 0.0) | prep_stats(c, stream, true, 2, 0.0) |
         prep_apply(c, stream);
  if (!rc && P.prep_beta >= 0.0)
    rc = prep_stats(c, stream, false, 1, P.prep_beta) |
         prep_stats(c, stream, true, 1, 2.0 - P.prep_beta) | prep_apply(c, stream);
  if (!rc) rc = prec == OPDHG_FP32 ? prep_finish<float>(c, stream) : prep_finish<double>(c, stream);
  // the constant step's eta0 from the power iteration (after the scalars,
  // whose eta0 it replaces)
  if (!rc && P.prep_power) rc = power_norm(c, stream);
  if (rc) return fail(OPDHG_ERR_DEVICE, std::string("preparation kernels: ") + device_error_string());
  std::vector<double> dr(P.m), dc(P.n), sc(2);
  if (P.m) HIP_TRY(hipMemcpyAsync(dr.data(), c.dr, 8 * P.m, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(dc.data(), c.dc, 8 * P.n, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(sc.data(), c.scr + 4 * kPrepGrid + 1, 16, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  P.dr.assign(P.m, 1.0);
  P.dc.assign(P.n, 1.0);
  for (int64_t i2 = 0; i2 < P.m; ++i2) P.dr[P.perm_a[i2]] = dr[i2];
  for (int64_t j2 = 0; j2 < P.n; ++j2) P.dc[P.perm_t[j2]] = dc[j2];
  P.eta0 = sc[0];
  P.omega0 = sc[1];
  return OPDHG_OK;
}

// Both CSR copies in device order, built on the device from the caller's
// arrays (already uploaded to the slot's staging).
static int device_structure(uint8_t* base, const SlotLayout& L, const Prepared& P,
                            hipStream_t stream) {
  StructCfg c{};
  c.src_rp = reinterpret_cast<const int64_t*>(base + L.st_rp);
  c.src_ci = reinterpret_cast<const int32_t*>(base + L.st_ci);
  c.src_val = reinterpret_cast<const double*>(base + L.st_val);
  c.perm_a = reinterpret_cast<const int32_t*>(base + L.st_perm_a);
  c.inv_a = reinterpret_cast<const int32_t*>(base + L.st_inv_a);
  c.inv_t = reinterpret_cast<const int32_t*>(base + L.st_inv_t);
  c.rp_a = reinterpret_cast<const int32_t*>(base + L.rp_a);
  c.rp_t = reinterpret_cast<const int32_t*>(base + L.rp_t);
  c.cur = reinterpret_cast<int32_t*>(base + L.st_cur);
  c.tmp_i = reinterpret_cast<int32_t*>(base + L.st_ti);
  c.tmp_k = reinterpret_cast<int32_t*>(base + L.st_tk);
  c.ci_a = reinterpret_cast<int32_t*>(base + L.ci_a);
  c.raw_a = reinterpret_cast<double*>(base + L.raw_a);
  c.ci_t = reinterpret_cast<int32_t*>(base + L.ci_t);
  c.raw_t = reinterpret_cast<double*>(base + L.raw_t);
  c.m = (int32_t)P.m;
  c.n = (int32_t)P.n;
  c.nlong_a = (int32_t)P.cend_a[0];
  c.nmed_t = (int32_t)P.cend_t[1];
  if (struct_build(c, stream))
    return fail(OPDHG_ERR_DEVICE, std::string("structure kernels: ") + device_error_string());
  return OPDHG_OK;
}

int upload_slot(uint8_t* base, const SlotLayout& L, Prepared& P, int prec, hipStream_t stream,
                SlotImage& img) {
  if (prec == OPDHG_FP32) slot_image<float>(L, P, img);
  else slot_image<double>(L, P, img);
  for (const auto& r : image_ranges(L, P))
    HIP_TRY(hipMemcpyAsync(base + r.first, img.data() + r.first, r.second - r.first,
                           hipMemcpyHostToDevice, stream));
  if (P.dstruct) {
    HIP_TRY(hipMemcpyAsync(base + L.st_rp, P.h_rp, 8 * (P.m + 1), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(base + L.st_ci, P.h_ci, 4 * P.nnz, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(base + L.st_val, P.h_val, 8 * P.nnz, hipMemcpyHostToDevice, stream));
    int rc = device_structure(base, L, P, stream);
    if (rc) return rc;
  }
  if (P.dprep) return device_prepare(base, L, P, prec, stream);
  return OPDHG_OK;
}

template <typename V>
static void get_vec(const uint8_t* src, size_t count, double* out) {
  const V* s = reinterpret_cast<const V*>(src);
  for (size_t i = 0; i < count; ++i) out[i] = (double)s[i];
}

// Download `count` elements of a V-typed device vector as doubles.
int download_vec(const void* dptr, size_t count, int prec, hipStream_t stream, double* out) {
  if (!out || count == 0) return OPDHG_OK;
  const size_t V = prec == OPDHG_FP32 ? 4 : 8;
  std::vector<uint8_t> tmp(count * V);
  HIP_TRY(hipMemcpyAsync(tmp.data(), dptr, count * V, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (prec == OPDHG_FP32) get_vec<float>(tmp.data(), count, out);
  else get_vec<double>(tmp.data(), count, out);
  return OPDHG_OK;
}

void fill_result(const Ctl& c, double seconds, opdhg_result* r) {
  std::memset(r, 0, sizeof(*r));
  r->status = c.status;
  r->which = c.which;
  r->iterations = c.k;
  r->attempts = c.attempts;
  r->restarts = c.restarts;
  // every final status comes from an evaluation (a numerical failure's too,
  // on the current iterate); a paused session has none yet
  const bool evaluated = c.status != kRunning;
  const double nan = std::numeric_limits<double>::quiet_NaN();
  r->primal_obj = evaluated ? c.out_pobj : nan;
  r->dual_obj = evaluated ? c.out_dobj : nan;
  r->rel_primal = evaluated ? c.out_relp : nan;
  r->rel_dual = evaluated ? c.out_reld : nan;
  r->rel_gap = evaluated ? c.out_relg : nan;
  r->rel_kkt = evaluated ? c.out_rel : nan;
  r->solve_seconds = seconds;
  r->eta = c.eta;
  r->omega = c.omega;
}

static const int32_t kOne = 1;

// Run a group's replays until every LP is done, k_target is reached, or
// the time limit passes. ctls points at `count` consecutive control blocks
// on the device only when the group is one LP; a batch passes its list.
int run_group(Group& grp, const std::vector<Ctl*>& d_ctls, std::vector<Ctl>& h_ctls,
              Ctl* pinned, int64_t k_target, double time_limit, double* elapsed) {
  const size_t cnt = d_ctls.size();
  auto t0 = std::chrono::steady_clock::now();
  int64_t last_progress = -1;
  int stalls = 0;
  // pause point
  for (size_t i = 0; i < cnt; ++i) {
    HIP_TRY(hipMemcpyAsync(pinned + i, d_ctls[i], sizeof(Ctl), hipMemcpyDeviceToHost, grp.stream));
  }
  HIP_TRY(hipStreamSynchronize(grp.stream));
  bool any_running = false;
  for (size_t i = 0; i < cnt; ++i) {
    h_ctls[i] = pinned[i];
    if (h_ctls[i].status == kRunning) {
      h_ctls[i].k_limit = k_target < 0 ? std::numeric_limits<int64_t>::max() : k_target;
      HIP_TRY(hipMemcpyAsync(&d_ctls[i]->k_limit, &h_ctls[i].k_limit, sizeof(int64_t),
                             hipMemcpyHostToDevice, grp.stream));
      any_running = true;
    }
  }
  HIP_TRY(hipStreamSynchronize(grp.stream));
  bool stop_sent = false;
  while (any_running) {
    int rc = grp.replay();
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(pinned, grp.cfg.board, sizeof(Ctl) * cnt, hipMemcpyDeviceToHost,
                           grp.stream));
    HIP_TRY(hipStreamSynchronize(grp.stream));
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    any_running = false;
    bool all_paused = true;
    int64_t progress = 0;
    for (size_t i = 0; i < cnt; ++i) {
      h_ctls[i] = pinned[i];
      const Ctl& c = h_ctls[i];
      progress += c.attempts + c.restarts + c.k;
      if (c.status == kRunning) {
        any_running = true;
        const bool paused = k_target >= 0 && c.k >= k_target;
        if (!paused) all_paused = false;
      }
    }
    if (!any_running || all_paused) break;
    if (progress == last_progress) {
      if (++stalls > 3) return fail(OPDHG_ERR_DEVICE, "device iteration made no progress");
    } else {
      stalls = 0;
    }
    last_progress = progress;
    if (!stop_sent && el > time_limit) {
      for (size_t i = 0; i < cnt; ++i) {
        if (h_ctls[i].status != kRunning) continue;
        HIP_TRY(hipMemcpyAsync(&d_ctls[i]->stop_request, &kOne, sizeof(kOne),
                               hipMemcpyHostToDevice, grp.stream));
        HIP_TRY(hipMemcpyAsync(&d_ctls[i]->need_eval, &kOne, sizeof(kOne),
                               hipMemcpyHostToDevice, grp.stream));
      }
      stop_sent = true;
    }
  }
  HIP_TRY(hipStreamSynchronize(grp.stream));
  *elapsed += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return OPDHG_OK;
}

}  // namespace opdhg

using namespace opdhg;

struct opdhg_session {
  SessionImpl impl;
};

extern "C" {

void opdhg_default_params(opdhg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->tol = 1e-4;
  p->max_iter = 100000;
  p->time_limit_s = 600.0;
  p->precision = OPDHG_FP64;
  p->schedule = OPDHG_SCHEDULE_ADAGRAD_DIAG;
  p->lr = 0.0;
  p->phi = 20;
  p->normalize = 1;
  p->precond_floor = 0.0;
  p->ruiz_iters = 10;
  p->pc_beta = 1.0;
  p->eval_every = 64;
  p->max_step_retries = 60;
  p->beta_suff = 0.2;
  p->beta_nec = 0.8;
  p->beta_art = 0.36;
  p->pw_smoothing = 0.5;
  p->step_growth = 0.6;
  p->step_reduction = 0.3;
  p->tile_nnz = 0;
  p->lanes = 0;
  p->workgroups = 0;
  p->step_rule = OPDHG_STEP_ADAPTIVE;
  p->restart_scheme = OPDHG_RESTART_ADAPTIVE;
  p->l2_rescale = 0;
  p->power_iters = 200;
  p->step_scale = 0.9;
  p->power_tol = 1e-7;
  p->step_norm = OPDHG_STEP_NORM_PLAIN;
  p->windows = OPDHG_WINDOWS_AUTO;
  p->window_buckets = 0;
  p->window_rows = 0;
  p->prep = OPDHG_PREP_AUTO;
  p->eval_slots = 0;
}

int opdhg_validate(const opdhg_lp* lp) { return validate_lp(lp); }

int opdhg_workspace_bytes(const opdhg_lp* lp, const opdhg_params* p, size_t* bytes) {
  int rc = validate_lp(lp);
  if (rc) return rc;
  if ((rc = validate_params(p))) return rc;
  if (!bytes) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bytes is NULL");
  Prepared P;
  if ((rc = prepare(lp, p, P, true))) return rc;
  SlotLayout L = slot_layout(P, p->precision);
  *bytes = L.total + tables_bytes({&P}, grid_cap(p));
  return OPDHG_OK;
}

int opdhg_rescale(const opdhg_lp* lp, const opdhg_params* p, double* scaled_val, double* d_row,
                  double* d_col) {
  int rc = validate_lp(lp);
  if (rc) return rc;
  if ((rc = validate_params(p))) return rc;
  std::vector<double> sval, dr, dc;
  rescale_host(lp, p, sval, dr, dc);
  if (scaled_val) std::copy(sval.begin(), sval.end(), scaled_val);
  if (d_row) std::copy(dr.begin(), dr.end(), d_row);
  if (d_col) std::copy(dc.begin(), dc.end(), d_col);
  return OPDHG_OK;
}

int opdhg_spectral_norm(const opdhg_lp* lp, const opdhg_params* p, double* norm_out) {
  int rc = validate_lp(lp);
  if (rc) return rc;
  if ((rc = validate_params(p))) return rc;
  if (!norm_out) return fail(OPDHG_ERR_INVALID_ARGUMENT, "norm_out is NULL");
  ColIndex C;
  build_col_index(lp, C);
  std::vector<double> sval, dr, dc;
  rescale_with(lp, C, p->ruiz_iters, p->l2_rescale != 0, p->pc_beta, sval, dr, dc);
  *norm_out = spectral_norm_with(lp, C, sval, p->power_iters, p->power_tol);
  return OPDHG_OK;
}

}  // extern "C"

namespace opdhg {

// Session set-up shared by opdhg_session_create and the allocation-free
// solve: validation, preparation, upload, launch tables, the first
// products and the launch sequence. need_out (if set) receives the device
// bytes the LP needs, also when the workspace is too small.
}  // namespace opdhg

// One LP prepared for a session: validation, structure, tiling, windows
// (and the scaled data when the host prepares it), its slot layout and the
// exact workspace bytes.
struct opdhg_prepared {
  opdhg_params p{};
  Prepared P;
  SlotLayout L;
  size_t need = 0;
  bool used = false;
};

namespace opdhg {

static int prepared_make(const opdhg_lp* lp, const opdhg_params* p, opdhg_prepared& pr) {
  int rc = validate_lp(lp);
  if (rc) return rc;
  if ((rc = validate_params(p))) return rc;
  pr.p = *p;
  if ((rc = prepare(lp, p, pr.P, false))) return rc;
  pr.L = slot_layout(pr.P, p->precision);
  pr.need = pr.L.total + tables_bytes({&pr.P}, grid_cap(p));
  return OPDHG_OK;
}

static int session_from_prepared(opdhg_prepared& pr, void* d_workspace, size_t workspace_bytes,
                                 void* hip_stream, bool direct, opdhg_session** out) {
  if (!out) return fail(OPDHG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (pr.used) return fail(OPDHG_ERR_INVALID_ARGUMENT, "prepared LP was used already");
  if (!d_workspace) return fail(OPDHG_ERR_INVALID_ARGUMENT, "workspace is NULL");
  const opdhg_params* p = &pr.p;
  const size_t need = pr.need;
  if (workspace_bytes < need)
    return fail(OPDHG_ERR_WORKSPACE_TOO_SMALL,
                "workspace needs " + std::to_string(need) + " bytes");
  int rc = OPDHG_OK;
  auto s = std::make_unique<opdhg_session>();
  SessionImpl& S = s->impl;
  pr.used = true;  // the prepared data moves into the session
  S.P = std::move(pr.P);
  S.L = pr.L;
  S.ws = static_cast<uint8_t*>(d_workspace);
  S.time_limit = p->time_limit_s;
  S.direct = direct;
  if ((rc = S.grp.init(hip_stream, p->precision, direct))) return rc;
  S.grp.mid_every = mid_eval_every(p, 1);
  SlotImage img;
  if ((rc = upload_slot(S.ws, S.L, S.P, p->precision, S.grp.stream, img))) return rc;
  S.lpd = slot_pointers(S.ws, S.L, S.P);
  S.d_tables = S.ws + S.L.total;
  std::vector<uint8_t> staging;
  int64_t nwt = 0, nwa = 0;
  if ((rc = write_tables(S.d_tables, {S.lpd}, {&S.P}, grid_cap(p), S.grp.stream, staging,
                         &S.grp.cfg, &nwt, &nwa)))
    return rc;
  if ((rc = S.grp.launch_init())) return fail(OPDHG_ERR_DEVICE, device_error_string());
  HIP_TRY(hipStreamSynchronize(S.grp.stream));
  if ((rc = S.grp.capture(std::max(1, p->eval_every)))) return rc;
  if (direct) S.h_ctl = &S.h_ctl_local;
  else HIP_TRY(hipHostMalloc((void**)&S.h_ctl, sizeof(Ctl), hipHostMallocDefault));
  *out = s.release();
  return OPDHG_OK;
}

int session_create(const opdhg_lp* lp, const opdhg_params* p, void* d_workspace,
                   size_t workspace_bytes, void* hip_stream, bool direct, opdhg_session** out,
                   size_t* need_out) {
  if (!out) return fail(OPDHG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!d_workspace) {
    int rc = validate_lp(lp);
    if (!rc) rc = validate_params(p);
    return rc ? rc : fail(OPDHG_ERR_INVALID_ARGUMENT, "workspace is NULL");
  }
  opdhg_prepared pr;
  int rc = prepared_make(lp, p, pr);
  if (rc) return rc;
  if (need_out) *need_out = pr.need;
  return session_from_prepared(pr, d_workspace, workspace_bytes, hip_stream, direct, out);
}

}  // namespace opdhg

extern "C" {

int opdhg_session_create(const opdhg_lp* lp, const opdhg_params* p, void* d_workspace,
                         size_t workspace_bytes, void* hip_stream, opdhg_session** out) {
  return session_create(lp, p, d_workspace, workspace_bytes, hip_stream, false, out, nullptr);
}

int opdhg_prepare(const opdhg_lp* lp, const opdhg_params* p, opdhg_prepared** out) {
  if (!out) return fail(OPDHG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  auto pr = std::make_unique<opdhg_prepared>();
  int rc = prepared_make(lp, p, *pr);
  if (rc) return rc;
  *out = pr.release();
  return OPDHG_OK;
}

int opdhg_prepared_bytes(const opdhg_prepared* pr, size_t* bytes) {
  if (!pr || !bytes) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  *bytes = pr->need;
  return OPDHG_OK;
}

int opdhg_session_create_prepared(opdhg_prepared* pr, void* d_workspace, size_t workspace_bytes,
                                  void* hip_stream, opdhg_session** out) {
  if (!pr) return fail(OPDHG_ERR_INVALID_ARGUMENT, "prepared LP is NULL");
  return session_from_prepared(*pr, d_workspace, workspace_bytes, hip_stream, false, out);
}

void opdhg_prepared_destroy(opdhg_prepared* pr) { delete pr; }

int opdhg_session_run(opdhg_session* s, int64_t k_target) {
  if (!s) return fail(OPDHG_ERR_INVALID_ARGUMENT, "session is NULL");
  SessionImpl& S = s->impl;
  std::vector<Ctl*> ctls = {S.lpd.ctl};
  std::vector<Ctl> h(1);
  return run_group(S.grp, ctls, h, S.h_ctl, k_target, S.time_limit - S.elapsed, &S.elapsed);
}

int opdhg_session_replay(opdhg_session* s, int replays) {
  if (!s || replays < 0) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  SessionImpl& S = s->impl;
  const int64_t unlimited = std::numeric_limits<int64_t>::max();
  HIP_TRY(hipMemcpyAsync(&S.lpd.ctl->k_limit, &unlimited, sizeof(unlimited),
                         hipMemcpyHostToDevice, S.grp.stream));
  HIP_TRY(hipStreamSynchronize(S.grp.stream));
  auto t0 = std::chrono::steady_clock::now();
  for (int r = 0; r < replays; ++r) {
    int rc = S.grp.replay();
    if (rc) return rc;
  }
  HIP_TRY(hipStreamSynchronize(S.grp.stream));
  S.elapsed += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return OPDHG_OK;
}

int opdhg_session_state(opdhg_session* s, double* x, double* y, double* T, double* Sigma,
                        opdhg_state* st) {
  if (!s) return fail(OPDHG_ERR_INVALID_ARGUMENT, "session is NULL");
  SessionImpl& S = s->impl;
  Ctl c;
  HIP_TRY(hipMemcpyAsync(S.h_ctl, S.lpd.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, S.grp.stream));
  HIP_TRY(hipStreamSynchronize(S.grp.stream));
  c = *S.h_ctl;
  if (c.learn_pending) {
    // apply the accepted learner step now (the next attempt would have)
    if (S.grp.launch_learn_flush()) return fail(OPDHG_ERR_DEVICE, device_error_string());
    static const int32_t zero = 0;
    HIP_TRY(hipMemcpyAsync(&S.lpd.ctl->learn_pending, &zero, sizeof(zero),
                           hipMemcpyHostToDevice, S.grp.stream));
    HIP_TRY(hipStreamSynchronize(S.grp.stream));
    c.learn_pending = 0;
  }
  int rc = 0;
  const int prec = S.grp.prec;
  std::vector<double> tn(S.P.n), tm(S.P.m);
  struct {
    const void* src;
    double* dst;
    bool primal;
  } outs[4] = {{S.lpd.x[c.cur], x, true}, {S.lpd.y[c.cur], y, false},
               {S.lpd.T, T, true}, {S.lpd.S, Sigma, false}};
  for (auto& o : outs) {
    if (!o.dst) continue;
    std::vector<double>& tmp = o.primal ? tn : tm;
    if ((rc = download_vec(o.src, tmp.size(), prec, S.grp.stream, tmp.data()))) return rc;
    unpermute(tmp.data(), o.primal ? S.P.perm_t : S.P.perm_a, nullptr, o.dst);
  }
  if (st) {
    st->k = c.k;
    st->t = c.t;
    st->attempts = c.attempts;
    st->restarts = c.restarts;
    st->status = c.status;
    st->need_eval = c.need_eval;
    st->eta = c.eta;
    st->omega = c.omega;
    st->w = c.w;
  }
  return OPDHG_OK;
}

int opdhg_session_result(opdhg_session* s, double* x_out, double* y_out, opdhg_result* res) {
  if (!s) return fail(OPDHG_ERR_INVALID_ARGUMENT, "session is NULL");
  SessionImpl& S = s->impl;
  HIP_TRY(hipMemcpyAsync(S.h_ctl, S.lpd.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, S.grp.stream));
  HIP_TRY(hipStreamSynchronize(S.grp.stream));
  const Ctl c = *S.h_ctl;
  int rc = 0;
  const int prec = S.grp.prec;
  if (x_out) {
    std::vector<double> tmp(S.P.n);
    if ((rc = download_vec(S.lpd.x[c.cur], S.P.n, prec, S.grp.stream, tmp.data()))) return rc;
    unpermute(tmp.data(), S.P.perm_t, S.P.dc.data(), x_out);
  }
  if (y_out && S.P.m) {
    std::vector<double> tmp(S.P.m);
    if ((rc = download_vec(S.lpd.y[c.cur], S.P.m, prec, S.grp.stream, tmp.data()))) return rc;
    unpermute(tmp.data(), S.P.perm_a, S.P.dr.data(), y_out);
  }
  if (res) fill_result(c, S.elapsed, res);
  return OPDHG_OK;
}

// Average time of reps back-to-back launches of one forced kernel.
static int time_forced(SessionImpl& S, int reps, bool primal, double* avg_ms) {
  auto launch = [&] { return primal ? S.grp.launch_primal_forced() : S.grp.launch_dual_forced(); };
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = launch();  // warm-up
  HIP_TRY(hipEventRecord(e0, S.grp.stream));
  for (int r = 0; r < reps && rc == 0; ++r) rc = launch();
  HIP_TRY(hipEventRecord(e1, S.grp.stream));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return fail(OPDHG_ERR_DEVICE, device_error_string());
  *avg_ms = ms / reps;
  return OPDHG_OK;
}

int opdhg_session_time_primal_kernel(opdhg_session* s, int reps, double* avg_ms) {
  if (!s || reps < 1 || !avg_ms) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  return time_forced(s->impl, reps, true, avg_ms);
}

int opdhg_session_time_kernels(opdhg_session* s, int reps, double* primal_ms, double* dual_ms) {
  if (!s || reps < 1 || !primal_ms || !dual_ms)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  int rc = time_forced(s->impl, reps, true, primal_ms);
  if (!rc) rc = time_forced(s->impl, reps, false, dual_ms);
  return rc;
}

void opdhg_session_destroy(opdhg_session* s) {
  if (!s) return;
  SessionImpl& S = s->impl;
  if (S.grp.stream || S.grp.cap_stream) (void)hipStreamSynchronize(S.grp.stream);
  S.grp.release();
  if (S.h_ctl && !S.direct) (void)hipHostFree(S.h_ctl);
  delete s;
}

int opdhg_solve(const opdhg_lp* lp, const opdhg_params* p, void* d_workspace,
                size_t workspace_bytes, void* hip_stream, double* x_out, double* y_out,
                opdhg_result* res) {
  opdhg_session* s = nullptr;
  int rc = opdhg_session_create(lp, p, d_workspace, workspace_bytes, hip_stream, &s);
  if (rc) return rc;
  rc = opdhg_session_run(s, -1);
  if (!rc) rc = opdhg_session_result(s, x_out, y_out, res);
  opdhg_session_destroy(s);
  return rc;
}

// Parameters a packed set is prepared with. Under OPDHG_PREP_AUTO a set
// whose nonzeros reach the device-preparation threshold in total is
// prepared on the device, where that gives the host's numbers bit for bit
// (Pock-Chambolle exponent 1 or none), so every LP of the set still equals
// its solo solve. The workspace sizing takes the same decision.
static opdhg_params batch_params(int count, const opdhg_lp* lps, const opdhg_params* p) {
  opdhg_params q = *p;
  if (p->prep != OPDHG_PREP_AUTO) return q;
  if (!(p->pc_beta == 1.0 || p->pc_beta < 0.0)) return q;
  int64_t total = 0;
  for (int i = 0; i < count; ++i) total += lps[i].nnz;
  if (total >= kDevicePrepNnz) q.prep = OPDHG_PREP_DEVICE;
  return q;
}

int opdhg_batch_workspace_bytes(int count, const opdhg_lp* lps, const opdhg_params* p_in,
                                size_t* bytes) {
  if (count < 0 || (count > 0 && !lps) || !bytes)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  int rc = validate_params(p_in);
  if (rc) return rc;
  const opdhg_params pb = batch_params(count, lps, p_in);
  const opdhg_params* p = &pb;
  // the LPs' structures are sized on up to 16 host threads
  std::vector<Prepared> P(count);
  std::vector<int> rcs(count, OPDHG_OK);
  std::vector<std::string> msgs(count);
  std::atomic<int> next{0};
  auto work = [&] {
    for (int i = next++; i < count; i = next++) {
      int r = validate_lp(&lps[i]);
      if (!r) r = prepare(&lps[i], p, P[i], true);
      if (r) {
        rcs[i] = r;
        msgs[i] = opdhg_last_error();
      }
    }
  };
  const int nth = std::max(1, std::min({count, host_threads(), 16}));
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  size_t total = 0;
  ListSizes z;
  for (int i = 0; i < count; ++i) {
    if (rcs[i]) return fail(rcs[i], "LP " + std::to_string(i) + ": " + msgs[i]);
    total += slot_layout(P[i], p->precision).total;
    z.add(P[i]);
  }
  *bytes = total + tables_bytes(z, grid_cap(p));
  return OPDHG_OK;
}

}  // extern "C"

// A packed set prepared once: the LPs' validation, structure, tiling and
// windows (and, with host preparation, their scaled data), the slot layouts
// and the exact workspace bytes.
struct opdhg_batch {
  int count = 0;
  std::vector<opdhg_lp> lps;  // the caller's arrays, borrowed until the solve
  opdhg_params p{};
  std::vector<Prepared> P;
  std::vector<SlotLayout> L;
  std::vector<size_t> offs;
  size_t off = 0, need = 0;
};

static int batch_prepare(int count, const opdhg_lp* lps, const opdhg_params* p_in,
                         opdhg_batch& B) {
  if (count < 0 || (count > 0 && !lps)) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  int rc = validate_params(p_in);
  if (rc) return rc;
  B.count = count;
  B.lps.assign(lps, lps + count);
  B.p = batch_params(count, lps, p_in);
  const opdhg_params* p = &B.p;
  std::vector<Prepared>& P = B.P;
  std::vector<SlotLayout>& L = B.L;
  P.assign(count, Prepared());
  L.assign(count, SlotLayout());
  B.offs.assign(count, 0);
  // validation, rescaling, transposes and tiling of each LP are independent
  std::vector<int> rcs(count, OPDHG_OK);
  std::vector<std::string> msgs(count);
  std::atomic<int> next{0};
  auto work = [&] {
    for (int i = next++; i < count; i = next++) {
      int r = validate_lp(&lps[i]);
      if (!r) r = prepare(&lps[i], p, P[i], false);
      if (r) {
        rcs[i] = r;
        msgs[i] = opdhg_last_error();
      }
    }
  };
  const int nth = std::max(1, std::min({count, host_threads(), 16}));
  std::vector<std::thread> pool;
  for (int t = 1; t < nth; ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    if (rcs[i]) return fail(rcs[i], "LP " + std::to_string(i) + ": " + msgs[i]);
    L[i] = slot_layout(P[i], p->precision);
    B.offs[i] = off;
    off += L[i].total;
  }
  ListSizes z;
  for (int i = 0; i < count; ++i) z.add(P[i]);
  B.off = off;
  B.need = off + tables_bytes(z, grid_cap(p));
  return OPDHG_OK;
}

static int batch_solve(opdhg_batch& B, void* d_workspace, size_t workspace_bytes,
                       void* hip_stream, double* const* x_out, double* const* y_out,
                       opdhg_result* res) {
  const int count = B.count;
  if (count == 0) return OPDHG_OK;
  if (!d_workspace || !res) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  int rc = OPDHG_OK;
  const opdhg_params* p = &B.p;
  std::vector<Prepared>& P = B.P;
  std::vector<SlotLayout>& L = B.L;
  std::vector<size_t>& offs = B.offs;
  const size_t off = B.off;
  std::vector<std::string> msgs(count);
  const size_t need = B.need;
  if (workspace_bytes < need)
    return fail(OPDHG_ERR_WORKSPACE_TOO_SMALL, "workspace needs " + std::to_string(need) + " bytes");
  uint8_t* ws = static_cast<uint8_t*>(d_workspace);
  Group grp;
  if ((rc = grp.init(hip_stream, p->precision))) return rc;
  grp.mid_every = mid_eval_every(p, count);
  std::vector<LpDev> lpd(count);
  {
    // The slots are filled and copied by several threads, each with its own
    // image and stream (default priority): one thread's copy overlaps the
    // others' fills. Each waits for its copy before it reuses its image, and
    // all have finished before the set's launches are enqueued.
    std::atomic<int> nx{0};
    std::vector<int> urc(count, OPDHG_OK);
    auto up = [&] {
      hipStream_t s = nullptr;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        for (int i = nx++; i < count; i = nx++) {
          urc[i] = OPDHG_ERR_DEVICE;
          msgs[i] = "hipStreamCreateWithFlags failed";
        }
        return;
      }
      SlotImage im;
      for (int i = nx++; i < count; i = nx++) {
        int r = upload_slot(ws + offs[i], L[i], P[i], p->precision, s, im);
        if (!r && hipStreamSynchronize(s) != hipSuccess) r = fail(OPDHG_ERR_DEVICE, "upload failed");
        if (r) {
          urc[i] = r;
          msgs[i] = opdhg_last_error();
        }
      }
      (void)hipStreamDestroy(s);
    };
    const int nup = std::max(1, std::min({count, host_threads(), 8}));
    std::vector<std::thread> ups;
    for (int t = 1; t < nup; ++t) ups.emplace_back(up);
    up();
    for (auto& t : ups) t.join();
    for (int i = 0; i < count; ++i) {
      if (urc[i]) {
        grp.release();
        return fail(urc[i], "LP " + std::to_string(i) + ": " + msgs[i]);
      }
      lpd[i] = slot_pointers(ws + offs[i], L[i], P[i]);
    }
  }
  std::vector<uint8_t> staging;
  int64_t wt = 0, wa = 0;
  std::vector<const Prepared*> preps(count);
  for (int i = 0; i < count; ++i) preps[i] = &P[i];
  if ((rc = write_tables(ws + off, lpd, preps, grid_cap(p), grp.stream, staging, &grp.cfg, &wt,
                         &wa))) {
    grp.release();
    return rc;
  }
  if (grp.launch_init()) {
    grp.release();
    return fail(OPDHG_ERR_DEVICE, device_error_string());
  }
  (void)hipStreamSynchronize(grp.stream);
  if ((rc = grp.capture(std::max(1, p->eval_every)))) {
    grp.release();
    return rc;
  }
  Ctl* pinned = nullptr;
  if (hipHostMalloc((void**)&pinned, sizeof(Ctl) * count, hipHostMallocDefault) != hipSuccess) {
    grp.release();
    return fail(OPDHG_ERR_DEVICE, "pinned host allocation failed");
  }
  std::vector<Ctl*> ctls(count);
  for (int i = 0; i < count; ++i) ctls[i] = lpd[i].ctl;
  std::vector<Ctl> h(count);
  double elapsed = 0.0;
  rc = run_group(grp, ctls, h, pinned, -1, p->time_limit_s, &elapsed);
  for (int i = 0; i < count && rc == 0; ++i) {
    const Ctl& c = h[i];
    if (x_out && x_out[i]) {
      std::vector<double> tmp(P[i].n);
      if ((rc = download_vec(lpd[i].x[c.cur], P[i].n, p->precision, grp.stream, tmp.data())))
        break;
      unpermute(tmp.data(), P[i].perm_t, P[i].dc.data(), x_out[i]);
    }
    if (y_out && y_out[i] && P[i].m) {
      std::vector<double> tmp(P[i].m);
      if ((rc = download_vec(lpd[i].y[c.cur], P[i].m, p->precision, grp.stream, tmp.data())))
        break;
      unpermute(tmp.data(), P[i].perm_a, P[i].dr.data(), y_out[i]);
    }
    fill_result(c, elapsed, &res[i]);
  }
  (void)hipHostFree(pinned);
  grp.release();
  return rc;
}

extern "C" {

int opdhg_solve_batch(int count, const opdhg_lp* lps, const opdhg_params* p_in,
                      void* d_workspace, size_t workspace_bytes, void* hip_stream,
                      double* const* x_out, double* const* y_out, opdhg_result* res) {
  if (count < 0 || (count > 0 && (!lps || !res)) || !d_workspace)
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  opdhg_batch B;
  int rc = batch_prepare(count, lps, p_in, B);
  if (rc) return rc;
  return batch_solve(B, d_workspace, workspace_bytes, hip_stream, x_out, y_out, res);
}

int opdhg_batch_prepare(int count, const opdhg_lp* lps, const opdhg_params* p,
                        opdhg_batch** out) {
  if (!out) return fail(OPDHG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  auto B = std::make_unique<opdhg_batch>();
  int rc = batch_prepare(count, lps, p, *B);
  if (rc) return rc;
  *out = B.release();
  return OPDHG_OK;
}

int opdhg_batch_bytes(const opdhg_batch* b, size_t* bytes) {
  if (!b || !bytes) return fail(OPDHG_ERR_INVALID_ARGUMENT, "bad arguments");
  *bytes = b->need;
  return OPDHG_OK;
}

int opdhg_batch_solve(opdhg_batch* b, void* d_workspace, size_t workspace_bytes,
                      void* hip_stream, double* const* x_out, double* const* y_out,
                      opdhg_result* res) {
  if (!b) return fail(OPDHG_ERR_INVALID_ARGUMENT, "batch is NULL");
  if (b->count > 0 && b->P.empty())
    return fail(OPDHG_ERR_INVALID_ARGUMENT, "batch was solved already");
  const int rc = batch_solve(*b, d_workspace, workspace_bytes, hip_stream, x_out, y_out, res);
  b->P.clear();  // the prepared data went into the workspace
  return rc;
}

void opdhg_batch_destroy(opdhg_batch* b) { delete b; }

const char* opdhg_last_error(void) { return g_err.c_str(); }

const char* opdhg_status_name(int status) {
  switch (status) {
    case OPDHG_STATUS_OPTIMAL: return "OPTIMAL";
    case OPDHG_STATUS_ITERATION_LIMIT: return "ITERATION_LIMIT";
    case OPDHG_STATUS_TIME_LIMIT: return "TIME_LIMIT";
    case OPDHG_STATUS_NUMERICAL_ERROR: return "NUMERICAL_ERROR";
    case OPDHG_STATUS_RUNNING: return "RUNNING";
    default: return "UNKNOWN";
  }
}

const char* opdhg_build_info(void) { return "opdhg 0.1 gfx950"; }

}  // extern "C"
