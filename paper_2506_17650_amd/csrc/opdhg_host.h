// Host-side structures of the opdhg library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <utility>
#include <string>
#include <vector>

#include "opdhg.h"
#include "opdhg_internal.h"

namespace opdhg {

int fail(int code, const std::string& msg);
int fail_hip(hipError_t e, const char* what);
int host_threads();  // hardware threads of the host (at least 1)

// Return the HIP error of expr as OPDHG_ERR_DEVICE (with a message).
#define HIP_TRY(expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return fail_hip(e_, #expr);  \
  } while (0)
int validate_lp(const opdhg_lp* lp);
int validate_params(const opdhg_params* p);

// Allocator whose default construction leaves trivially constructible
// elements uninitialised: resize() then writes nothing, and the threads
// that fill an array touch its pages themselves, in parallel, instead of
// one thread zero-filling (and faulting in) every page first.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U>&) {}
  template <typename U>
  void construct(U* p) noexcept {
    ::new ((void*)p) U;
  }
  template <typename U, typename... A>
  void construct(U* p, A&&... a) {
    ::new ((void*)p) U(std::forward<A>(a)...);
  }
};
// The nonzero-sized host arrays of a prepared LP.
template <typename T>
using HostArray = std::vector<T, NoInitAlloc<T>>;
// Host image of an LP slot (filled in parallel, then copied to the device).
using SlotImage = HostArray<uint8_t>;

// Windowed chunks of one CSR side (see WinItem): rows and passes of each
// chunk, the passes' slices and LDS ranges, the slices (entry offset and
// length, and the chunk-local row of each lane), and the entries in slice
// order (window-local column) with the device-order CSR position of each
// (-1 for padding).
struct WinPlan {
  std::vector<int32_t> r0, r1, pass0, npass;
  std::vector<int32_t> nseg, seg0;  // per chunk: segments after its rows, first segment id
  std::vector<WinPass> passes;
  std::vector<WinRange> ranges;
  std::vector<WinSlice> slices;
  HostArray<uint16_t> lane;  // kWinSlice per slice
  HostArray<uint16_t> col;   // filled by the planning threads (not zeroed first)
  HostArray<int64_t> src;
  // long rows split into segments: the rows (device order), and per row the
  // ids of its segments' partials in order (CSR over srow). The windowed
  // plan's segments come first (nsrow_win rows, nsegs_win partials); rows
  // that stay in tiles and are longer than kSplitNnz follow, as pieces of
  // kPieceNnz nonzeros (step_tiles rebuilds that part for each tiling).
  std::vector<int32_t> srow, sptr, sids;
  int32_t nsegs = 0;
  size_t nsrow_win = 0;
  int32_t nsegs_win = 0;
  size_t chunks() const { return r0.size(); }
  // workgroups of the finishing kernel (kSegRows segmented rows each)
  size_t seg_items() const { return (srow.size() + kSegRows - 1) / kSegRows; }
};

// LPs of at least this many nonzeros are prepared on the device under
// OPDHG_PREP_AUTO.
constexpr int64_t kDevicePrepNnz = int64_t(1) << 20;

// An LP after validation, rescaling and transposition, in FP64 on the host.
// Arrays marked "device order" follow the relabelling by row class:
// device row i of A is original row perm_a[i], device variable j is
// original variable perm_t[j].
struct Prepared {
  int64_t m = 0, n = 0, nnz = 0;
  std::vector<int32_t> perm_a, perm_t;
  std::vector<int32_t> rp_a, rp_t;  // device order
  HostArray<int32_t> ci_a, ci_t;    // device order
  HostArray<double> va_a, va_t;     // device order
  std::vector<double> b, c, l, u, x0;           // device order
  std::vector<double> dr_dev, dc_dev;           // device order
  std::vector<double> dr, dc;                   // original order (unscaling)
  std::vector<int8_t> sense, bfin;              // device order
  std::vector<Tile> tiles_a, tiles_t;    // every row (evaluations, initial products)
  std::vector<Tile> stiles_a, stiles_t;  // rows the step kernels take in tiles (not windowed)
  WinPlan win_a, win_t;                  // windowed rows of the step kernels (FP32)
  int64_t cend_a[3] = {0, 0, 0}, cend_t[3] = {0, 0, 0};  // ends of the row classes
  std::vector<double> pow_tab;  // step-rule factors, 2 * kPowTab
  DevParams prm;
  double eta0 = 1.0, omega0 = 1.0;
  // device-side preparation: the host keeps the structure and sends the
  // unscaled values in device order; dr, dc, eta0 and omega0 come back
  // after the preparation kernels
  bool dprep = false;
  int prep_ruiz = 0;
  bool prep_l2 = false;
  double prep_beta = -1.0;
  // the constant step: the power iteration's limits and eta0's scale
  bool prep_power = false;
  int prep_power_iters = 0;
  double prep_power_tol = 0.0, prep_step_scale = 1.0;
  HostArray<double> raw_a, raw_t;
  std::vector<double> raw_b, raw_c, raw_l, raw_u;
  // device-side structure (with dprep, no windows): both CSR copies are
  // built on the device from the caller's arrays, which must stay valid
  // until the slot is uploaded; the host keeps lengths, orders and tiles
  bool dstruct = false;
  const int64_t* h_rp = nullptr;
  const int32_t* h_ci = nullptr;
  const double* h_val = nullptr;
  std::vector<int32_t> inv_a, inv_t;
  // partial slots per side: evaluation tiles, or step tiles plus windowed chunks
  int64_t part_stride_t() const {
    return (int64_t)std::max(tiles_t.size(),
                             stiles_t.size() + win_t.chunks() + win_t.seg_items());
  }
  int64_t part_stride_a() const {
    return (int64_t)std::max(tiles_a.size(),
                             stiles_a.size() + win_a.chunks() + win_a.seg_items());
  }
};

// Byte offsets of every array of one LP slot in the workspace.
struct SlotLayout {
  static constexpr int kNVecN = 11;  // c l u T Hp Gp x0 x1 xs0 xs1 xa
  static constexpr int kNVecM = 12;  // b S Hd Gd y0 y1 ys0 ys1 ya Ax0 Ax1 Axa
  size_t ctl = 0, prm = 0, tiles_a = 0, tiles_t = 0, part_a = 0, part_t = 0, pow_tab = 0;
  size_t pow_ring = 0;
  size_t rp_a = 0, ci_a = 0, va_a = 0, rp_t = 0, ci_t = 0, va_t = 0;
  size_t vn[kNVecN] = {};
  size_t vm[kNVecM] = {};
  size_t dc = 0, bfin = 0, dr = 0, sense = 0;
  // windowed entries of each side (0 when none)
  size_t wcol_t = 0, wlane_t = 0, wslice_t = 0, wval_t = 0, wpass_t = 0, wrange_t = 0;
  size_t wcol_a = 0, wlane_a = 0, wslice_a = 0, wval_a = 0, wpass_a = 0, wrange_a = 0;
  size_t segp_t = 0, srow_t = 0, sptr_t = 0, sids_t = 0;  // segmented rows (0 when none)
  size_t segp_a = 0, srow_a = 0, sptr_a = 0, sids_a = 0;
  // the opening evaluation's sparse products (FP32 with windowed chunks)
  bool has_evp = false;
  size_t evp_t0 = 0, evp_t1 = 0, evp_a = 0;
  // device-side preparation (0 when the host prepares)
  size_t raw_a = 0, raw_t = 0, raw_b = 0, raw_c = 0, raw_l = 0, raw_u = 0, sr = 0, sc = 0;
  size_t pscr = 0, wsrc_t = 0, wsrc_a = 0;
  // device-side structure (0 when the host builds it): the caller's CSR,
  // the orders, the fill cursors and the entries' places
  size_t st_rp = 0, st_perm_a = 0, st_inv_a = 0, st_inv_t = 0, st_cur = 0, st_ci = 0,
         st_val = 0, st_ti = 0, st_tk = 0;
  size_t total = 0;
};

int prepare(const opdhg_lp* lp, const opdhg_params* p, Prepared& out, bool structure_only);
SlotLayout slot_layout(const Prepared& P, int prec);
LpDev slot_pointers(uint8_t* base, const SlotLayout& L, const Prepared& P);
// Writes the slot's image; with device-side preparation also runs the
// preparation kernels and fills P.dr, P.dc, P.eta0 and P.omega0 from the
// device (synchronizes the stream then).
int upload_slot(uint8_t* base, const SlotLayout& L, Prepared& P, int prec, hipStream_t stream,
                SlotImage& img);
// Launch tables of a set of LPs at dst: LP table, both work lists (chunked
// over at most cap workgroups), counts and the Ctl board. With capacity > 0,
// OPDHG_ERR_OVER_BUDGET when they need more bytes. With fixed_launch the
// launch grids in cfg are kept (they must cover the new grids).
int write_tables(uint8_t* dst, const std::vector<LpDev>& lps,
                 const std::vector<const Prepared*>& preps, int64_t cap, hipStream_t stream,
                 std::vector<uint8_t>& staging, LaunchCfg* cfg, int64_t* nwt, int64_t* nwa,
                 size_t capacity = 0, bool fixed_launch = false);
// Bytes of the launch tables of a fixed set (evaluation and step lists,
// windowed chunks), or of the server's shared tables (evaluation lists,
// which its step kernels also run).
size_t tables_bytes(const std::vector<const Prepared*>& preps, int64_t cap);
size_t tables_bytes(int64_t nlps, int64_t nwork_t, int64_t nwork_a, int64_t cap);
// The step tiles of an LP: its rows outside windowed chunks, tiled.
void step_tiles(Prepared& P, int64_t cap, int lanes);
// Work list of one side for a set of LPs (tiles of LP 0, then LP 1, ...),
// chunked over at most cap workgroups and padded to grid * chunk items;
// fills each item's slot / last flags and each LP's slot count.
// step: the step kernels' tiles (stiles) and slot counts (nslot_st / nslot_sa).
void side_items(std::vector<LpDev>& lps, const std::vector<const Prepared*>& preps, bool tside,
                int64_t cap, int* grid, int* chunk, std::vector<WorkItem>& out, bool step = false);
// Workgroup cap of the sparse-product launches under these parameters.
int64_t grid_cap(const opdhg_params* p);
void chunking(int64_t n, int64_t cap, int* grid, int* chunk);
int download_vec(const void* dptr, size_t count, int prec, hipStream_t stream, double* out);
void fill_result(const Ctl& c, double seconds, opdhg_result* r);
void rescale_host(const opdhg_lp* lp, const opdhg_params* p, std::vector<double>& sval,
                  std::vector<double>& dr, std::vector<double>& dc);
std::vector<Tile> build_tiles(const int32_t* rp, int64_t rows, int64_t cap, int lanes_fixed);
void unpermute(const double* dev, const std::vector<int32_t>& perm, const double* scale,
               double* out);
Ctl initial_ctl(const Prepared& P);

// Attempt slots between the guarded evaluation steps inside a launch
// sequence, by default: every 8 slots for one LP, every 4 for a set of
// several (each LP of a set reaches its evaluation points at its own
// times). mid_eval_every() resolves opdhg_params::eval_slots.
constexpr int kMidEvalEvery = 8;
constexpr int kMidEvalEveryShared = 4;
int mid_eval_every(const opdhg_params* p, int64_t nlps);

// A set of LPs launched together, with its captured launch sequence: one
// evaluation step, then `attempts` step attempts with a guarded evaluation
// step after every mid_every of them (none when mid_every <= 0). An LP
// whose iteration count reaches an evaluation point inside the sequence
// (after a rejected attempt, say) is evaluated there and goes on within
// mid_every slots, instead of waiting for the next sequence. A guarded step
// in which no LP is due returns after one load per kernel (Counts::hint).
//
// Direct mode (for callers that cannot let the library create HIP objects):
// no captured graph, no streams or events of the library's own; each replay
// launches the same sequence on the caller's stream, and a side's tile and
// windowed kernels run one after the other.
struct Group {
  hipStream_t stream = nullptr;      // caller's stream (replays, copies)
  hipStream_t cap_stream = nullptr;  // private stream used only for capture
  hipGraphExec_t exec = nullptr;
  // a side's tile kernel runs on side_stream beside its windowed kernel
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  LaunchCfg cfg{};
  int prec = 0;
  bool direct = false;
  int seq_attempts = 0;  // attempts per sequence (direct mode)
  int mid_every = kMidEvalEvery;
  int init(void* stream, int prec, bool direct = false);
  int launch_side(bool primal, int force, hipStream_t s);
  // enqueue one launch sequence (evaluation, attempts, board) on s
  int enqueue(hipStream_t s, int attempts);
  int capture(int attempts_per_replay);
  int launch_init();
  int launch_primal_forced();
  int launch_dual_forced();
  int launch_learn_flush();
  int replay();
  void release();
};

int run_group(Group& grp, const std::vector<Ctl*>& d_ctls, std::vector<Ctl>& h_ctls,
              Ctl* pinned, int64_t k_target, double time_limit, double* elapsed);

// Session set-up behind opdhg_session_create; direct: a launch group in
// direct mode and pageable readback (nothing allocated on the device or
// pinned). need_out (optional) receives the device bytes the LP needs.
int session_create(const opdhg_lp* lp, const opdhg_params* p, void* d_workspace,
                   size_t workspace_bytes, void* hip_stream, bool direct, opdhg_session** out,
                   size_t* need_out);

}  // namespace opdhg
