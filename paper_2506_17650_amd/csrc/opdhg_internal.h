// Internal structures shared by the host driver and the HIP kernels.
//
// Device layout of one LP ("slot"): both CSR copies (A and A^T, int32 row
// pointers and column indices, values in the compute precision V), the
// iteration vectors in V, the rescaling diagonals in FP64, per-tile FP64
// reduction partials, the tile tables, a control block (Ctl) and the
// per-LP constants (DevParams). Everything sits in the caller's workspace.
//
// Double buffering: x, y, A x, and the running sums of x and y have two
// copies; Ctl::cur names the current one. An attempt writes the other copy,
// and accepting it flips Ctl::cur, so a rejected attempt leaves no trace.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace opdhg {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kPartStride = 32;    // doubles of reduction partials per tile (16 double-doubles)
constexpr int kPowTab = 8192;      // host-computed step-rule factors for the first attempts
constexpr int kPowRing = 64;       // factors for the attempts of one launch sequence (at most
                                   // kPowRing attempts each)
constexpr int kGridCap = 2048;     // default workgroups of a launch (chunks of the work list)
constexpr int kMaxGrid = 65536;    // largest workgroup count a caller may ask for
constexpr int kTileCap = 1024;     // nonzeros of a stream tile (staged in LDS)

// Status values (match OPDHG_STATUS_* of the public header).
constexpr int kOptimal = 0;
constexpr int kIterLimit = 1;
constexpr int kTimeLimit = 2;
constexpr int kNumError = 3;
constexpr int kRunning = 4;

// Per-LP constants, written once at upload.
struct DevParams {
  double tol;
  double lr;
  double floor;
  double beta_suff, beta_nec, beta_art;
  double pw_smoothing;
  double step_growth, step_reduction;
  double b_norm, c_norm;  // norms of the unscaled b and c
  double c0;              // objective offset
  int64_t max_iter;
  int32_t phi;
  int32_t normalize;
  int32_t schedule;
  int32_t eval_every;
  int32_t max_retries;
  int32_t flags;  // kConstantStep | kNoRestart | kWeightedStep | kLowerZero | kNoUpper
};

constexpr int32_t kConstantStep = 1;  // every attempt accepted, eta unchanged (vanilla PDHG)
constexpr int32_t kNoRestart = 2;     // evaluations test termination only
constexpr int32_t kWeightedStep = 4;  // step-rule movement in the T^-1 and Sigma^-1 norms
// every lower bound is 0 / every upper bound is +inf: the primal step knows
// those bounds without reading them
constexpr int32_t kLowerZero = 8;
constexpr int32_t kNoUpper = 16;

// Per-LP control block: the scalar state of the iteration. Written by the
// decision kernels (step, termination / restart), the first tile of the
// primal kernel (clears the restart flags), and the host between launches.
struct Ctl {
  double eta;       // step size of the next attempt
  double omega;     // primal weight
  double w;         // sum of accepted step sizes of this restart period
  double eta_acc;   // step size of the last accepted attempt
  double g2;        // |c - A^T y|^2 of the last accepted attempt
  double r2;        // |b - A x|^2 of the last accepted attempt
  double gp2;       // |G^p|^2 of the last accepted attempt (unnormalized)
  double gd2;       // |G^d|^2
  double hp_norm;   // AdaGrad accumulators of the norm schedule
  double hd_norm;
  double anc_rp2, anc_rd2, anc_gap;  // KKT parts of the restart anchor
  double prev_cand;                  // candidate's weighted KKT at the last evaluation
  double restart_w;                  // w of the period a restart closes
  double out_pobj, out_dobj, out_relp, out_reld, out_relg, out_rel;
  double last_eta_bar;
  int64_t k;         // accepted iterations
  int64_t t;         // accepted iterations since the last restart
  int64_t attempts;  // all attempts
  int64_t restarts;
  int64_t retries;   // rejections of the current iteration
  int64_t k_limit;   // attempts pause when k reaches it (host-controlled)
  int64_t ring_base; // the step-rule factor ring holds attempts ring_base+1 .. +kPowRing
  int32_t status;
  int32_t cur;           // current buffer (0 or 1)
  int32_t need_eval;     // an evaluation is due before the next attempt
  int32_t learn_pending; // the learner must apply the accepted gradients
  int32_t restart_pending;
  int32_t restart_avg;   // the restart point is the average
  int32_t finalize_avg;  // terminal with the average: copy it into the current buffers
  int32_t anchor_set;
  int32_t which;         // 0 current, 1 average (returned iterate)
  int32_t stop_request;  // host asks for a final evaluation (time limit)
  int32_t learn_now;     // the next attempt is an update iteration (k mod phi == 0)
  int32_t weighted_step; // movement partials divided by T and Sigma (read with the other fields)
  int32_t fail_pending;  // a numerical failure ends the solve at the next evaluation, which
                         // reports the current iterate with NUMERICAL_ERROR
  int32_t pad3, pad4, pad5;
};

// Tile: rows [rb, re) of one CSR side with nonzeros [s, e).
// lanes > 0: stream tile (e - s <= kTileCap, re - rb <= kBlock / lanes),
// each row reduced from LDS by `lanes` threads; lanes == 0: one row longer
// than kTileCap, reduced by the whole workgroup; lanes < 0 (step lists
// only): a piece of a row longer than kSplitNnz, whose sum the workgroup
// stores as segment partial `seg` for the finishing kernel.
struct Tile {
  int32_t rb, re, s, e, lanes, seg;
};

// Rows longer than kSplitNnz that the step kernels take in tiles are split
// into pieces of kPieceNnz nonzeros, one workgroup each, so that one long
// row does not hold a single workgroup for the whole launch.
constexpr int kSplitNnz = 16384;
constexpr int kPieceNnz = 4096;

// Windowed sparse products (FP32). Rows of one side whose gathered vector
// entries fall into a few column ranges are taken in chunks of consecutive
// rows by workgroups of kWinBlock threads. For each pass the workgroup
// copies a window of vector entries (whole buckets of kWinBucket columns)
// into LDS, then streams the pass's entries and
// gathers from LDS; row sums of the passes add up in LDS and feed the same
// row epilogues as the tile kernels. A pass's rows, ordered by their entry
// count in the pass, form slices of kWinSlice rows, one row per lane of a
// wavefront; a slice stores its entries (window-local column, value) k-major,
// entry k of lane l at e0 + k * kWinSlice + l, padded to its longest row.
constexpr int kWinBlock = 1024;
constexpr int kWinSlice = 64;
constexpr uint16_t kWinNoRow = 0xFFFF;  // an empty lane of a slice
constexpr int kWinBucket = 512;
constexpr int kWinParamBucket = 1024;  // the unit of the window_buckets parameter
constexpr int kWinRows = 10240;
// The LDS of a windowed workgroup: a chunk of several passes holds one
// pass's window of up to kWinBuckets buckets beside the chunk's row sums; a
// chunk of one pass keeps its row sums in registers during the pass, so its
// window takes up to kWinOneBuckets buckets and the row sums reuse that LDS
// afterwards.
constexpr int kWinBuckets = 56;
constexpr int kWinCap = kWinBuckets * kWinBucket;
constexpr int kWinOneBuckets = kWinBuckets + kWinRows / kWinBucket;
constexpr int kWinOneCap = kWinOneBuckets * kWinBucket;
constexpr int kWinMaxPass = 4;
constexpr int kWinWaves = kWinBlock / 64;
// slices of one pass per wave (a pass has at most kWinRows rows)
constexpr int kWinWaveSlices = kWinRows / kWinSlice / kWinWaves;
// LDS of a windowed workgroup: window (and row sums), reduction
constexpr size_t kWinLds = (size_t)kWinOneCap * 4 + kWinWaves * 4 * 16;
static_assert(kWinOneCap == kWinCap + kWinRows, "one layout of LDS for both kinds of chunk");

// Slices [s0, s1) of a pass and the vector ranges [range0, range0 + nrange)
// it stages, in window order.
struct WinPass {
  int32_t s0, s1, range0, nrange;
};
// A slice: entries e0 + k * kWinSlice + lane for k < len (e0 a multiple of
// kWinSlice); the chunk-local row of each lane is in a parallel array.
struct WinSlice {
  int32_t e0, len;
};
struct WinRange {
  int32_t src, len;  // vector entries [src, src + len), device order
};
// A windowed chunk: rows [r0, r1) of one LP side, passes [pass0, pass0 + npass),
// then nseg segments of long rows (partials seg0 .. seg0 + nseg - 1).
struct WinItem {
  Ctl* ctl;
  int32_t lp, slot;
  int32_t r0, r1;
  int32_t pass0, npass;
  int32_t nseg, seg0;
};
// Segmented long rows [s0, s1) of one LP side's list, finished by one
// workgroup: kSegLanes lanes per row add its partials.
constexpr int kSegLanes = 16;
constexpr int kSegRows = 256 / kSegLanes;
struct SegItem {
  Ctl* ctl;
  int32_t lp, slot;
  int32_t s0, s1;
};

// One LP slot as the kernels see it (device pointers into the workspace).
struct LpDev {
  int32_t m, n;
  int32_t ntiles_t, ntiles_a;  // tiles over A^T rows (n) and A rows (m); partial stride
  int32_t nslot_t, nslot_a;    // partial slots of the evaluation kernels (one per chunk of
                               // the evaluation list touching the LP)
  int32_t nslot_st, nslot_sa;  // partial slots of the step kernels (one per step tile, then
                               // one per windowed chunk and segment workgroup)
  int32_t item0_t, item0_a;    // position of the LP's first item in each evaluation list
  const int32_t* rp_a;
  const int32_t* ci_a;
  const void* va_a;
  const int32_t* rp_t;
  const int32_t* ci_t;
  const void* va_t;
  const Tile* tiles_a;
  const Tile* tiles_t;
  // n-vectors (type V)
  void* c;
  void* l;
  void* u;
  void* T;
  void* Hp;
  void* Gp;
  void* x[2];
  void* xs[2];
  void* xa;
  // m-vectors (type V)
  void* b;
  void* S;
  void* Hd;
  void* Gd;
  void* y[2];
  void* ys[2];
  void* ya;
  void* Ax[2];
  void* Axa;
  // FP64 scaling diagonals and per-variable / per-row flags
  const double* dr;
  const double* dc;
  const int8_t* sense;  // m: 0 '=', 1 '>='
  const int8_t* bfin;   // n: bit 0 l finite, bit 1 u finite
  double* part_t;       // ntiles_t * kPartStride
  double* part_a;       // ntiles_a * kPartStride
  const double* pow_tab;  // 2 * kPowTab: (j+1)^-reduction, then (j+1)^-growth, j = 1..kPowTab
  double* pow_ring;       // 2 * kPowRing: the factors for j = ring_base+1 .. +kPowRing
  Ctl* ctl;
  const DevParams* prm;
  // copies of the parameters the step decision reads, so that they arrive
  // with the record instead of one dependent load later
  double s_lr;
  int64_t s_max_iter;
  int32_t s_phi, s_schedule, s_normalize, s_eval_every, s_max_retries, s_flags;
  // windowed rows of each side (FP32; empty when the side has none)
  const uint16_t* wcol_t;   // window-local column of each entry
  const uint16_t* wlane_t;  // chunk-local row of each slice lane (kWinNoRow: none)
  const WinSlice* wslice_t;
  const void* wval_t;       // value of each entry (type V)
  const WinPass* wpass_t;
  const WinRange* wrange_t;
  const uint16_t* wcol_a;
  const uint16_t* wlane_a;
  const WinSlice* wslice_a;
  const void* wval_a;
  const WinPass* wpass_a;
  const WinRange* wrange_a;
  // long rows split into segments over windowed chunks: the segments'
  // partial row sums (type V), the rows and their partials' ids (CSR)
  void* segp_t;
  const int32_t* srow_t;
  const int32_t* sptr_t;
  const int32_t* sids_t;
  void* segp_a;
  const int32_t* srow_a;
  const int32_t* sptr_a;
  const int32_t* sids_a;
  // FP32 LPs with windowed chunks: the opening evaluation's sparse
  // products, computed by the windowed machinery before the evaluation
  // kernels read them (A^T y, A^T y_avg over n; A x_avg over m); null
  // otherwise (the evaluation kernels then gather per nonzero)
  float* evp_t0;
  float* evp_t1;
  float* evp_a;
};

// A set of LPs launched together. A work item is one tile of one LP, with
// the tile's rows and the LP's control block inline so a workgroup reaches
// everything it needs in one dependent load. The kernels loop over the
// items with a fixed grid, so the set can change between launches without
// new launch parameters; lp < 0 marks padding.
struct WorkItem {
  Ctl* ctl;
  int32_t lp;     // index into the LP table
  int32_t tile;   // index of the tile within its side of the LP
  int32_t rb, re; // rows [rb, re)
  int32_t s, e;   // nonzeros [s, e)
  int32_t lanes;  // see Tile
  int32_t slot;   // partial slot of this item: its tile's index in the LP's list
  int32_t seg;    // lanes < 0 (a piece of a split long row): its segment partial; else -1
  int32_t first;  // 1 on the LP's first item of the list
};

// Item counts and chunking of a set, in device memory. Chunk c of a side
// holds items [c * chunk, (c + 1) * chunk) of that side's list, which is
// padded to grid * chunk items. The kernels read these at run time, so a
// captured launch sequence serves any set whose grids fit its launch grids
// (the server rewrites the tables between replays).
struct Counts {
  int32_t nwork_t, nwork_a, nlps, pad;
  int32_t grid_t, chunk_t;  // chunks (a multiple of 8 when above 8) and items per chunk
  int32_t grid_a, chunk_a;
  // Hints for the guarded evaluation steps inside a launch sequence (a
  // performance hint only: the evaluation that opens each sequence ignores
  // them). The step decision sets both words when it makes an evaluation
  // due; guarded step b reads word b & 1 and returns at once when it is 0;
  // step b clears word (b + 1) & 1, the next step's, at its start.
  int32_t hint[2];
  int32_t pad2[2];
};

// Host-side launch wrappers (kernels.hip). V is float or double.
// What the step decision reads from an LP's record: its control block,
// factor ring, the step kernels' partials (stride and slot count per side)
// and the parameters it uses.
struct DecideRec {
  Ctl* ctl;
  const double* ring;
  const double* part_t;
  const double* part_a;
  int32_t ntiles_t, ntiles_a, ns_t, ns_a;
  double lr;
  int64_t max_iter;
  int32_t phi, schedule, normalize, eval_every, max_retries, flags;
};

struct LaunchCfg {
  const LpDev* lps;        // device pointers
  const WorkItem* work_t;  // A^T-side tiles of all LPs
  const WorkItem* work_a;  // A-side tiles
  const Counts* counts;
  Ctl* board;              // after each launch sequence: copy of every LP's Ctl, in LP order
  // launch grids; each covers the device-side grid it serves (workgroups
  // past the device grid exit at once)
  int launch_t, launch_a;  // sparse-product kernels of each side
  int launch_ta;           // kernels that visit both sides
  int launch_lp;           // one workgroup per LP (decision kernels, board)
  // host copy of the device-side chunking
  int grid_t, chunk_t, grid_a, chunk_a;
  // the step kernels' work: tile lists (rows not taken by windowed chunks)
  // and windowed chunks. With step_fixed the tile lists' chunking is the
  // one below (a fixed set of LPs); else step_t / step_a point at the
  // evaluation lists, which run with the device-side chunking.
  const WorkItem* step_t;
  const WorkItem* step_a;
  const WinItem* win_t;
  const WinItem* win_a;
  int sgrid_t, schunk_t, sgrid_a, schunk_a;
  int nwin_t, nwin_a;  // windowed chunks per side (launch grid rounded up to 8)
  int step_fixed;
  int evprod;  // LPs of the set with evaluation products (evp_*): 0 none, 1 some, 2 all
  const SegItem* seg_t;  // segmented long rows, finished after the windowed chunks
  const SegItem* seg_a;
  int nseg_t, nseg_a;
  // a fixed set of one LP: its decision record comes with the launch
  // arguments, so the decision kernel skips reading the LP table
  int solo, pad2_;
  DecideRec solo_rec;
};

template <typename V>
struct Kernels {
  static int init_products(const LaunchCfg& c, void* stream);
  static int primal(const LaunchCfg& c, void* stream, int force);
  static int dual(const LaunchCfg& c, void* stream, int force = 0);
  // windowed chunks of each side (FP32 only; nothing to launch when the set has none)
  static int primal_win(const LaunchCfg& c, void* stream, int force);
  static int dual_win(const LaunchCfg& c, void* stream, int force = 0);
  // segmented long rows: adds each row's segment partials and runs its epilogue
  static int primal_seg(const LaunchCfg& c, void* stream, int force);
  static int dual_seg(const LaunchCfg& c, void* stream, int force = 0);
  static int decide(const LaunchCfg& c, void* stream);
  static int learn_flush(const LaunchCfg& c, void* stream);
  // mid: 0 for the evaluation opening a launch sequence, b > 0 for the b-th
  // guarded evaluation step inside it (see Counts::hint)
  // the opening evaluation's sparse products of LPs with windowed chunks
  // (FP32; nothing to launch otherwise): tiles, windowed chunks and
  // segments of each side, one vector at a time
  static int eval_products(const LaunchCfg& c, void* stream);
  static int eval_t(const LaunchCfg& c, void* stream, int mid);
  static int eval_a(const LaunchCfg& c, void* stream, int mid);
  static int eval_decide(const LaunchCfg& c, void* stream, int mid);
  static int apply(const LaunchCfg& c, void* stream, int mid);
};

// Copies every LP's Ctl into c.board (precision independent).
int launch_board(const LaunchCfg& c, void* stream);

// Device-side preparation of one slot (FP64 arithmetic, results in V):
// the rescaling passes over the two stored CSR copies in device order,
// then the scaled values, vectors, windowed values and the first step size
// and primal weight. Every row statistic follows the host's expression and
// order (maxima; double-double sums added one entry at a time).
constexpr int kPrepGrid = 256;  // workgroups of the vector kernel (norm partials)
struct PrepCfg {
  const int32_t* rp_a;
  const int32_t* ci_a;
  const int32_t* rp_t;
  const int32_t* ci_t;
  const double* raw_a;  // unscaled values, device order of each CSR copy
  const double* raw_t;
  const double* raw_b;  // unscaled b (m), c, l, u (n), device order
  const double* raw_c;
  const double* raw_l;
  const double* raw_u;
  double* dr;  // diagonals, device order (start at 1)
  double* dc;
  double* sr;  // row / column statistics of a pass
  double* sc;
  double* scr;  // 4 * kPrepGrid norm partials, then amax bits, eta0, omega0, then the
                // power iteration's lam, done and zero flags (kPrepScr doubles)
  void* va_a;
  void* va_t;
  void* b;
  void* c;
  void* l;
  void* u;
  void* x0;
  void* xa;
  void* wval_t;
  void* wval_a;
  const int32_t* wsrc_t;
  const int32_t* wsrc_a;
  int64_t went_t, went_a;
  Ctl* ctl;
  int32_t m, n;
  int32_t nlong_a, nlong_t;  // rows of more than 256 nonzeros (the first in device order)
  // the constant step (vanilla PDHG): eta0 = step_scale / |A~|_2, the norm
  // from power_iters rounds of power iteration stopped at power_tol
  double step_scale, power_tol;
  int32_t power_iters, pad;
};
constexpr int kPrepScr = 4 * kPrepGrid + 6;
// Device-side structure of one slot (the host keeps only the row and
// column lengths, the row-class orders and the tiles): the caller's CSR
// goes up as given, and two kernels build both copies in device order.
// k_struct_rows copies each row of A to device order (columns relabelled)
// and drops every entry into its A^T row at a fill cursor; k_struct_cols
// then puts each A^T row in ascending original row order by rank, the
// order of the host's column index, so both copies equal the host's bit
// for bit. Columns are at most kStructMaxCol long (else the host builds the
// structure).
constexpr int kStructMaxCol = 4096;
struct StructCfg {
  const int64_t* src_rp;   // m + 1, the caller's row pointers
  const int32_t* src_ci;   // nnz, the caller's column indices
  const double* src_val;   // nnz, the caller's values
  const int32_t* perm_a;   // device row -> original row (m)
  const int32_t* inv_a;    // original row -> device row (m)
  const int32_t* inv_t;    // original column -> device column (n)
  const int32_t* rp_a;     // device order row pointers of A (m + 1)
  const int32_t* rp_t;     // and of A^T (n + 1)
  int32_t* cur;            // n fill cursors, starting at rp_t[j]
  int32_t* tmp_i;          // nnz: original row of each entry at its cursor position
  int32_t* tmp_k;          // nnz: its position in the caller's arrays
  int32_t* ci_a;
  double* raw_a;
  int32_t* ci_t;
  double* raw_t;
  int32_t m, n;
  int32_t nlong_a;  // rows of A longer than 256 (first in device order)
  int32_t nmed_t;   // rows of A^T longer than 32 (first in device order)
};
int struct_build(const StructCfg& c, void* stream);

// kind 0: maxima of |a~|, 1: sums of |a~|^e, 2: L2 norms
int prep_stats(const PrepCfg& c, void* stream, bool tside, int kind, double e);
int prep_apply(const PrepCfg& c, void* stream);  // dr /= sqrt(sr), dc /= sqrt(sc)
int power_norm(const PrepCfg& c, void* stream);  // the constant step's eta0 (power iteration)
template <typename V>
int prep_finish(const PrepCfg& c, void* stream);
// Sets the windowed kernels' LDS attribute (once per process); 0 on success.
int window_kernels_ready();

const char* device_error_string();

}  // namespace opdhg
