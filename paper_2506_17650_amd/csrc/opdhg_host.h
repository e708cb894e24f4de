// Host-side structures of the opdhg library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

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

// An LP after validation, rescaling and transposition, in FP64 on the host.
// Arrays marked "device order" follow the relabelling by row class:
// device row i of A is original row perm_a[i], device variable j is
// original variable perm_t[j].
struct Prepared {
  int64_t m = 0, n = 0, nnz = 0;
  std::vector<int32_t> perm_a, perm_t;
  std::vector<int32_t> rp_a, ci_a, rp_t, ci_t;  // device order
  std::vector<double> va_a, va_t;               // device order
  std::vector<double> b, c, l, u, x0;           // device order
  std::vector<double> dr_dev, dc_dev;           // device order
  std::vector<double> dr, dc;                   // original order (unscaling)
  std::vector<int8_t> sense, bfin;              // device order
  std::vector<Tile> tiles_a, tiles_t;
  std::vector<double> pow_tab;  // step-rule factors, 2 * kPowTab
  DevParams prm;
  double eta0 = 1.0, omega0 = 1.0;
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
  size_t total = 0;
};

int prepare(const opdhg_lp* lp, const opdhg_params* p, Prepared& out, bool structure_only);
SlotLayout slot_layout(int64_t m, int64_t n, int64_t nnz, int64_t ntiles_t, int64_t ntiles_a,
                       int prec);
LpDev slot_pointers(uint8_t* base, const SlotLayout& L, const Prepared& P);
int upload_slot(uint8_t* base, const SlotLayout& L, const Prepared& P, int prec,
                hipStream_t stream, std::vector<uint8_t>& img);
// Launch tables of a set of LPs at dst: LP table, both work lists (chunked
// over at most cap workgroups), counts and the Ctl board. With capacity > 0,
// OPDHG_ERR_OVER_BUDGET when they need more bytes. With fixed_launch the
// launch grids in cfg are kept (they must cover the new grids).
int write_tables(uint8_t* dst, const std::vector<LpDev>& lps,
                 const std::vector<const Prepared*>& preps, int64_t cap, hipStream_t stream,
                 std::vector<uint8_t>& staging, LaunchCfg* cfg, int64_t* nwt, int64_t* nwa,
                 size_t capacity = 0, bool fixed_launch = false);
size_t tables_bytes(int64_t nlps, int64_t nwork_t, int64_t nwork_a, int64_t cap);
// Work list of one side for a set of LPs (tiles of LP 0, then LP 1, ...),
// chunked over at most cap workgroups and padded to grid * chunk items;
// fills each item's slot / last flags and each LP's slot count.
void side_items(std::vector<LpDev>& lps, const std::vector<const Prepared*>& preps, bool tside,
                int64_t cap, int* grid, int* chunk, std::vector<WorkItem>& out);
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

// A set of LPs launched together, with its captured launch sequence:
// one evaluation step then `attempts` step attempts.
struct Group {
  hipStream_t stream = nullptr;      // caller's stream (replays, copies)
  hipStream_t cap_stream = nullptr;  // private stream used only for capture
  hipGraphExec_t exec = nullptr;
  LaunchCfg cfg{};
  int prec = 0;
  int init(void* stream, int prec);
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

}  // namespace opdhg
