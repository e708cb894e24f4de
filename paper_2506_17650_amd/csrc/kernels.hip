// HIP kernels of restarted PDHG with online preconditioning (gfx950).
//
// Every kernel covers a set of LPs, so one launch serves one LP, a packed
// batch or the server's changing mix. The rows of each CSR side (A or A^T)
// are cut into tiles; a work item is one tile of one LP. Each workgroup of
// 256 threads (4 wave64) takes a fixed, contiguous chunk of the work list.
//
// A stream tile holds up to kTileCap nonzeros of consecutive rows. Its
// workgroup first streams the tile's column indices and values with
// coalesced loads, gathers the vector entries and writes the products to
// LDS, all loads of the tile in flight together; then each row is reduced
// from LDS by a group of `lanes` threads and finished by a per-row epilogue
// whose vector loads were issued before the stream. A row longer than
// kTileCap is a tile of its own, reduced by the whole workgroup.
//
// The epilogues fuse the method's vector work into the sparse products and
// accumulate FP64 partial sums per thread. The step kernels store one
// partial per tile (a DPP scan per wave, then the waves' totals added once
// per window of work items); the evaluation kernels store one per chunk and
// LP. A one-workgroup-per-LP decision kernel sums an LP's partials in a
// fixed order and takes its scalar decision. Workgroups never wait for or
// signal each other inside a launch; kernel boundaries carry every result
// to the next step.
//
// Per attempt (the PDHG step of Algorithm 1, eq. (6)):
//   k_primal  CSR(A^T) SpMV of y, g = c - A^T y, x' = proj_[l,u](x - (eta/w) T g),
//             running sum of x, primal online gradient on update iterations
//             (eq. (7)), partials |x'-x|^2, |g|^2, |G^p|^2
//   k_dual    CSR(A) SpMV of x', A x_bar = 2 A x' - A x, dual step and sign
//             projection, running sum of y, dual online gradient, partials
//             |y'-y|^2, (y'-y).(A x'-A x), |b-Ax|^2, |G^d|^2
//   k_decide  adaptive step rule: accept (flip buffers) or retry
// The normalized online-gradient step with AdaGrad on T and Sigma
// (the learner of Algorithm 1) after an accepted update iteration is applied by
// the next attempt's k_primal (T) and k_dual (Sigma) to the rows they
// visit, before those rows use the preconditioner.
// Every eval_every accepted iterations (at the start of a launch sequence,
// or at one of the guarded evaluation steps inside it):
//   k_eval_t  CSR(A^T) SpMV of y and of the average of y: reduced costs,
//             dual residuals, bound terms of the dual objective, c^T x, and
//             distances to the restart anchor, for current and average
//   k_eval_a  CSR(A) SpMV of the average of x: primal residuals, b^T y,
//             distances
//   k_eval_decide  termination and restart decision
//   k_apply   moves the iterate to the restart point, resets the sums and the
//             anchor (preconditioners kept), or copies a returned average out
//
// Summation. In FP64 mode every FP64 reduction and every SpMV row sum is
// accumulated in double-double: each product is split exactly with an FMA
// into p + e, p is added with an error-free two-sum and all round-off is
// gathered in a second double, which is folded in once at the end. The
// result is the correctly rounded sum except when the exact value lies
// within about n * 2^-106 (relative) of a rounding boundary, so it does not
// depend on the tiling, the lane count, the grid, or what else shares the
// launch. In FP32 mode the SpMV products and row sums are FP32 and the step
// kernels' partial sums plain FP64 in a fixed order, one partial per tile,
// so their values depend on the tile sizes but not on the grid or on what
// else shares the launch; the evaluation's sums stay double-double.
#include <hip/hip_runtime.h>

#include <math.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "crmath.h"
#include "opdhg_internal.h"

namespace opdhg {

namespace {

// ---- double-double accumulation ----
struct DD {
  double hi, lo;
};

__device__ __forceinline__ DD dd_zero() { return DD{0.0, 0.0}; }

// a += x, with the round-off of the high part kept in lo
__device__ __forceinline__ void dd_add(DD& a, double x) {
  const double s = a.hi + x;
  const double bb = s - a.hi;
  const double err = (a.hi - (s - bb)) + (x - bb);
  a.hi = s;
  a.lo += err;
}

// a += x * y with the product split exactly (p + e == x * y)
__device__ __forceinline__ void dd_add_prod(DD& a, double x, double y) {
  const double p = x * y;
  const double e = fma(x, y, -p);
  dd_add(a, p);
  a.lo += e;
}

__device__ __forceinline__ DD dd_merge(DD a, const DD& b) {
  dd_add(a, b.hi);
  a.lo += b.lo;
  return a;
}

__device__ __forceinline__ double dd_value(const DD& a) { return a.hi + a.lo; }

// a += x * y as a double-double, or (PLAIN) in FP64 alone with lo kept at
// 0. The FP32 step kernels use the plain form: their results move with the
// tiling by rounding anyway, and a fixed order keeps them run-to-run
// identical. FP64 runs keep the double-double, on which their independence
// of the tiling rests.
template <bool PLAIN>
__device__ __forceinline__ void acc_prod(DD& a, double x, double y) {
  if constexpr (PLAIN) a.hi = fma(x, y, a.hi);
  else dd_add_prod(a, x, y);
}

// ---- memory access ----
// Pointers into the workspace reach the kernels through tables, so the
// compiler sees generic pointers and emits flat accesses, which count
// toward both the vector-memory and the LDS counters: every wait for an LDS
// result then also waits for outstanding HBM loads and stores. Global views
// of the same addresses compile to global_* accesses that only count toward
// the vector-memory counter.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> gp(T* p) {
  return (gptr<T>)p;
}

// Element idx of a global array with a 32-bit byte offset: with the base
// in scalar registers this is one global load with a 32-bit vector offset
// (a 64-bit address would take two registers per load in flight). Every
// array of a slot is below 4 GiB (checked on the host).
template <typename T>
__device__ __forceinline__ T ldg(gptr<const T> base, uint32_t idx) {
  const uint32_t off = idx * (uint32_t)sizeof(T);
  return *reinterpret_cast<gptr<const T>>(reinterpret_cast<gptr<const char>>(base) + off);
}

template <typename T>
__device__ __forceinline__ T ldg(gptr<T> base, uint32_t idx) {
  return ldg<T>((gptr<const T>)base, idx);
}

template <typename T>
__device__ __forceinline__ void stg(gptr<T> base, uint32_t idx, T v) {
  const uint32_t off = idx * (uint32_t)sizeof(T);
  *reinterpret_cast<gptr<T>>(reinterpret_cast<gptr<char>>(base) + off) = v;
}

// Barrier for data exchanged through LDS only: waits for this wave's LDS
// accesses (lgkmcnt), not for its global loads and stores, which stay in
// flight across the barrier. A workgroup-scope fence, even one limited to
// LDS, makes the compiler drain every global store first (vmcnt(0)), which
// puts a store round trip in front of every reduction that follows a row
// epilogue. The compiler-only fences keep memory accesses on their side.
// No kernel here exchanges global data between the waves of a workgroup.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  // s_waitcnt lgkmcnt(0), with the vmcnt and expcnt fields at their maxima
  // (no wait on them)
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Chunk of the work list taken by this workgroup. Workgroups are handed to
// the 8 XCDs round-robin (workgroup b to XCD b mod 8), so with a grid that
// is a multiple of 8, XCD x takes the contiguous chunks
// [x * grid/8, (x + 1) * grid/8): the rows an XCD's tiles gather from stay
// in that XCD's L2 instead of being spread over all eight.
// g is the side's chunk count (read from the device-side counts); the
// launch grid may be larger, and workgroups b >= g get -1 (no chunk).
__device__ __forceinline__ int chunk_index(int g) {
  const int b = blockIdx.x;
  if (b >= g) return -1;
  if (g & 7) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

__device__ __forceinline__ DD dd_shfl_xor(const DD& a, int off) {
  return DD{__shfl_xor(a.hi, off, 64), __shfl_xor(a.lo, off, 64)};
}

// The value of another lane moved by DPP (a VALU operand modifier, no LDS
// traffic): CTRL selects the pattern, ROWS the rows of 16 lanes written;
// lanes without a source, and rows not written, get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

template <int CTRL, int ROWS, bool PLAIN, int NV>
__device__ __forceinline__ void dd_dpp_step(DD (&v)[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if constexpr (PLAIN) v[q].hi += dpp_f64<CTRL, ROWS>(v[q].hi);
    else v[q] = dd_merge(v[q], DD{dpp_f64<CTRL, ROWS>(v[q].hi), dpp_f64<CTRL, ROWS>(v[q].lo)});
  }
}

// Merge NV double-doubles over the workgroup (NW waves) in a fixed order;
// thread 0 gets the totals. s_red holds NW * NV DD. Within a wave a scan of
// DPP moves brings the wave's total to lane 63: row_shr by 1, 2, 4 and 8
// (lane 15 of each row of 16 holds the row's sum), row_bcast:15 into rows
// 1 and 3, then row_bcast:31 into rows 2 and 3. Every level runs in the
// VALU, so the reductions of all workgroups on a CU do not queue on LDS.
// PLAIN: FP64 sums of the high parts only (see acc_prod).
template <int NV, bool PLAIN>
__device__ __forceinline__ void wave_scan(DD (&v)[NV]) {
  dd_dpp_step<0x111, 0xF, PLAIN>(v);  // row_shr:1
  dd_dpp_step<0x112, 0xF, PLAIN>(v);  // row_shr:2
  dd_dpp_step<0x114, 0xF, PLAIN>(v);  // row_shr:4
  dd_dpp_step<0x118, 0xF, PLAIN>(v);  // row_shr:8
  dd_dpp_step<0x142, 0xA, PLAIN>(v);  // row_bcast:15
  dd_dpp_step<0x143, 0xC, PLAIN>(v);  // row_bcast:31
}

template <int NV, int NW = kBlock / 64, bool PLAIN = false>
__device__ __forceinline__ void block_sum(DD (&v)[NV], DD* s_red) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  wave_scan<NV, PLAIN>(v);
  if (lane == 63) {
#pragma unroll
    for (int q = 0; q < NV; ++q) s_red[wave * NV + q] = v[q];
  }
  lds_barrier();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      DD t = s_red[q];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        if constexpr (PLAIN) t.hi += s_red[w * NV + q].hi;
        else t = dd_merge(t, s_red[w * NV + q]);
      }
      v[q] = t;
    }
  }
  lds_barrier();
}

// Store workgroup totals in partial slot `slot` (thread 0). Partials are
// laid out quantity-major (hi and lo of quantity q at 2q * stride + slot and
// (2q + 1) * stride + slot) so the decision kernel reads them coalesced.
template <int NV>
__device__ __forceinline__ void store_partials(double* part, int stride, int slot,
                                               const DD (&v)[NV]) {
  if (threadIdx.x == 0) {
    gptr<double> g = gp(part);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      g[(size_t)(2 * q) * stride + slot] = v[q].hi;
      g[(size_t)(2 * q + 1) * stride + slot] = v[q].lo;
    }
  }
}

// Fixed-order merge of NV double-double partials over `count` slots (whole
// workgroup; quantity-major with the given stride); thread 0 gets the
// rounded totals. Partials were written by
// earlier launches. Each thread loads B tiles' partials before merging
// them, so the loads of a batch are in flight together.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int stride,
                                             int count, double (&out)[NV], DD* s_red) {
  constexpr int B = NV <= 4 ? 8 : 2;
  DD v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = dd_zero();
  const gptr<const double> g = gp(part);
  for (int base = threadIdx.x; base < count; base += kBlock * B) {
    double h[B][NV], l[B][NV];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      // out-of-range slots re-read slot `base` (valid) and are zeroed
      const int t = base + k * kBlock;
      const bool ok = t < count;
      const int tc = ok ? t : base;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const double hv = g[(size_t)(2 * q) * stride + tc];
        const double lv = g[(size_t)(2 * q + 1) * stride + tc];
        h[k][q] = ok ? hv : 0.0;
        l[k][q] = ok ? lv : 0.0;
      }
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] = dd_merge(v[q], DD{h[k][q], l[k][q]});
    }
  }
  block_sum<NV>(v, s_red);
#pragma unroll
  for (int q = 0; q < NV; ++q) out[q] = dd_value(v[q]);
}

// The same for two partial arrays at once (NA quantities over ca slots of
// pa, then NB over cb slots of pb): one pass, so the loads of both arrays
// are in flight together. PLAIN: the partials are plain FP64 sums (their
// low words are zero), read and added as plain doubles.
template <int NA, int NB, bool PLAIN, typename Mid>
__device__ __forceinline__ void sum_partials2(const double* pa, int sa, int ca, const double* pb,
                                              int sb, int cb, double (&out)[NA + NB],
                                              DD* s_red, Mid&& mid) {
  constexpr int B = 8;  // 2048 slots per round: one round of loads for most launch sets
  DD v[NA + NB];
  if constexpr (!PLAIN) {  // plain sums are set to zero by the first round
#pragma unroll
    for (int q = 0; q < NA + NB; ++q) v[q] = dd_zero();
  }
  const gptr<const double> ga = gp(pa), gb = gp(pb);
  const int count = ca > cb ? ca : cb;
  // Every thread runs the first round; mid() runs between its loads and
  // its merges, so that loads the caller issues there overlap them. Groups
  // of kBlock slots that lie past a side's count are skipped (a uniform
  // test); inside a group, slots past the count read slot 0 and add zero.
  auto round = [&](int r0, bool first) {
    const int t0 = r0 + (int)threadIdx.x;
    double h[B][NA + NB], l[B][NA + NB];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int t = t0 + k * kBlock;
      const int ta = t < ca ? t : 0, tb = t < cb ? t : 0;
      // only loads behind the uniform tests: the masks apply at the merge
#pragma unroll
      for (int q = 0; q < NA + NB; ++q) h[k][q] = l[k][q] = 0.0;
      if (r0 + k * kBlock < ca) {
#pragma unroll
        for (int q = 0; q < NA; ++q) {
          h[k][q] = ga[(size_t)(2 * q) * sa + ta];
          if constexpr (!PLAIN) l[k][q] = ga[(size_t)(2 * q + 1) * sa + ta];
        }
      }
      if (r0 + k * kBlock < cb) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          h[k][NA + q] = gb[(size_t)(2 * q) * sb + tb];
          if constexpr (!PLAIN) l[k][NA + q] = gb[(size_t)(2 * q + 1) * sb + tb];
        }
      }
    }
    if (first) {
      mid();
      // plain sums start from a zero the compiler cannot see: with a known
      // zero it moves the first additions into the load branches above,
      // each then waiting there for its loads
      if constexpr (PLAIN) {
        double z = 0.0;
        asm volatile("" : "+v"(z));
#pragma unroll
        for (int q = 0; q < NA + NB; ++q) v[q] = DD{z, 0.0};
      }
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {
      if (r0 + k * kBlock < count) {
        const int t = t0 + k * kBlock;
        const bool oka = t < ca, okb = t < cb;
#pragma unroll
        for (int q = 0; q < NA + NB; ++q) {
          const bool ok = q < NA ? oka : okb;
          if constexpr (PLAIN) v[q].hi += ok ? h[k][q] : 0.0;
          else v[q] = dd_merge(v[q], DD{ok ? h[k][q] : 0.0, ok ? l[k][q] : 0.0});
        }
      }
    }
  };
  round(0, true);
  for (int r0 = kBlock * B; r0 < count; r0 += kBlock * B) round(r0, false);
  block_sum<NA + NB, kBlock / 64, PLAIN>(v, s_red);
#pragma unroll
  for (int q = 0; q < NA + NB; ++q) out[q] = dd_value(v[q]);
}

// ---- numbers of the sparse products: exact products and double-double
// row sums in FP64, plain FP32 products and sums in FP32 ----
template <typename V>
struct Num;

template <>
struct Num<double> {
  struct Prod {
    double p, e;  // p + e is the exact product
  };
  static __device__ __forceinline__ Prod mul(double a, double x) {
    const double p = a * x;
    return Prod{p, fma(a, x, -p)};
  }
  // q, or zero, by a bit mask (a select of a loaded value can be turned
  // into a branch with the load inside)
  static __device__ __forceinline__ Prod mask(bool keep, const Prod& q) {
    const unsigned long long m = -(unsigned long long)keep;
    return Prod{__longlong_as_double(__double_as_longlong(q.p) & m),
                __longlong_as_double(__double_as_longlong(q.e) & m)};
  }
  struct Acc {
    DD v;
    __device__ __forceinline__ void zero() { v = dd_zero(); }
    __device__ __forceinline__ void add(const Prod& q) {
      dd_add(v, q.p);
      v.lo += q.e;
    }
    __device__ __forceinline__ void merge_xor(int off) { v = dd_merge(v, dd_shfl_xor(v, off)); }
    __device__ __forceinline__ void merge(const Acc& o) { v = dd_merge(v, o.v); }
    __device__ __forceinline__ double value() const { return dd_value(v); }
  };
};

template <>
struct Num<float> {
  using Prod = float;
  static __device__ __forceinline__ float mul(float a, float x) { return a * x; }
  static __device__ __forceinline__ float mask(bool keep, float q) {
    return __uint_as_float(__float_as_uint(q) & -(unsigned)keep);
  }
  struct Acc {
    float v;
    __device__ __forceinline__ void zero() { v = 0.f; }
    __device__ __forceinline__ void add(float q) { v += q; }
    __device__ __forceinline__ void merge_xor(int off) { v += __shfl_xor(v, off, 64); }
    __device__ __forceinline__ void merge(const Acc& o) { v += o.v; }
    __device__ __forceinline__ float value() const { return v; }
  };
};

template <typename V>
using Prod = typename Num<V>::Prod;
template <typename V>
using Acc = typename Num<V>::Acc;

// Segment partials of split rows: FP32 runs keep a float per segment; FP64
// runs keep the double-double sum (hi, lo), so that a split row's value is
// rounded once, after its pieces are merged, as an unsplit row's is.
__device__ __forceinline__ void seg_store(void* base, int sid, const Acc<float>& a) {
  stg(gp(static_cast<float*>(base)), (uint32_t)sid, a.v);
}
__device__ __forceinline__ void seg_store(void* base, int sid, const Acc<double>& a) {
  const gptr<double> g = gp(static_cast<double*>(base));
  stg(g, (uint32_t)(2 * sid), a.v.hi);
  stg(g, (uint32_t)(2 * sid + 1), a.v.lo);
}
__device__ __forceinline__ void seg_load(const void* base, int sid, Acc<float>& a) {
  a.v = ldg(gp(static_cast<const float*>(base)), (uint32_t)sid);
}
__device__ __forceinline__ void seg_load(const void* base, int sid, Acc<double>& a) {
  const gptr<const double> g = gp(static_cast<const double*>(base));
  a.v = DD{ldg(g, (uint32_t)(2 * sid)), ldg(g, (uint32_t)(2 * sid + 1))};
}

// Vector q at column c: vec[q][c], or vec[q][c] / div[q] for the average.
template <typename V>
__device__ __forceinline__ V vec_at(const gptr<const V>* vec, const double* div, int q, int c) {
  const V v = ldg(vec[q], (uint32_t)c);
  return div[q] > 0.0 ? (V)((double)v / div[q]) : v;
}

// LDS of a workgroup for the sparse products: kTileCap products per
// vector, and room for the cross-wave sums of a long row.
template <typename V, int NA>
struct SpmvShared {
  Prod<V> prod[NA][kTileCap];
  Acc<V> wave[4][NA];
};

constexpr int kK = kTileCap / kBlock;  // nonzeros per thread of a stream tile

// Registers of one stream tile between its load stage and its finish.
template <typename V, typename Pre>
struct StreamTile {
  V a[kK];
  int c[kK];
  int rp0, rp1;
  Pre pre;
};

// Stream tile, stage 1: every load of the tile that depends on no other
// load: the epilogue's vector loads (pre = load(row), issued by every
// thread of a row's group for a clamped valid row so that no load sits
// behind a branch), the row's pointers, and the tile's values and column
// indices (clamped to the tile's last nonzero, so the loads issue back to
// back). Stream tiles group `lanes` threads per row: group g owns row rb+g.
template <typename V, typename Pre, typename Load>
__device__ __forceinline__ void stream_load(const WorkItem& it, gptr<const int32_t> rp,
                                            gptr<const int32_t> ci, gptr<const V> va,
                                            Load&& load, StreamTile<V, Pre>& T) {
  const int tid = threadIdx.x;
  const int r = it.rb + (tid >> __builtin_ctz(it.lanes));
  const int rc = r < it.re ? r : it.re - 1;
  T.pre = load(rc);
  T.rp0 = ldg(rp, (uint32_t)rc);
  T.rp1 = ldg(rp, (uint32_t)rc + 1u);
  if (it.e > it.s) {  // a tile of empty rows has no nonzeros to read
    const int last = it.e - 1;
#pragma unroll
    for (int u = 0; u < kK; ++u) {
      const uint32_t k = (uint32_t)min(it.s + tid + u * kBlock, last);
      T.a[u] = ldg(va, k);
      T.c[u] = ldg(ci, k);
    }
  }
}

// Stage 2: the gathers of the NA vectors at the tile's columns.
template <typename V, int NA, typename Pre>
__device__ __forceinline__ void stream_gather(const WorkItem& it, const StreamTile<V, Pre>& T,
                                              const gptr<const V>* vec, const double* div,
                                              V (&x)[NA][kK]) {
  if (it.e > it.s) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
#pragma unroll
      for (int u = 0; u < kK; ++u) x[q][u] = vec_at(vec, div, q, T.c[u]);
    }
  }
}

// Stage 3: products into LDS (slots past the tile's end hold products of
// the repeated last nonzero; no row reads them), each row reduced by its
// group of lanes, and finish(row, sums[NA], pre) in the group's first lane.
// Called by the whole workgroup.
template <typename V, int NA, typename Pre, typename Finish>
__device__ __forceinline__ void stream_finish(const WorkItem& it, StreamTile<V, Pre>& T,
                                              const V (&x)[NA][kK], Finish&& finish,
                                              SpmvShared<V, NA>& sh) {
  const int tid = threadIdx.x;
  const int L = it.lanes;  // a power of two
  const int lane = tid & (L - 1);
  const int r = it.rb + (tid >> __builtin_ctz(L));
  const bool has_row = r < it.re;
  const int r0 = T.rp0 - it.s;
  const int r1 = r0 + ((T.rp1 - T.rp0) & -(int)has_row);  // empty range without a row
  if (it.e > it.s) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
#pragma unroll
      for (int u = 0; u < kK; ++u) sh.prod[q][tid + u * kBlock] = Num<V>::mul(T.a[u], x[q][u]);
    }
  }
  lds_barrier();
  if (has_row) {
    Acc<V> acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q].zero();
    int k = r0 + lane;
    // four products per pass so their LDS reads are in flight together;
    // they are added in the same order as one at a time
    for (; k + 3 * L < r1; k += 4 * L) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const Prod<V> p0 = sh.prod[q][k], p1 = sh.prod[q][k + L];
        const Prod<V> p2 = sh.prod[q][k + 2 * L], p3 = sh.prod[q][k + 3 * L];
        acc[q].add(p0);
        acc[q].add(p1);
        acc[q].add(p2);
        acc[q].add(p3);
      }
    }
    for (; k < r1; k += L) {
#pragma unroll
      for (int q = 0; q < NA; ++q) acc[q].add(sh.prod[q][k]);
    }
    for (int off = L >> 1; off > 0; off >>= 1) {
#pragma unroll
      for (int q = 0; q < NA; ++q) acc[q].merge_xor(off);
    }
    if (lane == 0) {
      V out[NA];
#pragma unroll
      for (int q = 0; q < NA; ++q) out[q] = acc[q].value();
      finish(r, out, T.pre);
    }
  }
  lds_barrier();
}

// A row longer than kTileCap (lanes == 0): every thread takes every
// kBlock-th nonzero, U at a time so their loads overlap; waves combine
// through LDS; thread 0 finishes the row.
template <typename V, int NA, typename Load, typename Finish>
__device__ __forceinline__ void long_row_tile(const WorkItem& it, gptr<const int32_t> ci,
                                              gptr<const V> va, const gptr<const V>* vec,
                                              const double* div, Load&& load, Finish&& finish,
                                              SpmvShared<V, NA>& sh) {
  const int tid = threadIdx.x;
  const int last = it.e - 1;
  const int r = it.rb;
  auto pre = load(r);
  Acc<V> acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q].zero();
  constexpr int U = 4;
  for (int k = it.s + tid; k < it.e; k += U * kBlock) {
    V a[U];
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t kk = (uint32_t)min(k + u * kBlock, last);
      a[u] = ldg(va, kk);
      c[u] = ldg(ci, kk);
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      V x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = vec_at(vec, div, q, c[u]);
      // a select, not a branch: a branch would let the compiler sink the
      // loads into it, one wait each
#pragma unroll
      for (int u = 0; u < U; ++u)
        acc[q].add(Num<V>::mask(k + u * kBlock < it.e, Num<V>::mul(a[u], x[u])));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q].merge_xor(off);
  }
  if ((tid & 63) == 0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) sh.wave[tid >> 6][q] = acc[q];
  }
  lds_barrier();
  if (tid == 0) {
    V out[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      Acc<V> t = sh.wave[0][q];
      t.merge(sh.wave[1][q]);
      t.merge(sh.wave[2][q]);
      t.merge(sh.wave[3][q]);
      out[q] = t.value();
    }
    finish(r, out, pre);
  }
  lds_barrier();
}

// A piece of a split long row (lanes < 0): the workgroup sums the piece's
// products with vector 0 as long_row_tile does and hands the sum to
// store(seg, acc) instead of running the row epilogue; the finishing kernel
// merges the row's pieces in order.
template <typename V, int NA, typename Store>
__device__ __forceinline__ void piece_tile(const WorkItem& it, gptr<const int32_t> ci,
                                           gptr<const V> va, const gptr<const V>* vec,
                                           const double* div, Store&& store,
                                           SpmvShared<V, NA>& sh) {
  const int tid = threadIdx.x;
  const int last = it.e - 1;
  Acc<V> acc;
  acc.zero();
  constexpr int U = 4;
  for (int k = it.s + tid; k < it.e; k += U * kBlock) {
    V a[U], x[U];
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t kk = (uint32_t)min(k + u * kBlock, last);
      a[u] = ldg(va, kk);
      c[u] = ldg(ci, kk);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = vec_at(vec, div, 0, c[u]);
#pragma unroll
    for (int u = 0; u < U; ++u)
      acc.add(Num<V>::mask(k + u * kBlock < it.e, Num<V>::mul(a[u], x[u])));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc.merge_xor(off);
  if ((tid & 63) == 0) sh.wave[tid >> 6][0] = acc;
  lds_barrier();
  if (tid == 0) {
    Acc<V> t = sh.wave[0][0];
    t.merge(sh.wave[1][0]);
    t.merge(sh.wave[2][0]);
    t.merge(sh.wave[3][0]);
    store(it.seg, t);
  }
  lds_barrier();
}

// One tile on its own (no overlap with neighbours): sparse dot products of
// its rows with NA vectors and the row epilogues. Called by the whole
// workgroup (every branch below is uniform over it).
template <typename V, int NA, typename Load, typename Finish>
__device__ __forceinline__ void spmv_tile(const WorkItem& it, gptr<const int32_t> rp,
                                          gptr<const int32_t> ci, gptr<const V> va,
                                          const gptr<const V>* vec, const double* div,
                                          Load&& load, Finish&& finish, SpmvShared<V, NA>& sh) {
  if (it.re <= it.rb) return;  // the placeholder tile of a side without rows
  if (it.lanes == 0) {
    long_row_tile<V, NA>(it, ci, va, vec, div, load, finish, sh);
    return;
  }
  using Pre = decltype(load(0));
  StreamTile<V, Pre> T;
  stream_load<V, Pre>(it, rp, ci, va, load, T);
  __builtin_amdgcn_sched_barrier(0);
  V x[NA][kK];
  stream_gather<V, NA, Pre>(it, T, vec, div, x);
  stream_finish<V, NA, Pre>(it, T, x, finish, sh);
}

template <typename V>
__device__ __forceinline__ V clampv(V v, V lo, V hi) {
  V t = v < lo ? lo : v;
  return t > hi ? hi : t;
}

// Whether an LP takes part in an evaluation step. The evaluation that opens
// a launch sequence serves every due LP; the guarded evaluations inside the
// sequence (mid) serve only LPs below their pause point, so a session paused
// at k_limit keeps the evaluation due there for its next run.
__device__ __forceinline__ bool eval_guard(const Ctl* c, int mid) {
  return c->status == kRunning && c->need_eval != 0 && (!mid || c->k < c->k_limit);
}

template <int NV>
__device__ __forceinline__ void dd_reset(DD (&v)[NV]) {
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = dd_zero();
}

// End of an LP's part of this workgroup's chunk: reduce the thread sums and
// store them in the LP's partial slot.
template <int NV, bool PLAIN = false>
__device__ __forceinline__ void flush_partials(DD (&p)[NV], DD* s_red, double* part, int stride,
                                               int slot) {
  block_sum<NV, kBlock / 64, PLAIN>(p, s_red);
  store_partials<NV>(part, stride, slot, p);
  dd_reset(p);
}

// Whether work item wi is the last of its LP in the chunk [i0, i0 + chunk)
// (an LP's items are consecutive in the list).
__device__ __forceinline__ bool last_of_lp(const WorkItem* work, int wi, int i0, int chunk,
                                           int lp) {
  return wi + 1 == i0 + chunk || work[wi + 1].lp != lp;
}

// ---------------------------------------------------------------------------
// scalar decisions (one workgroup per LP)
// ---------------------------------------------------------------------------

// Inputs of the step decision, read before the partial sums are merged so
// that their loads overlap those of the partials: the control-block fields
// it reads, the parameters it uses, and the step-rule factors
// (j+1)^-reduction and (j+1)^-growth of the attempt j it decides.
struct StepIn {
  double eta, omega, w, hp_norm, hd_norm;
  int64_t k, t, attempts, retries;
  int32_t cur;
  double lr;
  int64_t max_iter;
  int32_t phi, schedule, normalize, eval_every, max_retries, flags;
  double f_red, f_gro;
};

// Adaptive step rule (PDLP's): accept when eta <= eta_bar; the next step is
// min((1 - (j+1)^-red) eta_bar, (1 + (j+1)^-gro) eta), j counting attempts.
// c is the LP's control block (written here), in its fields as read before
// the decision; s holds the attempt's sums
// |x'-x|^2, |g|^2, |G^p|^2, |y'-y|^2, (y'-y).(A x'-A x), |b-Ax|^2, |G^d|^2.
// k mod d for k >= 0 and d >= 1: a 32-bit division while k fits in 32 bits
// (the 64-bit one is a long instruction sequence on the decision's serial path)
__device__ __forceinline__ int64_t mod_count(int64_t k, int32_t d) {
  return k <= (int64_t)INT32_MAX ? (int64_t)((uint32_t)k % (uint32_t)d) : k % d;
}

// Returns whether the decision made an evaluation due.
__device__ bool decide_step(Ctl& c, const StepIn& in, const double* s) {
  const double dx2 = s[0], g2 = s[1], gp2 = s[2];
  const double dy2 = s[3], inter = fabs(s[4]), r2 = s[5], gd2 = s[6];
  c.attempts = in.attempts + 1;
  // a numerical failure is reported by the next evaluation, on the current
  // iterate (the failed attempt is not committed)
  auto fail = [&]() {
    c.fail_pending = 1;
    c.need_eval = 1;
    return true;
  };
  if (!(isfinite(dx2) && isfinite(dy2) && isfinite(inter))) return fail();
  const double eta = in.eta, om = in.omega;
  const double movement = 0.5 * om * dx2 + 0.5 * dy2 / om;
  const double eta_bar = inter > 0.0 ? movement / inter : INFINITY;
  // the constant step (vanilla PDHG) accepts every attempt and keeps eta
  const bool constant = (in.flags & kConstantStep) != 0;
  double eta_next = eta;
  if (!constant) {
    const double first = (1.0 - in.f_red) * eta_bar;
    const double second = (1.0 + in.f_gro) * eta;
    eta_next = second < first ? second : first;
  }
  c.last_eta_bar = eta_bar;
  // a pending learner update was applied by this attempt's kernels
  c.learn_pending = 0;
  if (constant || eta <= eta_bar) {
    const bool learn = in.lr > 0.0 && mod_count(in.k, in.phi) == 0;
    const int64_t k1 = in.k + 1;
    c.eta_acc = eta;
    c.w = in.w + eta;
    c.k = k1;
    c.t = in.t + 1;
    c.cur = in.cur ^ 1;
    c.eta = eta_next;
    c.retries = 0;
    if (learn) {
      c.learn_pending = 1;
      c.g2 = g2;
      c.r2 = r2;
      c.gp2 = gp2;
      c.gd2 = gd2;
      if (in.schedule == 1) {  // AdaGrad on the norm: H += |G / scale|^2 = |G|^2 / scale^2
        const bool np = in.normalize && !(g2 > 0.0);
        const bool nd = in.normalize && !(r2 > 0.0);
        const double sp = in.normalize ? g2 : 1.0;
        const double sd = in.normalize ? r2 : 1.0;
        if (!np) c.hp_norm = in.hp_norm + gp2 / (sp * sp);
        if (!nd) c.hd_norm = in.hd_norm + gd2 / (sd * sd);
      }
    }
    c.learn_now = (in.lr > 0.0 && mod_count(k1, in.phi) == 0) ? 1 : 0;
    if (mod_count(k1, in.eval_every) == 0 || k1 >= in.max_iter) {
      c.need_eval = 1;
      return true;
    }
    return false;
  }
  const int64_t r1 = in.retries + 1;
  c.eta = eta_next;
  c.retries = r1;
  if (r1 > in.max_retries || !(eta_next > 0.0 && isfinite(eta_next))) return fail();
  return false;
}

__device__ __forceinline__ double wkkt(double rp2, double rd2, double gap, double om) {
  return sqrt(om * om * rp2 + rd2 / (om * om) + gap * gap);
}

// Evaluation parts: per iterate z (0 current, 1 average)
//   A^T side (6): |r_d|^2, |D_c^-1 r_d|^2, sum l lambda+, sum u lambda-, c^T x, |x - anchor|^2
//   A side   (4): |r_p|^2, |D_r^-1 r_p|^2, b^T y, |y - anchor|^2
constexpr int kEvT = 6;
constexpr int kEvA = 4;

// Termination, then PDLP's restart test (sufficient decay, necessary decay
// without progress, artificial), on the parts summed by the eval kernels.
__device__ void decide_eval(Ctl* c, const DevParams* p, const double* st, const double* sa) {
  const bool has_avg = c->w > 0.0;
  double rp2[2], rd2[2], pobj[2], dobj[2], dxa2[2], dya2[2], rel[2][4];
  for (int z = 0; z < 2; ++z) {
    const double* t = st + kEvT * z;
    const double* a = sa + kEvA * z;
    rd2[z] = t[0];
    const double rd2u = t[1];
    const double bound = t[2] - t[3];
    dxa2[z] = t[5];
    rp2[z] = a[0];
    const double rp2u = a[1];
    dya2[z] = a[3];
    pobj[z] = t[4] + p->c0;
    dobj[z] = (a[2] + bound) + p->c0;
    rel[z][0] = sqrt(rp2u) / (1.0 + p->b_norm);
    rel[z][1] = sqrt(rd2u) / (1.0 + p->c_norm);
    rel[z][2] = fabs(pobj[z] - dobj[z]) / (1.0 + fabs(pobj[z]) + fabs(dobj[z]));
    const double m01 = rel[z][0] > rel[z][1] ? rel[z][0] : rel[z][1];
    rel[z][3] = m01 > rel[z][2] ? m01 : rel[z][2];
  }
  if (c->fail_pending) {
    // numerical failure: the current iterate with its KKT, as it stands
    c->out_pobj = pobj[0];
    c->out_dobj = dobj[0];
    c->out_relp = rel[0][0];
    c->out_reld = rel[0][1];
    c->out_relg = rel[0][2];
    c->out_rel = rel[0][3];
    c->which = 0;
    c->need_eval = 0;
    c->status = kNumError;
    return;
  }
  if (!c->anchor_set) {
    c->anc_rp2 = rp2[0];
    c->anc_rd2 = rd2[0];
    c->anc_gap = pobj[0] - dobj[0];
    c->anchor_set = 1;
  }
  const int b = (has_avg && rel[1][3] < rel[0][3]) ? 1 : 0;
  c->out_pobj = pobj[b];
  c->out_dobj = dobj[b];
  c->out_relp = rel[b][0];
  c->out_reld = rel[b][1];
  c->out_relg = rel[b][2];
  c->out_rel = rel[b][3];
  c->which = b;
  c->need_eval = 0;
  const bool optimal = rel[b][3] <= p->tol;
  if (optimal || c->k >= p->max_iter || c->stop_request) {
    c->status = optimal ? kOptimal : (c->stop_request ? kTimeLimit : kIterLimit);
    c->finalize_avg = b;
    c->restart_w = c->w;
    return;
  }
  if (c->t > 0 && !(p->flags & kNoRestart)) {
    const double om = c->omega;
    const double kc = wkkt(rp2[0], rd2[0], pobj[0] - dobj[0], om);
    const double ka = has_avg ? wkkt(rp2[1], rd2[1], pobj[1] - dobj[1], om) : INFINITY;
    const double kanc = wkkt(c->anc_rp2, c->anc_rd2, c->anc_gap, om);
    const int z = ka < kc ? 1 : 0;
    const double cand = z ? ka : kc;
    const bool restart = cand <= p->beta_suff * kanc ||
                         (cand <= p->beta_nec * kanc && cand > c->prev_cand) ||
                         (double)c->t >= p->beta_art * (double)c->k;
    if (restart) {
      const double dxn = sqrt(dxa2[z]);
      const double dyn = sqrt(dya2[z]);
      if (dxn > 1e-10 && dyn > 1e-10) {
        // correctly rounded exp and log: the same bits on every platform
        const double th = p->pw_smoothing;
        c->omega = crm::cr_exp(th * crm::cr_log(dyn / dxn) + (1.0 - th) * crm::cr_log(om));
      }
      c->anc_rp2 = rp2[z];
      c->anc_rd2 = rd2[z];
      c->anc_gap = pobj[z] - dobj[z];
      c->restart_pending = 1;
      c->restart_avg = z;
      c->restart_w = c->w;
      c->w = 0.0;
      c->t = 0;
      c->prev_cand = INFINITY;
      c->restarts += 1;
    } else {
      c->prev_cand = cand;
    }
  }
}

// Work items of a chunk are staged in LDS, kItemWin at a time, so that a
// tile's start waits on LDS only: a work item loaded through the vector
// memory path would make the tile's first wait also wait for the previous
// tile's stores.
constexpr int kItemWin = 32;
constexpr int kItemWords = sizeof(WorkItem) / 4;
static_assert(sizeof(WorkItem) % 4 == 0, "work items are copied as 32-bit words");

// A value that is the same in every thread, moved to scalar registers. A
// pointer loaded once per LP then needs no wait where the tiles use it.
template <typename T>
__device__ __forceinline__ T uni(T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, v)));
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// The control-block fields a step kernel reads, fetched together through
// the global address space into scalar registers: every load is issued
// before the first branch on any of them, so they cost one round trip
// instead of one per branch.
struct CtlView {
  double eta, omega, g2, r2, hp_norm, hd_norm;
  int64_t k, k_limit;
  int32_t status, cur, need_eval, learn_pending, restart_pending, finalize_avg, learn_now,
      weighted_step;
  // running, no evaluation due, below the pause point
  __device__ __forceinline__ bool attempt() const {
    return (status == kRunning) & (need_eval == 0) & (k < k_limit);
  }
};

__device__ __forceinline__ CtlView ctl_view(const Ctl* c) {
  const gptr<const Ctl> g = gp(c);
  CtlView v;
  v.eta = uni(g->eta);
  v.omega = uni(g->omega);
  v.g2 = uni(g->g2);
  v.r2 = uni(g->r2);
  v.hp_norm = uni(g->hp_norm);
  v.hd_norm = uni(g->hd_norm);
  v.k = uni(g->k);
  v.k_limit = uni(g->k_limit);
  v.status = uni(g->status);
  v.cur = uni(g->cur);
  v.need_eval = uni(g->need_eval);
  v.learn_pending = uni(g->learn_pending);
  v.restart_pending = uni(g->restart_pending);
  v.finalize_avg = uni(g->finalize_avg);
  v.learn_now = uni(g->learn_now);
  v.weighted_step = uni(g->weighted_step);
  return v;
}

// The same work item in every thread, moved to scalar registers: the
// compiler then branches on its fields and divides by its lane count with
// scalar instructions.
__device__ __forceinline__ WorkItem uniform_item(const WorkItem& w) {
  WorkItem u;
  const uint64_t cp = reinterpret_cast<uint64_t>(w.ctl);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)cp);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(cp >> 32));
  u.ctl = reinterpret_cast<Ctl*>(((uint64_t)hi << 32) | lo);
  u.lp = __builtin_amdgcn_readfirstlane(w.lp);
  u.tile = __builtin_amdgcn_readfirstlane(w.tile);
  u.rb = __builtin_amdgcn_readfirstlane(w.rb);
  u.re = __builtin_amdgcn_readfirstlane(w.re);
  u.s = __builtin_amdgcn_readfirstlane(w.s);
  u.e = __builtin_amdgcn_readfirstlane(w.e);
  u.lanes = __builtin_amdgcn_readfirstlane(w.lanes);
  u.slot = __builtin_amdgcn_readfirstlane(w.slot);
  u.seg = __builtin_amdgcn_readfirstlane(w.seg);
  u.first = __builtin_amdgcn_readfirstlane(w.first);
  return u;
}

// A side's chunking as the launch sees it, in scalar registers.
struct SideChunks {
  int grid, chunk;
};

__device__ __forceinline__ SideChunks side_chunks(const Counts* counts, bool tside) {
  const gptr<const Counts> c = gp(counts);
  return SideChunks{uni(tside ? c->grid_t : c->grid_a), uni(tside ? c->chunk_t : c->chunk_a)};
}

// Partial sums of the tiles of one window of work items: the four waves'
// totals of each tile (lane 63 after wave_scan) and where the tile's sums
// go (null: the tile's LP did not run).
template <int NV>
struct TilePartials {
  DD w[kItemWin][kBlock / 64][NV];
  double* dst[kItemWin];
  int stride[kItemWin];
  int slot[kItemWin];
};

// Drives a workgroup over its chunk of a side's work list, running the
// sparse product of each tile with the row epilogues load / finish, which
// accumulate the tile's partial sums in p. When the LP changes,
// begin(item) loads the LP's context (the pointers rp, ci, va, vec refer
// to variables it sets) and returns whether the LP takes part; dest()
// gives the LP's partial array and stride; commit() issues the row stores
// the epilogues held back, after the tile's wave totals are in LDS and
// before the next item can change the LP. Every tile stores its own
// partial sums in its item's slot: each wave's totals go to LDS after the
// tile (no barrier), and once per window of items the four waves' totals
// of each tile are added in a fixed order and stored, after the barrier
// the window needs anyway.
template <typename V, int NA, int NV, bool PLAIN, typename Begin, typename Load, typename Finish,
          typename Dest, typename Commit, typename Piece>
__device__ __forceinline__ void run_chunk_spmv(const WorkItem* __restrict__ work, SideChunks sc,
                                               WorkItem* s_items, const gptr<const int32_t>& rp,
                                               const gptr<const int32_t>& ci,
                                               const gptr<const V>& va, const gptr<const V>* vec,
                                               const double* div, Begin&& begin, Load&& load,
                                               Finish&& finish, Dest&& dest, Commit&& commit,
                                               Piece&& piece, DD (&p)[NV], TilePartials<NV>& tp,
                                               SpmvShared<V, NA>& sh) {
  const int chi = chunk_index(sc.grid);
  if (chi < 0) return;
  const int chunk = sc.chunk;
  const int w0 = chi * chunk;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int lp = -1;
  bool run = false;
  for (int k0 = 0; k0 < chunk; k0 += kItemWin) {
    const int cnt = min(kItemWin, chunk - k0);
    {
      const gptr<const int32_t> src = gp(reinterpret_cast<const int32_t*>(work + w0 + k0));
      int32_t* dst = reinterpret_cast<int32_t*>(s_items);
      for (int q = threadIdx.x; q < cnt * kItemWords; q += kBlock) dst[q] = src[q];
    }
    lds_barrier();
    for (int k = 0; k < cnt; ++k) {
      const WorkItem it = uniform_item(s_items[k]);
      bool on = false;
      if (it.lp >= 0) {
        if (it.lp != lp) {
          lp = it.lp;
          run = begin(it);
        }
        if (run) {
          // a piece of a split row stores its sum (its partial slot gets zeros)
          if (it.lanes < 0)
            piece_tile<V, NA>(it, ci, va, vec, div, piece, sh);
          else
            spmv_tile<V, NA>(it, rp, ci, va, vec, div, load, finish, sh);
          wave_scan<NV, PLAIN>(p);
          if (lane == 63) {
#pragma unroll
            for (int q = 0; q < NV; ++q) tp.w[k][wave][q] = p[q];
          }
          dd_reset(p);
          commit();
          on = true;
        }
      }
      if (threadIdx.x == 0) {
        double* d;
        int sd;
        dest(d, sd);
        tp.dst[k] = on ? d : nullptr;
        tp.stride[k] = sd;
        tp.slot[k] = it.slot;
      }
    }
    lds_barrier();  // the window's partials are in LDS; its items are rewritten next
    for (int x = threadIdx.x; x < cnt * NV; x += kBlock) {
      const int k = x / NV, q = x - k * NV;
      double* d = tp.dst[k];
      if (d) {
        DD t = tp.w[k][0][q];
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) {
          if constexpr (PLAIN) t.hi += tp.w[k][w][q].hi;
          else t = dd_merge(t, tp.w[k][w][q]);
        }
        const gptr<double> g = gp(d);
        const size_t sd = (size_t)tp.stride[k], sl = (size_t)tp.slot[k];
        g[(2 * q) * sd + sl] = t.hi;
        g[(2 * q + 1) * sd + sl] = t.lo;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// One projected online-gradient step on one preconditioner entry
// (the learner of Algorithm 1): G / scale (scale = |g|^2 or |b - Ax|^2 when
// normalizing, else 1), then AdaGrad (diagonal or on the norm) or a
// constant rate, then the clamp at the floor.
template <typename V>
__device__ __forceinline__ V learn_elem(V Pv, V& Hv, V Graw, double scale, const DevParams* p,
                                        double hnorm) {
  const V gv = (V)((double)Graw / scale);
  V step;
  if (p->schedule == 0) {
    Hv = Hv + gv * gv;
    step = Hv > V(0) ? gv / sqrt(Hv) : V(0);
  } else if (p->schedule == 1) {
    step = hnorm > 0.0 ? (V)((double)gv / sqrt(hnorm)) : V(0);
  } else {
    step = gv;
  }
  const V pv = Pv - (V)p->lr * step;
  const V fl = (V)p->floor;
  return pv < fl ? fl : pv;
}

// Whether a pending learner update (pending != 0) touches a side whose
// loss norm is nrm (|g|^2 on the primal side, |b - Ax|^2 on the dual side),
// and its scale.
__device__ __forceinline__ bool learn_side(int pending, double nrm, const DevParams* p,
                                           double* scale) {
  if (!pending) return false;
  if (p->normalize && !(nrm > 0.0)) return false;
  *scale = p->normalize ? nrm : 1.0;
  return true;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_init_products(LaunchCfg cfg) {
  __shared__ SpmvShared<V, 1> sh;
  const double nodiv[1] = {0.0};
  const SideChunks sc = side_chunks(cfg.counts, false);
  const int ch = chunk_index(sc.grid);
  if (ch < 0) return;
  const int i0 = ch * sc.chunk;
  for (int wi = i0; wi < i0 + sc.chunk; ++wi) {
    const WorkItem it = cfg.work_a[wi];
    if (it.lp < 0) continue;
    const LpDev& lp = cfg.lps[it.lp];
    const int cur = it.ctl->cur;
    const gptr<V> Ax = gp(static_cast<V*>(lp.Ax[cur]));
    const gptr<const V> vecs[1] = {gp(static_cast<const V*>(lp.x[cur]))};
    spmv_tile<V, 1>(
        it, gp(lp.rp_a), gp(lp.ci_a), gp(static_cast<const V*>(lp.va_a)), vecs, nodiv,
        [&](int) { return 0; }, [&](int i, V (&acc)[1], int) { Ax[i] = acc[0]; }, sh);
  }
}

template <typename V>
struct PrimalPre {
  V c, x, T, l, u, xs, H, G;
};

// Context of the primal step for one LP (A^T y, eq. (6)'s primal update and
// projection, the running sum, the primal online gradient of eq. (7) and
// the deferred learner update of T), loaded once per LP by begin(). Every
// value begin() reads is the same in all threads: it is moved to scalar
// registers (uni) so the branches on it are uniform and the pointers stay
// out of vector registers.
template <typename V>
struct PrimalStep {
  // FP32 runs accumulate the partial sums in plain FP64 (see acc_prod)
  static constexpr bool kPlain = sizeof(V) == 4;
  const LpDev* lp = nullptr;
  const DevParams* prm = nullptr;
  Ctl* c = nullptr;
  gptr<const V> cc = nullptr, lo = nullptr, hi = nullptr, x = nullptr, xs = nullptr;
  gptr<V> T = nullptr, Hp = nullptr, xn = nullptr, xsn = nullptr, Gp = nullptr;
  // sources of the AdaGrad state read with the row: H and G on update
  // attempts, else a vector the row reads anyway (values unused), so the
  // loads need no branch
  gptr<const V> Hsrc = nullptr, Gsrc = nullptr;
  gptr<const V> vecs[1] = {nullptr};  // the gathered vector, y
  gptr<const int32_t> rp = nullptr, ci = nullptr;
  gptr<const V> va = nullptr;
  double* part_ = nullptr;
  int stride_ = 0;
  void* segp_ = nullptr;  // segment partials of split rows
  V tau = V(0), etav = V(0);
  bool learn = false, upd = false, wstep = false, lzero = false, noup = false;
  double lscale = 1.0, hnorm = 0.0;

  // first: this workgroup takes the LP's first item (it clears the flags
  // below)
  __device__ __forceinline__ bool begin(const LaunchCfg& cfg, Ctl* ctl, int lpi, int first,
                                        int force) {
    c = ctl;
    lp = &cfg.lps[lpi];
    // The LP's record and its control block do not depend on each other:
    // both are read before the first wait.
    const CtlView v = ctl_view(ctl);
    const gptr<const LpDev> L = gp(lp);
    const void* const pc = uni(L->c);
    const void* const pl = uni(L->l);
    const void* const pu = uni(L->u);
    void* const pT = uni(L->T);
    void* const pH = uni(L->Hp);
    void* const pG = uni(L->Gp);
    void* const px0 = uni(L->x[0]);
    void* const px1 = uni(L->x[1]);
    void* const ps0 = uni(L->xs[0]);
    void* const ps1 = uni(L->xs[1]);
    const void* const py0 = uni(L->y[0]);
    const void* const py1 = uni(L->y[1]);
    const int32_t* const prp = uni(L->rp_t);
    const int32_t* const pci = uni(L->ci_t);
    const void* const pva = uni(L->va_t);
    const DevParams* const pprm = uni(L->prm);
    double* const ppart = uni(L->part_t);
    const int pstride = uni(L->ntiles_t);
    void* const pseg = uni(L->segp_t);
    const int32_t pflags = uni(L->s_flags);
    // the restart / final copy of the evaluation step ran before this
    // launch; the workgroup with the LP's first item clears the flags
    if (first && threadIdx.x == 0 && (v.restart_pending | v.finalize_avg)) {
      c->restart_pending = 0;
      c->finalize_avg = 0;
    }
    if (!uni((int)(force || v.attempt()))) return false;
    const int cur = uni(v.cur);
    const double eta = uni(v.eta), om = uni(v.omega);
    tau = (V)(eta / om);
    etav = (V)eta;
    prm = uni(pprm);
    // a forced (timing) launch writes only the candidate buffers
    learn = uni((int)(!force && v.learn_now != 0)) != 0;
    wstep = uni(v.weighted_step) != 0;
    lscale = 1.0;
    upd = uni((int)(!force && v.learn_pending &&
                    learn_side(v.learn_pending, v.g2, prm, &lscale))) != 0;
    lscale = uni(lscale);
    hnorm = uni(v.hp_norm);
    cc = uni(gp(static_cast<const V*>(pc)));
    lo = uni(gp(static_cast<const V*>(pl)));
    hi = uni(gp(static_cast<const V*>(pu)));
    T = uni(gp(static_cast<V*>(pT)));
    Hp = uni(gp(static_cast<V*>(pH)));
    Gp = uni(gp(static_cast<V*>(pG)));
    x = uni(gp(static_cast<const V*>(cur ? px1 : px0)));
    xs = uni(gp(static_cast<const V*>(cur ? ps1 : ps0)));
    xn = uni(gp(static_cast<V*>(cur ? px0 : px1)));
    xsn = uni(gp(static_cast<V*>(cur ? ps0 : ps1)));
    vecs[0] = uni(gp(static_cast<const V*>(cur ? py1 : py0)));
    Hsrc = upd ? Hp : x;
    Gsrc = upd ? Gp : x;
    rp = uni(gp(prp));
    ci = uni(gp(pci));
    va = uni(gp(static_cast<const V*>(pva)));
    part_ = uni(ppart);
    stride_ = uni(pstride);
    segp_ = uni(pseg);
    lzero = (pflags & kLowerZero) != 0;
    noup = (pflags & kNoUpper) != 0;
    tau = uni(tau), etav = uni(etav);
    return true;
  }

  __device__ __forceinline__ PrimalPre<V> load(int j) const {
    PrimalPre<V> q;
    q.c = ldg(cc, (uint32_t)j);
    q.x = ldg(x, (uint32_t)j);
    q.T = ldg(T, (uint32_t)j);
    q.l = lzero ? V(0) : ldg(lo, (uint32_t)j);
    q.u = noup ? V(INFINITY) : ldg(hi, (uint32_t)j);
    q.xs = ldg(xs, (uint32_t)j);
    q.H = ldg(Hsrc, (uint32_t)j);
    q.G = ldg(Gsrc, (uint32_t)j);
    return q;
  }

  // The row epilogue's stores wait in registers until commit(), which runs
  // at the next row's epilogue or after the workgroup's partial sums are
  // stored: a store's data registers cannot be reused before the store
  // completes, so stores issued ahead of the reduction would make it wait
  // for them.
  mutable bool w_on = false;
  mutable int w_j = 0;
  mutable V w_x = V(0), w_xs = V(0), w_T = V(0), w_H = V(0), w_G = V(0);

  __device__ __forceinline__ void commit() const {
    if (!w_on) return;
    const uint32_t j = (uint32_t)w_j;
    if (upd) {
      stg(T, j, w_T);
      stg(Hp, j, w_H);
    }
    stg(xn, j, w_x);
    stg(xsn, j, w_xs);
    if (learn) stg(Gp, j, w_G);
    w_on = false;
  }

  // Row j with (A^T y)_j = aty: partials |x'-x|^2 (or its T^-1 norm),
  // |g|^2, |G^p|^2 into p; the row's new values go out at commit().
  __device__ __forceinline__ void finish(int j, V aty, PrimalPre<V>& q, DD (&p)[3]) const {
    commit();
    V Tj = q.T;
    V h = q.H;
    if (upd) Tj = learn_elem<V>(Tj, h, q.G, lscale, prm, hnorm);
    const V g = q.c - aty;
    const V xh = q.x - (tau * Tj) * g;
    const V xv = clampv(xh, q.l, q.u);
    const double dx = (double)xv - (double)q.x;
    // the movement of the step rule, optionally in the T^-1 norm
    const double tj = (double)Tj;
    const double wdx = !wstep ? dx : (tj > 0.0 ? dx / tj : 0.0);
    acc_prod<kPlain>(p[0], dx, wdx);
    acc_prod<kPlain>(p[1], (double)g, (double)g);
    V gp_ = V(0);
    if (learn) {
      const bool ind = (xh >= q.l) && (xh <= q.u);
      gp_ = ind ? -((tau * g) * g) : V(0);
      acc_prod<kPlain>(p[2], (double)gp_, (double)gp_);
    }
    w_on = true;
    w_j = j;
    w_x = xv;
    w_xs = q.xs + etav * xv;
    w_T = Tj;
    w_H = h;
    w_G = gp_;
  }

  __device__ __forceinline__ double* part() const { return part_; }
  __device__ __forceinline__ int stride() const { return stride_; }
  __device__ __forceinline__ void piece(int sid, const Acc<V>& a) const { seg_store(segp_, sid, a); }
};

template <typename V>
struct DualPre {
  V ax, b, y, ys, S, H, G;
  int8_t ineq;
};

// Context of the dual step for one LP (A x', the extrapolation, eq. (6)'s
// dual update and sign projection, the running sum, the dual online
// gradient of eq. (7) and the deferred learner update of Sigma).
template <typename V>
struct DualStep {
  static constexpr bool kPlain = sizeof(V) == 4;  // as in PrimalStep
  const LpDev* lp = nullptr;
  const DevParams* prm = nullptr;
  const Ctl* c = nullptr;
  gptr<const V> b = nullptr, y = nullptr, ys = nullptr, Ax = nullptr;
  gptr<V> S = nullptr, Hd = nullptr, yn = nullptr, ysn = nullptr, Axn = nullptr, Gd = nullptr;
  gptr<const V> Hsrc = nullptr, Gsrc = nullptr;  // as in PrimalStep
  gptr<const int8_t> sense = nullptr;
  gptr<const int32_t> rp = nullptr, ci = nullptr;
  gptr<const V> va = nullptr;
  gptr<const V> vecs[1] = {nullptr};  // the gathered vector, x'
  double* part_ = nullptr;
  int stride_ = 0;
  void* segp_ = nullptr;  // segment partials of split rows
  V sig = V(0), etav = V(0);
  bool learn = false, upd = false, wstep = false;
  double lscale = 1.0, hnorm = 0.0;

  __device__ __forceinline__ bool begin(const LaunchCfg& cfg, const Ctl* ctl, int lpi, int,
                                        int force) {
    c = ctl;
    lp = &cfg.lps[lpi];
    // as in PrimalStep: the LP's record and its control block are read
    // together, and uniform values live in scalar registers
    const CtlView v = ctl_view(ctl);
    const gptr<const LpDev> L = gp(lp);
    const void* const pb = uni(L->b);
    void* const pS = uni(L->S);
    void* const pH = uni(L->Hd);
    void* const pG = uni(L->Gd);
    void* const py0 = uni(L->y[0]);
    void* const py1 = uni(L->y[1]);
    void* const ps0 = uni(L->ys[0]);
    void* const ps1 = uni(L->ys[1]);
    void* const pa0 = uni(L->Ax[0]);
    void* const pa1 = uni(L->Ax[1]);
    const void* const px0 = uni(L->x[0]);
    const void* const px1 = uni(L->x[1]);
    const int8_t* const psense = uni(L->sense);
    const int32_t* const prp = uni(L->rp_a);
    const int32_t* const pci = uni(L->ci_a);
    const void* const pva = uni(L->va_a);
    const DevParams* const pprm = uni(L->prm);
    double* const ppart = uni(L->part_a);
    const int pstride = uni(L->ntiles_a);
    void* const pseg = uni(L->segp_a);
    if (!uni((int)(force || v.attempt()))) return false;
    const int cur = uni(v.cur);
    const double eta = uni(v.eta), om = uni(v.omega);
    sig = (V)(eta * om);
    etav = (V)eta;
    prm = uni(pprm);
    learn = uni((int)(!force && v.learn_now != 0)) != 0;
    wstep = uni(v.weighted_step) != 0;
    lscale = 1.0;
    upd = uni((int)(!force && v.learn_pending &&
                    learn_side(v.learn_pending, v.r2, prm, &lscale))) != 0;
    lscale = uni(lscale);
    hnorm = uni(v.hd_norm);
    b = uni(gp(static_cast<const V*>(pb)));
    S = uni(gp(static_cast<V*>(pS)));
    Hd = uni(gp(static_cast<V*>(pH)));
    Gd = uni(gp(static_cast<V*>(pG)));
    y = uni(gp(static_cast<const V*>(cur ? py1 : py0)));
    ys = uni(gp(static_cast<const V*>(cur ? ps1 : ps0)));
    Ax = uni(gp(static_cast<const V*>(cur ? pa1 : pa0)));
    yn = uni(gp(static_cast<V*>(cur ? py0 : py1)));
    ysn = uni(gp(static_cast<V*>(cur ? ps0 : ps1)));
    Axn = uni(gp(static_cast<V*>(cur ? pa0 : pa1)));
    // x' was written by this attempt's primal step into the other buffer
    vecs[0] = uni(gp(static_cast<const V*>(cur ? px0 : px1)));
    sense = uni(gp(psense));
    Hsrc = upd ? Hd : y;
    Gsrc = upd ? Gd : y;
    rp = uni(gp(prp));
    ci = uni(gp(pci));
    va = uni(gp(static_cast<const V*>(pva)));
    part_ = uni(ppart);
    stride_ = uni(pstride);
    segp_ = uni(pseg);
    sig = uni(sig), etav = uni(etav);
    return true;
  }

  __device__ __forceinline__ DualPre<V> load(int i) const {
    DualPre<V> q;
    q.ax = ldg(Ax, (uint32_t)i);
    q.b = ldg(b, (uint32_t)i);
    q.y = ldg(y, (uint32_t)i);
    q.ys = ldg(ys, (uint32_t)i);
    q.S = ldg(S, (uint32_t)i);
    q.ineq = ldg(sense, (uint32_t)i);
    q.H = ldg(Hsrc, (uint32_t)i);
    q.G = ldg(Gsrc, (uint32_t)i);
    return q;
  }

  // as in PrimalStep: the row's stores wait in registers until commit()
  mutable bool w_on = false;
  mutable int w_i = 0;
  mutable V w_y = V(0), w_ax = V(0), w_ys = V(0), w_S = V(0), w_H = V(0), w_G = V(0);

  __device__ __forceinline__ void commit() const {
    if (!w_on) return;
    const uint32_t i = (uint32_t)w_i;
    if (upd) {
      stg(S, i, w_S);
      stg(Hd, i, w_H);
    }
    stg(yn, i, w_y);
    stg(Axn, i, w_ax);
    stg(ysn, i, w_ys);
    if (learn) stg(Gd, i, w_G);
    w_on = false;
  }

  // Row i with (A x')_i = axn: partials |y'-y|^2 (or its Sigma^-1 norm),
  // (y'-y).(Ax'-Ax), |b-Ax|^2, |G^d|^2 into p; the row's new values go out
  // at commit().
  __device__ __forceinline__ void finish(int i, V axn, DualPre<V>& q, DD (&p)[4]) const {
    commit();
    V Si = q.S;
    V h = q.H;
    if (upd) Si = learn_elem<V>(Si, h, q.G, lscale, prm, hnorm);
    const V axbar = V(2) * axn - q.ax;
    const V rt = q.b - axbar;
    const V yh = q.y + (sig * Si) * rt;
    const bool ineq = q.ineq != 0;
    const V yv = (ineq && yh < V(0)) ? V(0) : yh;
    const double dy = (double)yv - (double)q.y;
    const double si = (double)Si;
    const double wdy = !wstep ? dy : (si > 0.0 ? dy / si : 0.0);
    acc_prod<kPlain>(p[0], dy, wdy);
    acc_prod<kPlain>(p[1], dy, (double)axn - (double)q.ax);
    const V r = q.b - q.ax;
    acc_prod<kPlain>(p[2], (double)r, (double)r);
    V gd = V(0);
    if (learn) {
      const bool ind = !ineq || yh >= V(0);
      gd = ind ? -((sig * r) * rt) : V(0);
      acc_prod<kPlain>(p[3], (double)gd, (double)gd);
    }
    w_on = true;
    w_i = i;
    w_y = yv;
    w_ax = axn;
    w_ys = q.ys + etav * yv;
    w_S = Si;
    w_H = h;
    w_G = gd;
  }

  __device__ __forceinline__ double* part() const { return part_; }
  __device__ __forceinline__ int stride() const { return stride_; }
  __device__ __forceinline__ void piece(int sid, const Acc<V>& a) const { seg_store(segp_, sid, a); }
};

// Chunking of a step kernel's tile list: fixed sets carry it in the launch
// arguments (no dependent load before the work items); the server's
// changing set reads the device-side counts.
// Makes each value live in a scalar register at this point. Kernel
// arguments read later behind branches would otherwise be loaded one
// cache line at a time, each load waiting for the branch before it.
template <typename T>
__device__ __forceinline__ void sgpr_ready1(const T& v) {
  asm volatile("" ::"s"(v));
}
template <typename... T>
__device__ __forceinline__ void sgpr_ready(const T&... v) {
  (sgpr_ready1(v), ...);
}

__device__ __forceinline__ SideChunks step_chunks(const LaunchCfg& cfg, bool tside) {
  const int fixed = cfg.step_fixed;
  const int g = tside ? cfg.sgrid_t : cfg.sgrid_a, ch = tside ? cfg.schunk_t : cfg.schunk_a;
  if (fixed) return SideChunks{g, ch};
  return side_chunks(cfg.counts, tside);
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_primal(LaunchCfg cfg, int force) {
  __shared__ SpmvShared<V, 1> sh;
  __shared__ TilePartials<3> tp;
  const double nodiv[1] = {0.0};
  DD p[3];
  dd_reset(p);
  PrimalStep<V> st;
  __shared__ WorkItem s_items[kItemWin];
  sgpr_ready(cfg.lps, cfg.step_t, cfg.counts, cfg.step_fixed, cfg.sgrid_t, cfg.schunk_t, force);
  run_chunk_spmv<V, 1, 3, PrimalStep<V>::kPlain>(
      cfg.step_t, step_chunks(cfg, true), s_items, st.rp, st.ci,
      st.va, st.vecs, nodiv,
      [&](const WorkItem& it) { return st.begin(cfg, it.ctl, it.lp, it.first, force); },
      [&](int j) { return st.load(j); },
      [&](int j, V (&acc)[1], PrimalPre<V>& q) { st.finish(j, acc[0], q, p); },
      [&](double*& d, int& sd) {
        d = st.part();
        sd = st.stride();
      },
      [&]() { st.commit(); }, [&](int sid, const Acc<V>& a) { st.piece(sid, a); }, p, tp, sh);
  st.commit();
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_dual(LaunchCfg cfg, int force) {
  __shared__ SpmvShared<V, 1> sh;
  __shared__ TilePartials<4> tp;
  const double nodiv[1] = {0.0};
  DD p[4];
  dd_reset(p);
  DualStep<V> st;
  __shared__ WorkItem s_items[kItemWin];
  sgpr_ready(cfg.lps, cfg.step_a, cfg.counts, cfg.step_fixed, cfg.sgrid_a, cfg.schunk_a, force);
  run_chunk_spmv<V, 1, 4, DualStep<V>::kPlain>(
      cfg.step_a, step_chunks(cfg, false), s_items, st.rp, st.ci,
      st.va, st.vecs, nodiv,
      [&](const WorkItem& it) { return st.begin(cfg, it.ctl, it.lp, it.first, force); },
      [&](int i) { return st.load(i); },
      [&](int i, V (&acc)[1], DualPre<V>& q) { st.finish(i, acc[0], q, p); },
      [&](double*& d, int& sd) {
        d = st.part();
        sd = st.stride();
      },
      [&]() { st.commit(); }, [&](int sid, const Acc<V>& a) { st.piece(sid, a); }, p, tp, sh);
  st.commit();
}

// Windowed step kernel (FP32): one workgroup of kWinBlock threads per
// windowed chunk. Each pass stages its vector ranges in LDS; then the
// pass's slices go to the waves in turn (slice j to wave j mod kWinWaves),
// each lane adding up its row's entries in order, gathering from LDS. A
// chunk of several passes adds each such sum to the row's total in LDS; a
// chunk of one pass keeps the sums in registers and writes them to LDS once
// the window is done with. A row has one lane in a pass, so every row sum is
// formed in one fixed order (the same for every grid and every co-resident
// LP). After the passes each thread runs the row epilogue for rows r0 + t,
// r0 + t + kWinBlock, ...
template <bool tside, typename Step, typename Pre, int NV>
__device__ __forceinline__ void win_chunk(const LaunchCfg& cfg, const WinItem* list, int nwin,
                                          int force) {
  extern __shared__ float wlds[];
  float* win = wlds;
  DD* s_red = reinterpret_cast<DD*>(wlds + kWinOneCap);
  const int chi = chunk_index(nwin);
  if (chi < 0) return;
  const WinItem it = list[chi];
  if (it.lp < 0) return;  // padding of the list to a multiple of 8
  // the window arrays' pointers are read with the step's context (one
  // round trip for both)
  const gptr<const LpDev> L = gp(&cfg.lps[it.lp]);
  const uint16_t* const pwc = tside ? L->wcol_t : L->wcol_a;
  const uint16_t* const pwl = tside ? L->wlane_t : L->wlane_a;
  const WinSlice* const pws = tside ? L->wslice_t : L->wslice_a;
  const void* const pwv = tside ? L->wval_t : L->wval_a;
  const WinPass* const ppass = tside ? L->wpass_t : L->wpass_a;
  const WinRange* const prange = tside ? L->wrange_t : L->wrange_a;
  Step st;
  if (!st.begin(cfg, it.ctl, it.lp, it.slot == 0, force)) return;
  const LpDev* lp = st.lp;
  const gptr<const uint16_t> wc = uni(gp(pwc));
  const gptr<const uint16_t> wl = uni(gp(pwl));
  const gptr<const WinSlice> slices = uni(gp(pws));
  const gptr<const float> wv = uni(gp(static_cast<const float*>(pwv)));
  const gptr<const WinPass> passes = uni(gp(ppass));
  const gptr<const WinRange> ranges = uni(gp(prange));
  const gptr<const float> vec = st.vecs[0];
  const int t = threadIdx.x;
  const int lane = t & (kWinSlice - 1);
  const int wave = __builtin_amdgcn_readfirstlane(t / kWinSlice);
  const int r0 = uni(it.r0), nrow = uni(it.r1 - it.r0), nseg = uni(it.nseg);
  __shared__ WinPass s_pass[kWinMaxPass];
  const int npass = min(uni(it.npass), kWinMaxPass);  // plans hold at most kWinMaxPass
  // A chunk of one pass keeps each slice's sums in registers until the
  // window is no longer needed and then writes them into its LDS; the row
  // sums of a chunk of several passes sit beside the window and add up.
  const bool one = npass == 1;
  float* const part = one ? wlds : wlds + kWinCap;
  if (t < npass) {
    const gptr<const WinPass> src = passes + (it.pass0 + t);
    s_pass[t] = WinPass{src->s0, src->s1, src->range0, src->nrange};
  }
  if (!one)
    for (int r = t; r < nrow + nseg; r += kWinBlock) part[r] = 0.f;
  // the first two rows' epilogue loads go out before the passes, so they
  // are in flight while the entries stream
  const int ra = min(t, nrow - 1), rb0 = min(t + kWinBlock, nrow - 1);
  Pre pa = st.load(r0 + ra);
  Pre pb = st.load(r0 + rb0);
  lds_barrier();
  float racc[kWinWaveSlices];
  int rrow[kWinWaveSlices];
#pragma unroll
  for (int j = 0; j < kWinWaveSlices; ++j) rrow[j] = kWinNoRow;
  constexpr int kU = 8;  // entries of a lane loaded together
  // A wave takes a pass's slices in turn. Each slice's first kU entries are
  // loaded while the previous slice is summed, or, for the pass's first
  // slice, while the window is staged (a lane's entries past kU load with
  // their own slice).
  // (the pass's slice records are copied to LDS at its start; the first
  // slice of each wave reads its record from memory, before that copy)
  __shared__ WinSlice s_sl[kWinRows / kWinSlice];
  auto head = [&](int sj, const WinSlice& rec, int& e0, int& len, int& row, float (&vv)[kU],
                  int (&cc)[kU]) {
    e0 = __builtin_amdgcn_readfirstlane(rec.e0);
    len = __builtin_amdgcn_readfirstlane(rec.len);
    row = ldg(wl, (uint32_t)(sj * kWinSlice + lane));
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool on = u < len;
      vv[u] = on ? ldg(wv, (uint32_t)(e0 + u * kWinSlice + lane)) : 0.f;
      cc[u] = on ? (int)ldg(wc, (uint32_t)(e0 + u * kWinSlice + lane)) : 0;
    }
  };
  for (int ps = 0; ps < npass; ++ps) {
    const int pr0 = s_pass[ps].range0, prn = s_pass[ps].nrange;
    const int sl0 = s_pass[ps].s0, sl1 = s_pass[ps].s1;
    int sj = sl0 + wave;
    int e0 = 0, len = 0, row = kWinNoRow;
    float vv[kU];
    int cc[kU];
    if (sj < sl1) {
      const gptr<const WinSlice> slp = slices + sj;
      head(sj, WinSlice{uni(slp->e0), uni(slp->len)}, e0, len, row, vv, cc);
    }
    // ranges start on bucket boundaries (multiples of 4 entries, here and
    // in the window), so they are copied 16 bytes at a time; only the
    // vector's last bucket can end on a partial group. The first two
    // groups of each thread in the pass's first range are loaded before the
    // barrier that ends the previous pass, so they arrive while it ends.
    using f32x4 = float __attribute__((ext_vector_type(4)));
    const int src0 = uni(ranges[pr0].src), len0 = uni(ranges[pr0].len);
    const bool early = (len0 >> 2) >= 2 * kWinBlock;
    f32x4 pf[2];
    if (early) {
      const gptr<const f32x4> v4 = reinterpret_cast<gptr<const f32x4>>(vec + src0);
      pf[0] = v4[t];
      pf[1] = v4[t + kWinBlock];
    }
    if (ps > 0) lds_barrier();  // the previous pass is done with the window and records
    for (int q = t; q < sl1 - sl0; q += kWinBlock) {
      const gptr<const WinSlice> slp = slices + (sl0 + q);
      s_sl[q] = WinSlice{slp->e0, slp->len};
    }
    int off = 0;
    for (int g = pr0; g < pr0 + prn; ++g) {
      const int src = ranges[g].src, glen = ranges[g].len;
      const gptr<const f32x4> v4 = reinterpret_cast<gptr<const f32x4>>(vec + src);
      f32x4* w4 = reinterpret_cast<f32x4*>(win + off);
      const int n4 = glen >> 2;
      int q = t;
      if (g == pr0 && early) {
        w4[t] = pf[0];
        w4[t + kWinBlock] = pf[1];
        q = t + 2 * kWinBlock;
      }
      for (; q + 3 * kWinBlock < n4; q += 4 * kWinBlock) {  // four loads in flight
        f32x4 a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = v4[q + u * kWinBlock];
#pragma unroll
        for (int u = 0; u < 4; ++u) w4[q + u * kWinBlock] = a[u];
      }
      for (; q < n4; q += kWinBlock) w4[q] = v4[q];
      for (q = (glen & ~3) + t; q < glen; q += kWinBlock) win[off + q] = ldg(vec, (uint32_t)(src + q));
      off += glen;
    }
    lds_barrier();
    // the wave's slices of the pass (at most kWinWaveSlices), unrolled so
    // that a chunk of one pass can keep each slice's sums in registers
#pragma unroll
    for (int j = 0; j < kWinWaveSlices; ++j) {
      if (sj >= sl1) break;
      const int nsj = sj + kWinWaves;
      int ne0 = 0, nlen = 0, nrow_ = kWinNoRow;
      float nvv[kU];
      int ncc[kU];
      if (nsj < sl1) head(nsj, s_sl[nsj - sl0], ne0, nlen, nrow_, nvv, ncc);
      float acc = 0.f;
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (u < len) acc += vv[u] * win[cc[u]];
      for (int k = kU; k < len; k += kU) {
        float tv[kU];
        int tc[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const bool on = k + u < len;
          tv[u] = on ? ldg(wv, (uint32_t)(e0 + (k + u) * kWinSlice + lane)) : 0.f;
          tc[u] = on ? (int)ldg(wc, (uint32_t)(e0 + (k + u) * kWinSlice + lane)) : 0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (k + u < len) acc += tv[u] * win[tc[u]];
      }
      if (one) {
        racc[j] = acc;
        rrow[j] = row;
      } else if (row != kWinNoRow) {
        part[row] += acc;
      }
      sj = nsj;
      e0 = ne0;
      len = nlen;
      row = nrow_;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        vv[u] = nvv[u];
        cc[u] = ncc[u];
      }
    }
  }
  lds_barrier();
  if (one) {  // the window is done with: its LDS takes the row sums
    for (int r = t; r < nrow + nseg; r += kWinBlock) part[r] = 0.f;  // rows without entries
    lds_barrier();
#pragma unroll
    for (int j = 0; j < kWinWaveSlices; ++j)
      if (rrow[j] != kWinNoRow) part[rrow[j]] = racc[j];
    lds_barrier();
  }
  DD p[NV];
  dd_reset(p);
  // the segments' partial row sums go out for the finishing kernel
  if (nseg > 0) {
    const gptr<float> sp = gp(static_cast<float*>(tside ? lp->segp_t : lp->segp_a));
    for (int q = t; q < nseg; q += kWinBlock) stg(sp, (uint32_t)(it.seg0 + q), part[nrow + q]);
  }
  // two rows per thread in flight: their vector loads are issued together
  for (int r = t; r < nrow; r += 2 * kWinBlock) {
    const int r2 = r + kWinBlock;
    const bool two = r2 < nrow;
    const bool first = r == t;
    Pre q0 = first ? pa : st.load(r0 + r);
    Pre q1 = first ? pb : st.load(r0 + (two ? r2 : r));
    st.finish(r0 + r, part[r], q0, p);
    if (two) st.finish(r0 + r2, part[r2], q1, p);
  }
  if (st.part() != nullptr) {  // (a product run stores rows only)
    block_sum<NV, kWinWaves, true>(p, s_red);
    store_partials<NV>(st.part(), st.stride(), it.slot, p);
  }
  st.commit();
}

// Segmented long rows: kSegLanes lanes per row. Lane l merges the row's
// partials l, l + kSegLanes, ... in order, the lanes combine in a fixed
// shuffle tree, and the row's first lane runs the row epilogue. The
// partials come from windowed chunks (FP32) and from the pieces of rows
// split in tiles (float in FP32 runs, double-double in FP64 runs).
template <typename V, typename Step, typename Pre, int NV>
__device__ __forceinline__ void seg_rows(const LaunchCfg& cfg, const SegItem* list, int nitems,
                                         bool tside, int force) {
  __shared__ DD s_red[4 * NV];
  const int chi = chunk_index(nitems);
  if (chi < 0) return;
  const SegItem it = list[chi];
  if (it.lp < 0) return;
  Step st;
  if (!st.begin(cfg, it.ctl, it.lp, it.slot == 0, force)) return;
  const LpDev* lp = st.lp;
  const void* const sp = uni(tside ? lp->segp_t : lp->segp_a);
  const gptr<const int32_t> srow = uni(gp(tside ? lp->srow_t : lp->srow_a));
  const gptr<const int32_t> sptr = uni(gp(tside ? lp->sptr_t : lp->sptr_a));
  const gptr<const int32_t> sids = uni(gp(tside ? lp->sids_t : lp->sids_a));
  DD p[NV];
  dd_reset(p);
  const int lane = (int)threadIdx.x % kSegLanes;
  const int q = it.s0 + (int)threadIdx.x / kSegLanes;
  const bool on = q < it.s1;
  const int qq = on ? q : it.s0;  // idle groups read row s0 and drop it
  const int row = ldg(srow, (uint32_t)qq);
  Pre pre = st.load(row);
  const int k0 = ldg(sptr, (uint32_t)qq), k1 = ldg(sptr, (uint32_t)(qq + 1));
  Acc<V> acc;
  acc.zero();
  // four partials of the lane in flight at a time, merged in order
  int k = k0 + lane;
  for (; k + 3 * kSegLanes < k1; k += 4 * kSegLanes) {
    int id[4];
    Acc<V> a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) id[u] = ldg(sids, (uint32_t)(k + u * kSegLanes));
#pragma unroll
    for (int u = 0; u < 4; ++u) seg_load(sp, id[u], a[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc.merge(a[u]);
  }
  for (; k < k1; k += kSegLanes) {
    Acc<V> a;
    seg_load(sp, ldg(sids, (uint32_t)k), a);
    acc.merge(a);
  }
  // xor offsets below kSegLanes stay inside the row's aligned lane group
#pragma unroll
  for (int off = kSegLanes / 2; off > 0; off >>= 1) acc.merge_xor(off);
  if (on && lane == 0) st.finish(row, (V)acc.value(), pre, p);
  if (st.part() != nullptr) {
    block_sum<NV, kBlock / 64, Step::kPlain>(p, s_red);
    store_partials<NV>(st.part(), st.stride(), it.slot, p);
  }
  st.commit();
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_primal_seg(LaunchCfg cfg, int force) {
  seg_rows<V, PrimalStep<V>, PrimalPre<V>, 3>(cfg, cfg.seg_t, cfg.nseg_t, true, force);
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_dual_seg(LaunchCfg cfg, int force) {
  seg_rows<V, DualStep<V>, DualPre<V>, 4>(cfg, cfg.seg_a, cfg.nseg_a, false, force);
}

// The opening evaluation's sparse products of an FP32 LP with windowed
// chunks, one vector at a time, through the step machinery (tiles, windowed
// chunks, segments): A^T y (WHICH 0) and A^T y_s / w (WHICH 1) over the rows
// of A^T, A x_s / w over the rows of A. A row's sum goes to the LP's
// product vector; no partial sums. The evaluation kernels then read the
// products instead of gathering per nonzero. Only LPs whose evaluation is
// due take part; a sum of the running sums is divided by w once per row
// (the tile evaluation divides each gathered entry: the two differ by
// FP32 rounding).
struct ProdPre {};

template <bool TSIDE, int WHICH>
struct ProdStep {
  static constexpr bool kPlain = true;
  const LpDev* lp = nullptr;
  gptr<const float> vecs[1] = {nullptr};
  gptr<const int32_t> rp = nullptr, ci = nullptr;
  gptr<const float> va = nullptr;
  gptr<float> out = nullptr;
  void* segp_ = nullptr;
  double w = 0.0;
  bool divide = false;

  __device__ __forceinline__ bool begin(const LaunchCfg& cfg, const Ctl* ctl, int lpi, int, int) {
    lp = &cfg.lps[lpi];
    const gptr<const LpDev> L = gp(lp);
    const gptr<const Ctl> g = gp(ctl);
    float* const po = uni(TSIDE ? (WHICH ? L->evp_t1 : L->evp_t0) : L->evp_a);
    const void* const pv0 = uni(TSIDE ? (WHICH ? L->ys[0] : L->y[0]) : L->xs[0]);
    const void* const pv1 = uni(TSIDE ? (WHICH ? L->ys[1] : L->y[1]) : L->xs[1]);
    const int32_t* const prp = uni(TSIDE ? L->rp_t : L->rp_a);
    const int32_t* const pci = uni(TSIDE ? L->ci_t : L->ci_a);
    const void* const pva = uni(TSIDE ? L->va_t : L->va_a);
    void* const pseg = uni(TSIDE ? L->segp_t : L->segp_a);
    const int status = uni(g->status), need = uni(g->need_eval), cur = uni(g->cur);
    const double wv = uni(g->w);
    if (!uni((int)(po != nullptr && status == kRunning && need != 0))) return false;
    out = uni(gp(po));
    vecs[0] = uni(gp(static_cast<const float*>(cur ? pv1 : pv0)));
    rp = uni(gp(prp));
    ci = uni(gp(pci));
    va = uni(gp(static_cast<const float*>(pva)));
    segp_ = uni(pseg);
    w = wv;
    divide = uni((int)((TSIDE ? WHICH == 1 : true) && wv > 0.0)) != 0;
    return true;
  }
  __device__ __forceinline__ ProdPre load(int) const { return ProdPre{}; }
  __device__ __forceinline__ void finish(int j, float sum, ProdPre&, DD (&)[1]) const {
    stg(out, (uint32_t)j, divide ? (float)((double)sum / w) : sum);
  }
  __device__ __forceinline__ void commit() const {}
  __device__ __forceinline__ double* part() const { return nullptr; }
  __device__ __forceinline__ int stride() const { return 0; }
  __device__ __forceinline__ void piece(int sid, const Acc<float>& a) const {
    seg_store(segp_, sid, a);
  }
};

template <bool TSIDE, int WHICH>
__global__ __launch_bounds__(kBlock) void k_prod_tiles(LaunchCfg cfg) {
  __shared__ SpmvShared<float, 1> sh;
  __shared__ TilePartials<1> tp;
  const double nodiv[1] = {0.0};
  DD p[1];
  dd_reset(p);
  ProdStep<TSIDE, WHICH> st;
  __shared__ WorkItem s_items[kItemWin];
  run_chunk_spmv<float, 1, 1, true>(
      TSIDE ? cfg.step_t : cfg.step_a, step_chunks(cfg, TSIDE), s_items, st.rp, st.ci, st.va,
      st.vecs, nodiv,
      [&](const WorkItem& it) { return st.begin(cfg, it.ctl, it.lp, it.first, 0); },
      [&](int j) { return st.load(j); },
      [&](int j, float (&acc)[1], ProdPre& q) { st.finish(j, acc[0], q, p); },
      [&](double*& d, int& sd) {
        d = st.part();
        sd = st.stride();
      },
      [&]() {}, [&](int sid, const Acc<float>& a) { st.piece(sid, a); }, p, tp, sh);
}

template <bool TSIDE, int WHICH>
__global__ __launch_bounds__(kWinBlock) void k_prod_win(LaunchCfg cfg) {
  win_chunk<TSIDE, ProdStep<TSIDE, WHICH>, ProdPre, 1>(cfg, TSIDE ? cfg.win_t : cfg.win_a,
                                                       TSIDE ? cfg.nwin_t : cfg.nwin_a, 0);
}

template <bool TSIDE, int WHICH>
__global__ __launch_bounds__(kBlock) void k_prod_seg(LaunchCfg cfg) {
  seg_rows<float, ProdStep<TSIDE, WHICH>, ProdPre, 1>(cfg, TSIDE ? cfg.seg_t : cfg.seg_a,
                                                      TSIDE ? cfg.nseg_t : cfg.nseg_a, TSIDE, 0);
}

__global__ __launch_bounds__(kWinBlock) void k_primal_win(LaunchCfg cfg, int force) {
  win_chunk<true, PrimalStep<float>, PrimalPre<float>, 3>(cfg, cfg.win_t, cfg.nwin_t, force);
}

__global__ __launch_bounds__(kWinBlock) void k_dual_win(LaunchCfg cfg, int force) {
  win_chunk<false, DualStep<float>, DualPre<float>, 4>(cfg, cfg.win_a, cfg.nwin_a, force);
}

// What the step decision needs from an LP's record, in scalar registers:
// pointers, partial-slot counts and the copies of the parameters it reads.
using DecideLp = DecideRec;

// Lane l's value of v (l uniform over the wave).
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ DecideLp decide_lp(const LpDev* rec) {
  const gptr<const LpDev> L = gp(rec);
  DecideLp d;
  d.ctl = uni(L->ctl);
  d.ring = uni((const double*)L->pow_ring);
  d.part_t = uni((const double*)L->part_t);
  d.part_a = uni((const double*)L->part_a);
  d.ntiles_t = uni(L->ntiles_t);
  d.ntiles_a = uni(L->ntiles_a);
  // slots of the step kernels (one per tile, then the windowed chunks)
  d.ns_t = uni(L->nslot_st);
  d.ns_a = uni(L->nslot_sa);
  d.lr = uni(L->s_lr);
  d.max_iter = uni(L->s_max_iter);
  d.phi = uni(L->s_phi);
  d.schedule = uni(L->s_schedule);
  d.normalize = uni(L->s_normalize);
  d.eval_every = uni(L->s_eval_every);
  d.max_retries = uni(L->s_max_retries);
  d.flags = uni(L->s_flags);
  return d;
}

// One workgroup per LP: the step decision of the attempt the step kernels
// just ran. The loads come in three rounds: the launch arguments; the LP
// count beside the first LP record (the launch grid never exceeds the LP
// table, and nothing the record points to is read before the count shows
// that the LP exists; a fixed set of one LP has its record in the launch
// arguments and skips this round); then the factor ring, the partial sums
// and the control block together. The factor of the attempt is read from
// the lane that holds it once the attempt count is known.
// One wave per SIMD: a single workgroup per LP runs this kernel, so the
// registers go to keeping the partial loads in flight at once.
// PLAIN: the step kernels' partials are plain FP64 sums (FP32 runs).
static_assert(kPowRing == 64, "lane l of a wave holds ring entries l and kPowRing + l");
template <bool PLAIN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_decide(
    LaunchCfg cfg) {
  __shared__ DD s_red[4 * 7];
  // all launch arguments in one round, the solo record's fields included
  const DecideRec& sr = cfg.solo_rec;
  sgpr_ready(cfg.lps, cfg.counts, cfg.solo, sr.ctl, sr.ring, sr.part_t, sr.part_a, sr.ntiles_t,
             sr.ntiles_a, sr.ns_t, sr.ns_a, sr.lr, sr.max_iter, sr.phi, sr.schedule,
             sr.normalize, sr.eval_every, sr.max_retries, sr.flags);
  int li = blockIdx.x;
  DecideLp d;
  int nlps;
  if (cfg.solo) {  // the record came with the launch arguments
    d = cfg.solo_rec;
    nlps = 1;
  } else {
    d = decide_lp(&cfg.lps[li]);
    nlps = uni(gp(cfg.counts)->nlps);
  }
  while (li < nlps) {
    const gptr<const Ctl> g = gp(d.ctl);
    StepIn in;
    in.lr = d.lr;
    in.max_iter = d.max_iter;
    in.phi = d.phi;
    in.schedule = d.schedule;
    in.normalize = d.normalize;
    in.eval_every = d.eval_every;
    in.max_retries = d.max_retries;
    in.flags = d.flags;
    // lane l of every wave reads ring entries l and kPowRing + l; they stay
    // in vector registers until after the partial sums
    const int lane = (int)threadIdx.x & 63;
    const double rv_red = gp(d.ring)[lane];
    const double rv_gro = gp(d.ring)[kPowRing + lane];
    int status = 0, need = 0;
    int64_t k_limit = 0, ring_base = 0;
    double sv[7];
    // the control block is read after the first round of partial loads is
    // issued, in the same round trip
    sum_partials2<3, 4, PLAIN>(d.part_t, d.ntiles_t, d.ns_t, d.part_a, d.ntiles_a, d.ns_a, sv, s_red,
                        [&]() {
                          // every load first, then the moves to scalar
                          // registers (each of which waits for its load)
                          const int st0 = g->status, ne0 = g->need_eval, cu0 = g->cur;
                          const int64_t kl0 = g->k_limit, rb0 = g->ring_base, k0 = g->k;
                          const int64_t t0 = g->t, at0 = g->attempts, re0 = g->retries;
                          const double et0 = g->eta, om0 = g->omega, w0 = g->w;
                          const double hp0 = g->hp_norm, hd0 = g->hd_norm;
                          status = uni(st0);
                          need = uni(ne0);
                          k_limit = uni(kl0);
                          ring_base = uni(rb0);
                          in.eta = uni(et0);
                          in.omega = uni(om0);
                          in.w = uni(w0);
                          in.hp_norm = uni(hp0);
                          in.hd_norm = uni(hd0);
                          in.k = uni(k0);
                          in.t = uni(t0);
                          in.attempts = uni(at0);
                          in.retries = uni(re0);
                          in.cur = uni(cu0);
                        });
    // the attempt decided here is j = attempts + 1, in the ring at
    // j - ring_base - 1 (the ring covers every attempt of the sequence);
    // the index is uniform, so its lane's values are read across the wave
    int64_t r = in.attempts - ring_base;
    r = r < 0 ? 0 : (r >= kPowRing ? kPowRing - 1 : r);
    in.f_red = lane_value(rv_red, (int)r);
    in.f_gro = lane_value(rv_gro, (int)r);
    if (status == kRunning && need == 0 && in.k < k_limit && threadIdx.x == 0) {
      if (decide_step(*d.ctl, in, sv)) {
        // the guarded evaluation steps ahead look for due LPs again
        const gptr<Counts> cn = gp(const_cast<Counts*>(cfg.counts));
        cn->hint[0] = 1;
        cn->hint[1] = 1;
      }
    }
    li += gridDim.x;
    if (li < nlps) {
      __syncthreads();  // s_red is reused by the next LP
      d = decide_lp(&cfg.lps[li]);
    }
  }
}

// Applies a pending learner update to every entry of T and Sigma without
// taking a step (used before the state of a paused solve is read).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_learn_flush(LaunchCfg cfg) {
  auto body = [&](const WorkItem& it, bool tside) {
    const LpDev& lp = cfg.lps[it.lp];
    const Ctl* c = it.ctl;
    double scale = 1.0;
    if (!learn_side(c->learn_pending, tside ? c->g2 : c->r2, lp.prm, &scale)) return;
    V* P = static_cast<V*>(tside ? lp.T : lp.S);
    V* H = static_cast<V*>(tside ? lp.Hp : lp.Hd);
    const V* G = static_cast<const V*>(tside ? lp.Gp : lp.Gd);
    const double hnorm = tside ? c->hp_norm : c->hd_norm;
    for (int r = it.rb + threadIdx.x; r < it.re; r += kBlock) {
      V h = H[r];
      P[r] = learn_elem<V>(P[r], h, G[r], scale, lp.prm, hnorm);
      H[r] = h;
    }
  };
  const SideChunks st = side_chunks(cfg.counts, true), sa = side_chunks(cfg.counts, false);
  const int b = blockIdx.x;
  if (b < st.grid)
    for (int wi = b * st.chunk; wi < (b + 1) * st.chunk; ++wi)
      if (cfg.work_t[wi].lp >= 0) body(cfg.work_t[wi], true);
  if (b < sa.grid)
    for (int wi = b * sa.chunk; wi < (b + 1) * sa.chunk; ++wi)
      if (cfg.work_a[wi].lp >= 0) body(cfg.work_a[wi], false);
}

// Reduced cost q = c - A^T y split by the variable's bound type into
// lambda (absorbed by the bounds) and the dual residual q - lambda.
__device__ __forceinline__ void reduced_cost(double q, int8_t bf, double& lam, double& rd) {
  const bool lf = bf & 1, uf = bf & 2;
  if (lf && uf) lam = q;
  else if (lf) lam = q > 0.0 ? q : 0.0;
  else if (uf) lam = q < 0.0 ? q : 0.0;
  else lam = 0.0;
  rd = q - lam;
}

// Entry of an evaluation kernel. Step `mid` of a launch sequence (0: the
// evaluation opening it, which always looks at every LP; b > 0: the b-th
// guarded step inside it) returns at once when its hint word is clear; the
// first kernel of each step (clear_next) clears the next step's word.
__device__ __forceinline__ bool eval_step_skips(const LaunchCfg& cfg, int mid, bool clear_next) {
  const gptr<Counts> cn = gp(const_cast<Counts*>(cfg.counts));
  if (clear_next && blockIdx.x == 0 && threadIdx.x == 0) cn->hint[(mid + 1) & 1] = 0;
  return mid != 0 && uni(cn->hint[mid & 1]) == 0;
}

// The evaluation's row terms (residuals, reduced costs, objectives,
// distances to the anchor) for the current iterate (z = 0) and the average
// (z = 1, when w > 0), added to double-double partials: over the rows of
// A^T (EvalT, given (A^T y)_j and (A^T y_avg)_j) and of A (EvalA, given
// (A x_avg)_i; A x of the current iterate is cached).
template <typename V>
struct EvalT {
  gptr<const V> cc, lo, hi, x, xs, xa;
  gptr<const double> dc;
  gptr<const int8_t> bfin;
  double w;
  bool has_avg;
  __device__ __forceinline__ EvalT(const LpDev& lp, const Ctl* c) {
    const int cur = c->cur;
    w = c->w;
    has_avg = w > 0.0;
    cc = gp(static_cast<const V*>(lp.c));
    lo = gp(static_cast<const V*>(lp.l));
    hi = gp(static_cast<const V*>(lp.u));
    x = gp(static_cast<const V*>(lp.x[cur]));
    xs = gp(static_cast<const V*>(lp.xs[cur]));
    xa = gp(static_cast<const V*>(lp.xa));
    dc = gp(lp.dc);
    bfin = gp(lp.bfin);
  }
  __device__ __forceinline__ void row(int j, const V (&acc)[2], DD* p) const {
    const double cj = (double)cc[j];
    const int8_t bf = bfin[j];
    const double lj = (double)lo[j], uj = (double)hi[j];
    const double xaj = (double)xa[j];
    // unrolled, so that the partials' indices are constants (a runtime
    // index would put them in scratch memory)
#pragma unroll
    for (int z = 0; z < 2; ++z) {
      if (z == 1 && !has_avg) break;
      const double xz = z == 0 ? (double)x[j] : (double)xs[j] / w;
      double lam, rd;
      reduced_cost(cj - (double)acc[z], bf, lam, rd);
      const double rdu = rd / dc[j];
      const double d = xz - xaj;
      DD* q = p + kEvT * z;
      dd_add_prod(q[0], rd, rd);
      dd_add_prod(q[1], rdu, rdu);
      if (bf & 1) dd_add_prod(q[2], lj, lam > 0.0 ? lam : 0.0);
      if (bf & 2) dd_add_prod(q[3], uj, lam < 0.0 ? -lam : 0.0);
      dd_add_prod(q[4], cj, xz);
      dd_add_prod(q[5], d, d);
    }
  }
};

template <typename V>
struct EvalA {
  gptr<const V> b, y, ys, ya, Ax;
  gptr<V> Axa;
  gptr<const double> dr;
  gptr<const int8_t> sense;
  double w;
  bool has_avg;
  __device__ __forceinline__ EvalA(const LpDev& lp, const Ctl* c) {
    const int cur = c->cur;
    w = c->w;
    has_avg = w > 0.0;
    b = gp(static_cast<const V*>(lp.b));
    y = gp(static_cast<const V*>(lp.y[cur]));
    ys = gp(static_cast<const V*>(lp.ys[cur]));
    ya = gp(static_cast<const V*>(lp.ya));
    Ax = gp(static_cast<const V*>(lp.Ax[cur]));
    Axa = gp(static_cast<V*>(lp.Axa));
    dr = gp(lp.dr);
    sense = gp(lp.sense);
  }
  __device__ __forceinline__ void row(int i, const V (&acc)[1], DD* p) const {
    const double bi = (double)b[i];
    const bool ineq = sense[i] != 0;
    const double yai = (double)ya[i];
    if (has_avg) Axa[i] = acc[0];
#pragma unroll
    for (int z = 0; z < 2; ++z) {  // unrolled: constant partial indices
      if (z == 1 && !has_avg) break;
      const double ax = z == 0 ? (double)Ax[i] : (double)acc[0];
      const double yz = z == 0 ? (double)y[i] : (double)ys[i] / w;
      double rp = bi - ax;
      if (ineq && rp < 0.0) rp = 0.0;
      const double rpu = rp / dr[i];
      const double d = yz - yai;
      DD* q = p + kEvA * z;
      dd_add_prod(q[0], rp, rp);
      dd_add_prod(q[1], rpu, rpu);
      dd_add_prod(q[2], bi, yz);
      dd_add_prod(q[3], d, d);
    }
  }
};

// Whether an LP's opening evaluation takes precomputed products (then
// k_eval_pre serves it and the tile kernels below skip it).
__device__ __forceinline__ bool eval_pre(const LpDev& lp, int mid, bool tside) {
  return mid == 0 && (tside ? lp.evp_t0 : lp.evp_a) != nullptr;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_eval_t(LaunchCfg cfg, int mid) {
  __shared__ SpmvShared<V, 2> sh;
  __shared__ DD s_red[4 * 2 * kEvT];
  if (eval_step_skips(cfg, mid, true)) return;
  DD p[2 * kEvT];
  dd_reset(p);
  const SideChunks sc = side_chunks(cfg.counts, true);
  const int ch = chunk_index(sc.grid);
  if (ch < 0) return;
  const int i0 = ch * sc.chunk;
  for (int wi = i0; wi < i0 + sc.chunk; ++wi) {
    const WorkItem it = cfg.work_t[wi];
    if (it.lp < 0) continue;
    // the evaluation's double-double sums do not depend on their order, so
    // the workgroup reduces an LP's part of the chunk once, into the slot of
    // the chunk's ordinal among those touching the LP
    const bool endc = last_of_lp(cfg.work_t, wi, i0, sc.chunk, it.lp);
    const Ctl* c = it.ctl;
    const LpDev& lp = cfg.lps[it.lp];
    if (!eval_guard(c, mid) || eval_pre(lp, mid, true)) {
      if (endc) dd_reset(p);
      continue;
    }
    const EvalT<V> E(lp, c);
    const gptr<const V> vecs[2] = {gp(static_cast<const V*>(lp.y[c->cur])),
                                   gp(static_cast<const V*>(lp.ys[c->cur]))};
    const double divs[2] = {0.0, E.has_avg ? E.w : -1.0};
    spmv_tile<V, 2>(it, gp(lp.rp_t), gp(lp.ci_t), gp(static_cast<const V*>(lp.va_t)), vecs,
                    divs, [&](int) { return 0; },
                    [&](int j, V (&acc)[2], int) { E.row(j, acc, p); }, sh);
    if (endc)
      flush_partials<2 * kEvT>(p, s_red, lp.part_t, lp.ntiles_t, ch - lp.item0_t / sc.chunk);
  }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_eval_a(LaunchCfg cfg, int mid) {
  __shared__ SpmvShared<V, 1> sh;
  __shared__ DD s_red[4 * 2 * kEvA];
  if (eval_step_skips(cfg, mid, false)) return;
  DD p[2 * kEvA];
  dd_reset(p);
  const SideChunks sc = side_chunks(cfg.counts, false);
  const int ch = chunk_index(sc.grid);
  if (ch < 0) return;
  const int i0 = ch * sc.chunk;
  for (int wi = i0; wi < i0 + sc.chunk; ++wi) {
    const WorkItem it = cfg.work_a[wi];
    if (it.lp < 0) continue;
    // as in k_eval_t: one reduction per LP and chunk
    const bool endc = last_of_lp(cfg.work_a, wi, i0, sc.chunk, it.lp);
    const Ctl* c = it.ctl;
    const LpDev& lp = cfg.lps[it.lp];
    if (!eval_guard(c, mid) || eval_pre(lp, mid, false)) {
      if (endc) dd_reset(p);
      continue;
    }
    const EvalA<V> E(lp, c);
    const gptr<const V> vecs[1] = {gp(static_cast<const V*>(lp.xs[c->cur]))};
    const double divs[1] = {E.has_avg ? E.w : -1.0};
    spmv_tile<V, 1>(it, gp(lp.rp_a), gp(lp.ci_a), gp(static_cast<const V*>(lp.va_a)), vecs,
                    divs, [&](int) { return 0; },
                    [&](int i, V (&acc)[1], int) { E.row(i, acc, p); }, sh);
    if (endc)
      flush_partials<2 * kEvA>(p, s_red, lp.part_a, lp.ntiles_a, ch - lp.item0_a / sc.chunk);
  }
}

// The opening evaluation of LPs with precomputed products (FP32 windowed
// LPs), streaming: the workgroups keep the evaluation lists' chunking, and
// a workgroup whose chunk is the s-th of the nslot touching an LP takes the
// s-th of nslot equal row ranges of that LP, a thread per row, and stores
// slot s (the slots the tile kernels would fill, the same total).
template <bool TSIDE>
__global__ __launch_bounds__(kBlock) void k_eval_pre(LaunchCfg cfg) {
  constexpr int NV = TSIDE ? 2 * kEvT : 2 * kEvA;
  __shared__ DD s_red[4 * NV];
  // the tile kernel of this side may not run (every LP of the set served
  // here): the A^T one clears the next guarded step's hint as it would
  (void)eval_step_skips(cfg, 0, TSIDE);
  const SideChunks sc = side_chunks(cfg.counts, TSIDE);
  const int ch = chunk_index(sc.grid);
  if (ch < 0) return;
  const WorkItem* work = TSIDE ? cfg.work_t : cfg.work_a;
  const int i0 = ch * sc.chunk;
  int prev = -1;
  for (int wi = i0; wi < i0 + sc.chunk; ++wi) {
    const int lpi = uni(work[wi].lp);
    if (lpi < 0 || lpi == prev) continue;  // an LP's items are consecutive
    prev = lpi;
    const LpDev& lp = cfg.lps[lpi];
    const Ctl* c = lp.ctl;
    if (!uni((int)(eval_guard(c, 0) && eval_pre(lp, 0, TSIDE)))) continue;
    const int c0 = (TSIDE ? lp.item0_t : lp.item0_a) / sc.chunk;
    const int ns = TSIDE ? lp.nslot_t : lp.nslot_a;
    const int slot = ch - c0;
    const int64_t rows = TSIDE ? lp.n : lp.m;
    const int r0 = (int)(rows * slot / ns), r1 = (int)(rows * (slot + 1) / ns);
    DD p[NV];
    dd_reset(p);
    if constexpr (TSIDE) {
      const EvalT<float> E(lp, c);
      const gptr<const float> e0 = gp(static_cast<const float*>(lp.evp_t0));
      const gptr<const float> e1 = gp(static_cast<const float*>(lp.evp_t1));
      for (int j = r0 + (int)threadIdx.x; j < r1; j += kBlock) {
        const float acc[2] = {ldg(e0, (uint32_t)j), ldg(e1, (uint32_t)j)};
        E.row(j, acc, p);
      }
      flush_partials<NV>(p, s_red, lp.part_t, lp.ntiles_t, slot);
    } else {
      const EvalA<float> E(lp, c);
      const gptr<const float> e = gp(static_cast<const float*>(lp.evp_a));
      for (int i = r0 + (int)threadIdx.x; i < r1; i += kBlock) {
        const float acc[1] = {ldg(e, (uint32_t)i)};
        E.row(i, acc, p);
      }
      flush_partials<NV>(p, s_red, lp.part_a, lp.ntiles_a, slot);
    }
  }
}

// One workgroup per LP: termination and restart decision of an evaluation.
// The evaluation that opens a launch sequence (mid == 0) also fills the
// step-rule factor ring for the sequence; the guarded ones inside it
// (mid = 1, 2, ...) leave the ring alone (it already covers every attempt
// of the sequence).
__global__ __launch_bounds__(kBlock) void k_eval_decide(LaunchCfg cfg, int mid) {
  __shared__ DD s_red[4 * 2 * kEvT];
  if (eval_step_skips(cfg, mid, false)) return;
  const int nlps = cfg.counts->nlps;
  for (int li = blockIdx.x; li < nlps; li += gridDim.x) {
    const LpDev& lp = cfg.lps[li];
    Ctl* c = lp.ctl;
    if (c->status != kRunning) continue;
    if (mid) {
      if (!eval_guard(c, 1)) continue;
      double st[2 * kEvT], sa[2 * kEvA];
      sum_partials<2 * kEvT>(lp.part_t, lp.ntiles_t, lp.nslot_t, st, s_red);
      sum_partials<2 * kEvA>(lp.part_a, lp.ntiles_a, lp.nslot_a, sa, s_red);
      if (threadIdx.x == 0) decide_eval(c, lp.prm, st, sa);
      __syncthreads();
      continue;
    }
    // step-rule factors for the attempts j = a0 + 1 .. a0 + kPowRing of this
    // launch sequence (which holds at most kPowRing attempts): the host
    // table's values while it covers j, else the same correctly rounded
    // powers computed here. The step decision reads the whole ring beside
    // its partial sums.
    const int64_t a0 = c->attempts;
    const DevParams* p = lp.prm;
    for (int t = threadIdx.x; t < kPowRing; t += kBlock) {
      const int64_t j = a0 + 1 + t;
      if (j <= kPowTab) {
        lp.pow_ring[t] = lp.pow_tab[j - 1];
        lp.pow_ring[kPowRing + t] = lp.pow_tab[kPowTab + j - 1];
      } else {
        const double j1 = (double)j + 1.0;
        lp.pow_ring[t] = crm::cr_pow(j1, -p->step_reduction);
        lp.pow_ring[kPowRing + t] = crm::cr_pow(j1, -p->step_growth);
      }
    }
    if (threadIdx.x == 0) c->ring_base = a0;
    if (!eval_guard(c, 0)) continue;
    double st[2 * kEvT], sa[2 * kEvA];
    sum_partials<2 * kEvT>(lp.part_t, lp.ntiles_t, lp.nslot_t, st, s_red);
    sum_partials<2 * kEvA>(lp.part_a, lp.ntiles_a, lp.nslot_a, sa, s_red);
    if (threadIdx.x == 0) decide_eval(c, lp.prm, st, sa);
    __syncthreads();
  }
}

// Restart application or the final copy of the returned average. The
// flags stay set until the next k_primal clears them, and restarting to the
// average reads the sums it then clears, so this kernel runs exactly once
// per evaluation step, right before attempt slots (every evaluation step of
// a launch sequence, the guarded ones included, is followed by at least one
// attempt slot before the next).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_apply(LaunchCfg cfg, int mid) {
  if (eval_step_skips(cfg, mid, false)) return;
  auto body = [&](const WorkItem& it, bool tside) {
    const Ctl* c = it.ctl;
    const bool restart = c->restart_pending != 0;
    const bool fin = c->finalize_avg != 0;
    if (!restart && !fin) return;
    const LpDev& lp = cfg.lps[it.lp];
    const int cur = c->cur;
    const bool to_avg = restart ? (c->restart_avg != 0) : true;
    const double w = c->restart_w;
    if (tside) {
      V* x = static_cast<V*>(lp.x[cur]);
      V* xs = static_cast<V*>(lp.xs[cur]);
      V* xa = static_cast<V*>(lp.xa);
      for (int j = it.rb + threadIdx.x; j < it.re; j += kBlock) {
        V xv = x[j];
        if (to_avg) {
          xv = (V)((double)xs[j] / w);
          x[j] = xv;
        }
        if (restart) {
          xa[j] = xv;
          xs[j] = V(0);
        }
      }
    } else {
      V* y = static_cast<V*>(lp.y[cur]);
      V* ys = static_cast<V*>(lp.ys[cur]);
      V* ya = static_cast<V*>(lp.ya);
      V* Ax = static_cast<V*>(lp.Ax[cur]);
      const V* Axa = static_cast<const V*>(lp.Axa);
      for (int i = it.rb + threadIdx.x; i < it.re; i += kBlock) {
        V yv = y[i];
        if (to_avg) {
          yv = (V)((double)ys[i] / w);
          y[i] = yv;
          if (restart) Ax[i] = Axa[i];
        }
        if (restart) {
          ya[i] = yv;
          ys[i] = V(0);
        }
      }
    }
  };
  const SideChunks st = side_chunks(cfg.counts, true), sa = side_chunks(cfg.counts, false);
  const int b = blockIdx.x;
  if (b < st.grid)
    for (int wi = b * st.chunk; wi < (b + 1) * st.chunk; ++wi)
      if (cfg.work_t[wi].lp >= 0) body(cfg.work_t[wi], true);
  if (b < sa.grid)
    for (int wi = b * sa.chunk; wi < (b + 1) * sa.chunk; ++wi)
      if (cfg.work_a[wi].lp >= 0) body(cfg.work_a[wi], false);
}

// Gathers every LP's control block into one array, so the host reads the
// state of a whole set with one copy.
__global__ __launch_bounds__(kBlock) void k_board(LaunchCfg cfg) {
  constexpr int kWords = sizeof(Ctl) / 8;
  static_assert(sizeof(Ctl) % 8 == 0, "Ctl is copied as 64-bit words");
  const int nlps = uni(gp(cfg.counts)->nlps);
  for (int li = blockIdx.x; li < nlps; li += gridDim.x) {
    const gptr<const uint64_t> src = gp(reinterpret_cast<const uint64_t*>(cfg.lps[li].ctl));
    const gptr<uint64_t> dst = gp(reinterpret_cast<uint64_t*>(cfg.board + li));
    for (int w = threadIdx.x; w < kWords; w += kBlock) dst[w] = src[w];
  }
}

}  // namespace

thread_local hipError_t g_last_device_error = hipSuccess;

const char* device_error_string() { return hipGetErrorString(g_last_device_error); }

static int launched() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_last_device_error = e;
    return -1;
  }
  return 0;
}

#define OPDHG_LAUNCH(kernel, grid, ...)                                                   \
  do {                                                                                    \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, __VA_ARGS__); \
    return launched();                                                                    \
  } while (0)

template <typename V>
int Kernels<V>::init_products(const LaunchCfg& c, void* stream) {
  OPDHG_LAUNCH(k_init_products<V>, c.launch_a, c);
}
template <typename V>
int Kernels<V>::primal(const LaunchCfg& c, void* stream, int force) {
  OPDHG_LAUNCH(k_primal<V>, c.step_fixed ? c.sgrid_t : c.launch_t, c, force);
}
template <typename V>
int Kernels<V>::dual(const LaunchCfg& c, void* stream, int force) {
  OPDHG_LAUNCH(k_dual<V>, c.step_fixed ? c.sgrid_a : c.launch_a, c, force);
}
// ---------------------------------------------------------------------------
// device-side preparation (FP64)
// ---------------------------------------------------------------------------

// The host's double-double accumulator, operation for operation (the
// preparation on either side gives the same bits).
struct SeqDD {
  double hi = 0.0, lo = 0.0;
  __device__ __forceinline__ void add(double x) {
    const double s = hi + x;
    const double bb = s - hi;
    lo += (hi - (s - bb)) + (x - bb);
    hi = s;
  }
  __device__ __forceinline__ void add_prod(double a, double b) {
    const double p = a * b;
    add(p);
    lo += fma(a, b, -p);
  }
  __device__ __forceinline__ double value() const { return hi + lo; }
};

// Row statistics of |a~_ij| = |a_ij| d_r,i d_c,j over the rows of A
// (tside 0) or of A^T (tside 1, a row per column of A), one thread per row,
// entries in stored order.
__global__ __launch_bounds__(kBlock) void k_prep_stats(PrepCfg a, int tside, int kind, double e) {
  const int rows = tside ? a.n : a.m;
  const int32_t* rp = tside ? a.rp_t : a.rp_a;
  const int32_t* ci = tside ? a.ci_t : a.ci_a;
  const double* raw = tside ? a.raw_t : a.raw_a;
  double* out = tside ? a.sc : a.sr;
  auto scaled = [&](int r, int k) {
    const double v = fabs(raw[k]);
    return tside ? (v * a.dr[ci[k]]) * a.dc[r] : (v * a.dr[r]) * a.dc[ci[k]];
  };
  int r_first = 0;
  if (kind == 0) {
    // maxima do not depend on the order: a wave per long row (the first
    // rows in device order), then a thread per row for the rest
    const int nlong = tside ? a.nlong_t : a.nlong_a;
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * (kBlock / 64);
    for (int r = (blockIdx.x * kBlock + threadIdx.x) >> 6; r < nlong; r += nw) {
      double mx = 0.0;
      for (int k = rp[r] + lane; k < rp[r + 1]; k += 64) {
        const double x = scaled(r, k);
        mx = mx < x ? x : mx;
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(mx, off, 64);
        mx = mx < o ? o : mx;
      }
      if (lane == 0) out[r] = mx;
    }
    r_first = nlong;
  }
  for (int r = r_first + blockIdx.x * kBlock + threadIdx.x; r < rows; r += gridDim.x * kBlock) {
    double mx = 0.0;
    SeqDD acc;
    for (int k = rp[r]; k < rp[r + 1]; ++k) {
      const double x = scaled(r, k);
      if (kind == 0) mx = mx < x ? x : mx;
      else if (kind == 1) acc.add(e == 1.0 ? x : pow(x, e));
      else acc.add(x * x);
    }
    out[r] = kind == 0 ? mx : (kind == 1 ? acc.value() : sqrt(acc.value()));
  }
}

// Power iteration on A~^T A~ for |A~|_2 (vanilla PDHG's constant step
// needs tau sigma |A~|_2^2 < 1, Section 2), round by round as on the host:
// v_0 = 1 / sqrt(n); each round forms av = A~ v and w = A~^T av, each row's
// products added one at a time in stored order in double-double and
// rounded once, with the entries formed from the raw values and the
// diagonals by the host's expression; then lam = |w| and v = w / lam. It
// stops after power_iters rounds, when lam moves by at most
// power_tol * lam, or when w = 0. av lives in sr, w in sc, and v = w / lam
// is formed where it is read. The rounds after the stop return at once.
constexpr int kPwLam = 4 * kPrepGrid + 3, kPwDone = kPwLam + 1, kPwZero = kPwLam + 2;

__global__ __launch_bounds__(kBlock) void k_power_av(PrepCfg a, int round) {
  if (round == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.scr[kPwLam] = 0.0;
      a.scr[kPwDone] = 0.0;
      a.scr[kPwZero] = 0.0;
    }
  } else if (a.scr[kPwDone] != 0.0) {
    return;
  }
  const double lam = round ? a.scr[kPwLam] : 1.0;
  const double v0 = 1.0 / sqrt((double)a.n);
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < a.m; r += gridDim.x * kBlock) {
    SeqDD acc;
    for (int k = a.rp_a[r]; k < a.rp_a[r + 1]; ++k) {
      const int c = a.ci_a[k];
      const double sv = (a.raw_a[k] * a.dr[r]) * a.dc[c];
      acc.add_prod(sv, round ? a.sc[c] / lam : v0);
    }
    a.sr[r] = acc.value();
  }
}

// w = A~^T av (sc), and per-workgroup double-double partials of |w|^2 in
// scr (kPrepGrid workgroups).
__global__ __launch_bounds__(kBlock) void k_power_w(PrepCfg a, int round) {
  __shared__ DD s_red[4];
  if (round > 0 && a.scr[kPwDone] != 0.0) return;
  DD p[1];
  p[0] = dd_zero();
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < a.n; j += gridDim.x * kBlock) {
    SeqDD acc;
    for (int k = a.rp_t[j]; k < a.rp_t[j + 1]; ++k) {
      const int i = a.ci_t[k];
      const double sv = (a.raw_t[k] * a.dr[i]) * a.dc[j];
      acc.add_prod(sv, a.sr[i]);
    }
    const double w = acc.value();
    a.sc[j] = w;
    dd_add_prod(p[0], w, w);
  }
  block_sum<1>(p, s_red);
  if (threadIdx.x == 0) {
    a.scr[2 * blockIdx.x + 0] = p[0].hi;
    a.scr[2 * blockIdx.x + 1] = p[0].lo;
  }
}

// lam = |w| and the stopping test of the round (one thread).
__global__ void k_power_step(PrepCfg a, int round) {
  if (threadIdx.x != 0 || (round > 0 && a.scr[kPwDone] != 0.0)) return;
  DD t = dd_zero();
  for (int g = 0; g < kPrepGrid; ++g) t = dd_merge(t, DD{a.scr[2 * g], a.scr[2 * g + 1]});
  const double lam_new = sqrt(dd_value(t));
  if (lam_new == 0.0) {
    a.scr[kPwZero] = 1.0;
    a.scr[kPwDone] = 1.0;
    return;
  }
  const double lam = a.scr[kPwLam];
  const bool done = fabs(lam_new - lam) <= a.power_tol * lam_new;
  a.scr[kPwLam] = lam_new;
  if (done) a.scr[kPwDone] = 1.0;
}

// eta0 = step_scale / |A~|_2 (step_scale when the norm is 0) into the
// control block and the scalars read back by the host.
__global__ void k_power_final(PrepCfg a) {
  if (threadIdx.x != 0) return;
  const double nu = a.scr[kPwZero] != 0.0 ? 0.0 : sqrt(a.scr[kPwLam]);
  const double eta0 = nu > 0.0 ? a.step_scale / nu : a.step_scale;
  a.ctl->eta = eta0;
  a.scr[4 * kPrepGrid + 1] = eta0;
}

// d_r /= sqrt(s_r), d_c /= sqrt(s_c), a zero statistic read as 1.
__global__ __launch_bounds__(kBlock) void k_prep_apply(PrepCfg a) {
  const int tot = a.m + a.n;
  for (int q = blockIdx.x * kBlock + threadIdx.x; q < tot; q += gridDim.x * kBlock) {
    if (q < a.m) a.dr[q] = a.dr[q] / sqrt(a.sr[q] == 0.0 ? 1.0 : a.sr[q]);
    else {
      const int j = q - a.m;
      a.dc[j] = a.dc[j] / sqrt(a.sc[j] == 0.0 ? 1.0 : a.sc[j]);
    }
  }
}

// ---- device-side structure ----

// Rows of A to device order; each entry also to its A^T row's cursor. A
// wave per row of more than 256 entries (the first rows in device order),
// a thread per row for the rest.
__global__ __launch_bounds__(kBlock) void k_struct_rows(StructCfg a) {
  auto entry = [&](int i, int64_t k, int d) {
    const int j2 = a.inv_t[a.src_ci[k]];
    a.ci_a[d] = j2;
    a.raw_a[d] = a.src_val[k];
    const int q = atomicAdd(&a.cur[j2], 1);
    a.tmp_i[q] = i;
    a.tmp_k[q] = (int)k;
  };
  const int lane = threadIdx.x & 63;
  const int w0 = (blockIdx.x * kBlock + threadIdx.x) >> 6, nw = gridDim.x * (kBlock / 64);
  for (int i2 = w0; i2 < a.nlong_a; i2 += nw) {
    const int i = a.perm_a[i2];
    const int64_t s = a.src_rp[i], e = a.src_rp[i + 1];
    for (int64_t k = s + lane; k < e; k += 64) entry(i, k, a.rp_a[i2] + (int)(k - s));
  }
  const int t0 = blockIdx.x * kBlock + threadIdx.x, nt = gridDim.x * kBlock;
  for (int i2 = a.nlong_a + t0; i2 < a.m; i2 += nt) {
    const int i = a.perm_a[i2];
    const int64_t s = a.src_rp[i], e = a.src_rp[i + 1];
    const int d0 = a.rp_a[i2];
    for (int64_t k = s; k < e; ++k) entry(i, k, d0 + (int)(k - s));
  }
}

// Each A^T row in ascending original row: an entry's place is its rank
// among the row's original rows (distinct: A has no duplicate entry). A
// wave per row of more than 32 entries (first in device order), with the
// row's original rows in LDS; a thread per row for the rest.
__global__ __launch_bounds__(kBlock) void k_struct_cols(StructCfg a) {
  __shared__ int32_t s_rows[kBlock / 64][kStructMaxCol];
  auto place = [&](int s, int p, int ip, int rank) {
    const int d = s + rank;
    a.ci_t[d] = a.inv_a[ip];
    a.raw_t[d] = a.src_val[a.tmp_k[p]];
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int w0 = blockIdx.x * (kBlock / 64) + wave, nw = gridDim.x * (kBlock / 64);
  int32_t* rows = s_rows[wave];
  for (int j2 = w0; j2 < a.nmed_t; j2 += nw) {
    const int s = a.rp_t[j2];
    const int L = min(a.rp_t[j2 + 1] - s, kStructMaxCol);  // the host checked L <= kStructMaxCol
    for (int p = lane; p < L; p += 64) rows[p] = a.tmp_i[s + p];
    // the wave's LDS writes before its reads (DS instructions of one wave
    // complete in order; the fences keep the compiler from moving them)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    for (int p = lane; p < L; p += 64) {
      const int ip = rows[p];
      int rank = 0;
      for (int q = 0; q < L; ++q) rank += rows[q] < ip ? 1 : 0;
      place(s, s + p, ip, rank);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  for (int j2 = a.nmed_t + blockIdx.x * kBlock + threadIdx.x; j2 < a.n; j2 += gridDim.x * kBlock) {
    const int s = a.rp_t[j2], e = a.rp_t[j2 + 1];
    for (int p = s; p < e; ++p) {
      const int ip = a.tmp_i[p];
      int rank = 0;
      for (int q = s; q < e; ++q) rank += a.tmp_i[q] < ip ? 1 : 0;
      place(s, p, ip, rank);
    }
  }
}

// Scaled values of both CSR copies, (a_ij d_r,i) d_c,j as the host forms
// them, and the largest |a~_ij| (order free: the maximum of the bit
// patterns of positive doubles).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_prep_values(PrepCfg a) {
  __shared__ unsigned long long s_max;
  if (threadIdx.x == 0) s_max = 0ull;
  __syncthreads();
  unsigned long long mx = 0ull;
  V* va = static_cast<V*>(a.va_a);
  V* vt = static_cast<V*>(a.va_t);
  auto put_a = [&](int r, int k) {
    const double v = (a.raw_a[k] * a.dr[r]) * a.dc[a.ci_a[k]];
    va[k] = (V)v;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(v));
    mx = mx < bits ? bits : mx;
  };
  auto put_t = [&](int r, int k) { vt[k] = (V)((a.raw_t[k] * a.dr[a.ci_t[k]]) * a.dc[r]); };
  // a wave per long row (the first rows in device order), a thread per row
  // for the rest; every entry is computed on its own
  const int lane = threadIdx.x & 63;
  const int w0 = (blockIdx.x * kBlock + threadIdx.x) >> 6, nw = gridDim.x * (kBlock / 64);
  const int t0 = blockIdx.x * kBlock + threadIdx.x, nt = gridDim.x * kBlock;
  for (int r = w0; r < a.nlong_a; r += nw)
    for (int k = a.rp_a[r] + lane; k < a.rp_a[r + 1]; k += 64) put_a(r, k);
  for (int r = a.nlong_a + t0; r < a.m; r += nt)
    for (int k = a.rp_a[r]; k < a.rp_a[r + 1]; ++k) put_a(r, k);
  for (int r = w0; r < a.nlong_t; r += nw)
    for (int k = a.rp_t[r] + lane; k < a.rp_t[r + 1]; k += 64) put_t(r, k);
  for (int r = a.nlong_t + t0; r < a.n; r += nt)
    for (int k = a.rp_t[r]; k < a.rp_t[r + 1]; ++k) put_t(r, k);
  atomicMax(&s_max, mx);
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(a.scr + 4 * kPrepGrid), s_max);
}

// Scaled vectors in V (b~ = d_r b, c~ = d_c c, l~ = l / d_c, u~ = u / d_c),
// the start point x = clamp(0, l~, u~), and per-workgroup double-double
// partials of |b~|^2 and |c~|^2 in FP64.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_prep_vectors(PrepCfg a) {
  __shared__ DD s_red[4 * 2];
  DD p[2];
  p[0] = dd_zero();
  p[1] = dd_zero();
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.m; i += gridDim.x * kBlock) {
    const double bi = a.dr[i] * a.raw_b[i];
    static_cast<V*>(a.b)[i] = (V)bi;
    dd_add_prod(p[0], bi, bi);
  }
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < a.n; j += gridDim.x * kBlock) {
    const double cj = a.dc[j] * a.raw_c[j];
    const double lj = a.raw_l[j] / a.dc[j];
    const double uj = a.raw_u[j] / a.dc[j];
    const double t = 0.0 < lj ? lj : 0.0;
    const double x0 = uj < t ? uj : t;
    static_cast<V*>(a.c)[j] = (V)cj;
    static_cast<V*>(a.l)[j] = (V)lj;
    static_cast<V*>(a.u)[j] = (V)uj;
    static_cast<V*>(a.x0)[j] = (V)x0;
    static_cast<V*>(a.xa)[j] = (V)x0;
    dd_add_prod(p[1], cj, cj);
  }
  block_sum<2>(p, s_red);
  if (threadIdx.x == 0) {
    a.scr[4 * blockIdx.x + 0] = p[0].hi;
    a.scr[4 * blockIdx.x + 1] = p[0].lo;
    a.scr[4 * blockIdx.x + 2] = p[1].hi;
    a.scr[4 * blockIdx.x + 3] = p[1].lo;
  }
}

// Windowed entries' values: copies of the scaled values they stand for.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_prep_windows(PrepCfg a) {
  const int64_t tot = a.went_t + a.went_a;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < tot; e += (int64_t)gridDim.x * kBlock) {
    if (e < a.went_t) {
      const int32_t s = a.wsrc_t[e];
      static_cast<V*>(a.wval_t)[e] = s < 0 ? V(0) : static_cast<const V*>(a.va_t)[s];
    } else {
      const int64_t f = e - a.went_t;
      const int32_t s = a.wsrc_a[f];
      static_cast<V*>(a.wval_a)[f] = s < 0 ? V(0) : static_cast<const V*>(a.va_a)[s];
    }
  }
}

// The first step size 1 / max |a~_ij| and primal weight |c~| / |b~| (1
// when either is below 1e-10): into the control block and scr.
__global__ __launch_bounds__(kBlock) void k_prep_scalars(PrepCfg a) {
  __shared__ DD s_red[4 * 2];
  DD p[2];
  p[0] = dd_zero();
  p[1] = dd_zero();
  if (threadIdx.x == 0) {
    for (int g = 0; g < kPrepGrid; ++g) {
      p[0] = dd_merge(p[0], DD{a.scr[4 * g + 0], a.scr[4 * g + 1]});
      p[1] = dd_merge(p[1], DD{a.scr[4 * g + 2], a.scr[4 * g + 3]});
    }
    const double bsn = sqrt(dd_value(p[0])), csn = sqrt(dd_value(p[1]));
    const double amax = __longlong_as_double(
        (long long)*reinterpret_cast<const unsigned long long*>(a.scr + 4 * kPrepGrid));
    const double eta0 = amax > 0.0 ? 1.0 / amax : 1.0;
    const double om0 = (csn > 1e-10 && bsn > 1e-10) ? csn / bsn : 1.0;
    a.ctl->eta = eta0;
    a.ctl->omega = om0;
    a.scr[4 * kPrepGrid + 1] = eta0;
    a.scr[4 * kPrepGrid + 2] = om0;
  }
  (void)s_red;
}

// The windowed kernels take more than the default 64 KiB of LDS; the
// attribute is set once per process, before the first launch.
static int win_attributes() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] {
    const void* ks[] = {(const void*)k_primal_win, (const void*)k_dual_win,
                        (const void*)k_prod_win<true, 0>, (const void*)k_prod_win<true, 1>,
                        (const void*)k_prod_win<false, 0>};
    for (const void* f : ks)
      if (err == hipSuccess)
        err = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kWinLds);
  });
  if (err != hipSuccess) g_last_device_error = err;
  return err == hipSuccess ? 0 : -1;
}

int window_kernels_ready() { return win_attributes(); }

template <typename V>
int Kernels<V>::primal_win(const LaunchCfg& c, void* stream, int force) {
  if (c.nwin_t <= 0) return 0;
  if constexpr (!std::is_same<V, float>::value) {
    return -1;  // windowed chunks are planned for FP32 only
  } else {
    if (win_attributes()) return -1;
    hipLaunchKernelGGL(k_primal_win, dim3(c.nwin_t), dim3(kWinBlock), kWinLds,
                       (hipStream_t)stream, c, force);
    return launched();
  }
}
template <typename V>
int Kernels<V>::dual_win(const LaunchCfg& c, void* stream, int force) {
  if (c.nwin_a <= 0) return 0;
  if constexpr (!std::is_same<V, float>::value) {
    return -1;
  } else {
    if (win_attributes()) return -1;
    hipLaunchKernelGGL(k_dual_win, dim3(c.nwin_a), dim3(kWinBlock), kWinLds,
                       (hipStream_t)stream, c, force);
    return launched();
  }
}
template <typename V>
int Kernels<V>::primal_seg(const LaunchCfg& c, void* stream, int force) {
  if (c.nseg_t <= 0) return 0;
  OPDHG_LAUNCH(k_primal_seg<V>, c.nseg_t, c, force);
}
template <typename V>
int Kernels<V>::dual_seg(const LaunchCfg& c, void* stream, int force) {
  if (c.nseg_a <= 0) return 0;
  OPDHG_LAUNCH(k_dual_seg<V>, c.nseg_a, c, force);
}
template <typename V>
int Kernels<V>::decide(const LaunchCfg& c, void* stream) {
  constexpr bool kPlainSums = sizeof(V) == 4;  // FP32 step kernels store plain sums
  OPDHG_LAUNCH(k_decide<kPlainSums>, c.launch_lp, c);
}
template <typename V>
int Kernels<V>::learn_flush(const LaunchCfg& c, void* stream) {
  OPDHG_LAUNCH(k_learn_flush<V>, c.launch_ta, c);
}
template <typename V>
int Kernels<V>::eval_products(const LaunchCfg& c, void* stream) {
  if (!c.evprod) return 0;
  if constexpr (!std::is_same<V, float>::value) {
    return -1;
  } else {
    if (win_attributes()) return -1;
    hipStream_t q = (hipStream_t)stream;
    // one vector at a time: its tiles and windowed chunks, then the
    // segments, whose partials both write
    auto side = [&](auto tside, auto which) -> int {
      constexpr bool T = decltype(tside)::value;
      constexpr int W = decltype(which)::value;
      const int sg = T ? c.sgrid_t : c.sgrid_a, nw = T ? c.nwin_t : c.nwin_a;
      const int ns = T ? c.nseg_t : c.nseg_a;
      if (sg > 0) {
        hipLaunchKernelGGL((k_prod_tiles<T, W>), dim3(sg), dim3(kBlock), 0, q, c);
        if (launched()) return -1;
      }
      if (nw > 0) {
        hipLaunchKernelGGL((k_prod_win<T, W>), dim3(nw), dim3(kWinBlock), kWinLds, q, c);
        if (launched()) return -1;
      }
      if (ns > 0) {
        hipLaunchKernelGGL((k_prod_seg<T, W>), dim3(ns), dim3(kBlock), 0, q, c);
        if (launched()) return -1;
      }
      return 0;
    };
    using t_ = std::true_type;
    using f_ = std::false_type;
    if (side(t_{}, std::integral_constant<int, 0>{})) return -1;
    if (side(t_{}, std::integral_constant<int, 1>{})) return -1;
    return side(f_{}, std::integral_constant<int, 0>{});
  }
}

// The opening evaluation of a set with evaluation products: the streaming
// kernel for the LPs that have them, the tile kernel for the others (not
// launched when every LP has them).
template <typename V>
int Kernels<V>::eval_t(const LaunchCfg& c, void* stream, int mid) {
  if constexpr (std::is_same<V, float>::value) {
    if (mid == 0 && c.evprod) {
      hipLaunchKernelGGL(k_eval_pre<true>, dim3(c.launch_t), dim3(kBlock), 0,
                         (hipStream_t)stream, c);
      if (launched()) return -1;
      if (c.evprod == 2) return 0;
    }
  }
  OPDHG_LAUNCH(k_eval_t<V>, c.launch_t, c, mid);
}
template <typename V>
int Kernels<V>::eval_a(const LaunchCfg& c, void* stream, int mid) {
  if constexpr (std::is_same<V, float>::value) {
    if (mid == 0 && c.evprod) {
      hipLaunchKernelGGL(k_eval_pre<false>, dim3(c.launch_a), dim3(kBlock), 0,
                         (hipStream_t)stream, c);
      if (launched()) return -1;
      if (c.evprod == 2) return 0;
    }
  }
  OPDHG_LAUNCH(k_eval_a<V>, c.launch_a, c, mid);
}
template <typename V>
int Kernels<V>::eval_decide(const LaunchCfg& c, void* stream, int mid) {
  OPDHG_LAUNCH(k_eval_decide, c.launch_lp, c, mid);
}
template <typename V>
int Kernels<V>::apply(const LaunchCfg& c, void* stream, int mid) {
  OPDHG_LAUNCH(k_apply<V>, c.launch_ta, c, mid);
}

int launch_board(const LaunchCfg& c, void* stream) { OPDHG_LAUNCH(k_board, c.launch_lp, c); }

int prep_stats(const PrepCfg& c, void* stream, bool tside, int kind, double e) {
  const int rows = tside ? c.n : c.m;
  const int grid = std::max(1, std::min(4096, (rows + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_prep_stats, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, c,
                     tside ? 1 : 0, kind, e);
  return launched();
}

int struct_build(const StructCfg& c, void* stream) {
  const int g1 = std::max(1, std::min(4096, (c.m + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_struct_rows, dim3(g1), dim3(kBlock), 0, (hipStream_t)stream, c);
  if (launched()) return -1;
  const int g2 = std::max(1, std::min(4096, (c.n + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_struct_cols, dim3(g2), dim3(kBlock), 0, (hipStream_t)stream, c);
  return launched();
}

int power_norm(const PrepCfg& c, void* stream) {
  const int ga = std::max(1, std::min(4096, (c.m + kBlock - 1) / kBlock));
  for (int r = 0; r < c.power_iters; ++r) {
    hipLaunchKernelGGL(k_power_av, dim3(ga), dim3(kBlock), 0, (hipStream_t)stream, c, r);
    if (launched()) return -1;
    hipLaunchKernelGGL(k_power_w, dim3(kPrepGrid), dim3(kBlock), 0, (hipStream_t)stream, c, r);
    if (launched()) return -1;
    hipLaunchKernelGGL(k_power_step, dim3(1), dim3(64), 0, (hipStream_t)stream, c, r);
    if (launched()) return -1;
  }
  hipLaunchKernelGGL(k_power_final, dim3(1), dim3(64), 0, (hipStream_t)stream, c);
  return launched();
}

int prep_apply(const PrepCfg& c, void* stream) {
  const int grid = std::max(1, std::min(4096, (c.m + c.n + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_prep_apply, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, c);
  return launched();
}

template <typename V>
int prep_finish(const PrepCfg& c, void* stream) {
  const int rows = std::max(c.m, c.n);
  const int grid = std::max(1, std::min(4096, (rows + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_prep_values<V>, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, c);
  if (launched()) return -1;
  hipLaunchKernelGGL(k_prep_vectors<V>, dim3(kPrepGrid), dim3(kBlock), 0, (hipStream_t)stream, c);
  if (launched()) return -1;
  if (c.went_t + c.went_a > 0) {
    const int64_t tot = c.went_t + c.went_a;
    const int wg = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (tot + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_prep_windows<V>, dim3(wg), dim3(kBlock), 0, (hipStream_t)stream, c);
    if (launched()) return -1;
  }
  hipLaunchKernelGGL(k_prep_scalars, dim3(1), dim3(kBlock), 0, (hipStream_t)stream, c);
  return launched();
}
template int prep_finish<double>(const PrepCfg&, void*);
template int prep_finish<float>(const PrepCfg&, void*);

template struct Kernels<double>;
template struct Kernels<float>;

}  // namespace opdhg
