// HIP kernels of restarted PDHG with online preconditioning (gfx950).
//
// Every kernel covers a set of LPs: it loops with a fixed grid over
// (lp, tile) work items, so one launch serves one LP, a packed batch or the
// server's changing mix. A tile is a range of CSR rows of one side (A or
// A^T) handled by one 256-thread workgroup, either as row groups of
// `lanes` threads (consecutive lanes read consecutive nonzeros, then an
// xor-shuffle tree sums the group) or, for one long row, by the whole
// workgroup. Per-row epilogues fuse the vector work of the method into the
// sparse product, and per-tile FP64 partial sums feed deterministic
// reductions: the last tile of an LP to finish (completion counter) sums
// all tiles' partials in a fixed order and takes the LP's scalar decision.
//
// Per attempt (Algorithm 1, line 1, eq. (6)):
//   k_primal  CSR(A^T) SpMV of y, g = c - A^T y, x' = proj_[l,u](x - (eta/w) T g),
//             running sum of x, primal online gradient on update iterations
//             (eq. (7)), partials |x'-x|^2, |g|^2, |G^p|^2
//   k_dual    CSR(A) SpMV of x', A x_bar = 2 A x' - A x, dual step and sign
//             projection, running sum of y, dual online gradient, partials
//             |y'-y|^2, (y'-y).(A x'-A x), |b-Ax|^2, |G^d|^2; the last tile
//             applies the adaptive step rule: accept (flip buffers) or retry
//   k_learn   normalized online-gradient step with AdaGrad on T and Sigma
//             (Algorithm 1, lines 4-8), every phi-th accepted iteration
// Every eval_every accepted iterations:
//   k_eval_t  CSR(A^T) SpMV of y and of the running sum of y: reduced costs,
//             dual residuals, bound terms of the dual objective, c^T x, and
//             distances to the restart anchor, for current and average
//   k_eval_a  CSR(A) SpMV of the running sum of x: primal residuals, b^T y,
//             distances; the last tile decides termination and restarts
//   k_apply   moves the iterate to the restart point, resets the sums and the
//             anchor (preconditioners kept), or copies a returned average out
//
// Summation. Every FP64 reduction (and, in FP64 mode, every SpMV row sum)
// is accumulated in double-double: each product is split exactly with an
// FMA into p + e, p is added with an error-free two-sum and all round-off
// is gathered in a second double, which is folded in once at the end. The
// result is the correctly rounded sum except when the exact value lies
// within about n * 2^-106 (relative) of a rounding boundary, so it does not
// depend on the tile size, the lane count, the grid, or what else shares
// the launch. In FP32 mode the SpMV accumulates in FP32 with FMA.
#include <hip/hip_runtime.h>

#include <math.h>

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

__device__ __forceinline__ DD dd_shfl_xor(const DD& a, int off) {
  return DD{__shfl_xor(a.hi, off, 64), __shfl_xor(a.lo, off, 64)};
}

// Merge NV double-doubles over the workgroup in a fixed tree; thread 0
// gets the totals. s_red holds 4 * NV DD.
template <int NV>
__device__ __forceinline__ void block_sum(DD (&v)[NV], DD* s_red) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = dd_merge(v[q], dd_shfl_xor(v[q], off));
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) s_red[wave * NV + q] = v[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q)
      v[q] = dd_merge(dd_merge(dd_merge(s_red[q], s_red[NV + q]), s_red[2 * NV + q]),
                      s_red[3 * NV + q]);
  }
  __syncthreads();
}

// Store the workgroup totals of a tile (thread 0).
template <int NV>
__device__ __forceinline__ void store_partials(double* out, const DD (&v)[NV]) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      out[2 * q] = v[q].hi;
      out[2 * q + 1] = v[q].lo;
    }
  }
}

__device__ __forceinline__ double load_agent(const double* p) {
  unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double(static_cast<long long>(v));
}

// Fixed-order merge of NV double-double partials over ntiles tiles (whole
// workgroup); thread 0 gets the rounded totals. Partials were written by
// other workgroups of this launch or of earlier launches.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* part, int ntiles, double (&out)[NV],
                                             DD* s_red) {
  DD v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = dd_zero();
  for (int t = threadIdx.x; t < ntiles; t += kBlock) {
    const double* src = part + (size_t)t * kPartStride;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = dd_merge(v[q], DD{load_agent(src + 2 * q),
                                                           load_agent(src + 2 * q + 1)});
  }
  block_sum<NV>(v, s_red);
#pragma unroll
  for (int q = 0; q < NV; ++q) out[q] = dd_value(v[q]);
}

// ---- SpMV row accumulators: double-double in FP64, FMA in FP32 ----
template <typename V>
struct RowAcc;

template <>
struct RowAcc<double> {
  DD v;
  __device__ __forceinline__ void zero() { v = dd_zero(); }
  __device__ __forceinline__ void add(double a, double x) { dd_add_prod(v, a, x); }
  __device__ __forceinline__ void merge_xor(int off) { v = dd_merge(v, dd_shfl_xor(v, off)); }
  __device__ __forceinline__ void merge(const RowAcc& o) { v = dd_merge(v, o.v); }
  __device__ __forceinline__ double value() const { return dd_value(v); }
};

template <>
struct RowAcc<float> {
  float v;
  __device__ __forceinline__ void zero() { v = 0.f; }
  __device__ __forceinline__ void add(float a, float x) { v = fmaf(a, x, v); }
  __device__ __forceinline__ void merge_xor(int off) { v += __shfl_xor(v, off, 64); }
  __device__ __forceinline__ void merge(const RowAcc& o) { v += o.v; }
  __device__ __forceinline__ float value() const { return v; }
};

// Completion counting: true in every thread of the workgroup that finished
// the last tile of its LP for this counter. The counter is reset by the
// caller of the final step.
__device__ __forceinline__ bool last_tile(int32_t* counter, int ntiles, int* s_flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    int prev = atomicAdd(counter, 1);
    *s_flag = (prev == ntiles - 1);
  }
  __syncthreads();
  const bool last = *s_flag != 0;
  if (last) __threadfence();
  return last;
}

// Sparse dot products of the rows of one tile with NA vectors, then a
// per-row epilogue epi(row, val[NA]) run by one thread per row. Vector q is
// read as vec[q][col] / div[q] when div[q] > 0 (the average iterate).
template <typename V, int NA, typename Epi>
__device__ __forceinline__ void tile_spmv(const Tile& tile, const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ ci,
                                          const V* __restrict__ va, const V* const* vec,
                                          const double* div, Epi&& epi,
                                          RowAcc<V>* s_long) {
  const int tid = threadIdx.x;
  if (tile.lanes == 0) {
    const int r = tile.rb;
    const int s = rp[r], e = rp[r + 1];
    RowAcc<V> acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q].zero();
    for (int i = s + tid; i < e; i += kBlock) {
      const V a = va[i];
      const int cc = ci[i];
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const V xv = div[q] > 0.0 ? (V)((double)vec[q][cc] / div[q]) : vec[q][cc];
        acc[q].add(a, xv);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
      for (int q = 0; q < NA; ++q) acc[q].merge_xor(off);
    }
    if ((tid & 63) == 0) {
#pragma unroll
      for (int q = 0; q < NA; ++q) s_long[(tid >> 6) * NA + q] = acc[q];
    }
    __syncthreads();
    if (tid == 0) {
      V out[NA];
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        RowAcc<V> t = s_long[q];
        t.merge(s_long[NA + q]);
        t.merge(s_long[2 * NA + q]);
        t.merge(s_long[3 * NA + q]);
        out[q] = t.value();
      }
      epi(r, out);
    }
    __syncthreads();
  } else {
    const int L = tile.lanes;
    const int lane = tid & (L - 1);
    const int ng = kBlock / L;
    for (int r = tile.rb + tid / L; r < tile.re; r += ng) {
      const int s = rp[r], e = rp[r + 1];
      RowAcc<V> acc[NA];
#pragma unroll
      for (int q = 0; q < NA; ++q) acc[q].zero();
      for (int i = s + lane; i < e; i += L) {
        const V a = va[i];
        const int cc = ci[i];
#pragma unroll
        for (int q = 0; q < NA; ++q) {
          const V xv = div[q] > 0.0 ? (V)((double)vec[q][cc] / div[q]) : vec[q][cc];
          acc[q].add(a, xv);
        }
      }
      for (int off = L >> 1; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[q].merge_xor(off);
      }
      if (lane == 0) {
        V out[NA];
#pragma unroll
        for (int q = 0; q < NA; ++q) out[q] = acc[q].value();
        epi(r, out);
      }
    }
  }
}

template <typename V>
__device__ __forceinline__ V clampv(V v, V lo, V hi) {
  V t = v < lo ? lo : v;
  return t > hi ? hi : t;
}

__device__ __forceinline__ bool attempt_guard(const Ctl* c) {
  return c->status == kRunning && c->need_eval == 0 && c->k < c->k_limit;
}

__device__ __forceinline__ bool eval_guard(const Ctl* c) {
  return c->status == kRunning && c->need_eval != 0;
}

// ---------------------------------------------------------------------------
// scalar decisions (thread 0 of the last workgroup of an LP)
// ---------------------------------------------------------------------------

// Factor (j+1)^-e of the step rule for attempt j: from the host-computed
// table for the first kPowTab attempts, else computed here.
__device__ __forceinline__ double step_factor(const double* tab, int which, int64_t j,
                                              double e) {
  if (j >= 1 && j <= kPowTab) return tab[which * kPowTab + (j - 1)];
  return pow((double)(j + 1), -e);
}

// Adaptive step rule (PDLP's): accept when eta <= eta_bar; the next step is
// min((1 - (j+1)^-red) eta_bar, (1 + (j+1)^-gro) eta), j counting attempts.
__device__ void decide_step(Ctl* c, const DevParams* p, const double* tab, const double* s) {
  const double dx2 = s[0], g2 = s[1], gp2 = s[2];
  const double dy2 = s[3], inter = fabs(s[4]), r2 = s[5], gd2 = s[6];
  c->attempts += 1;
  if (!(isfinite(dx2) && isfinite(dy2) && isfinite(inter))) {
    c->status = kNumError;
    return;
  }
  const double eta = c->eta, om = c->omega;
  const double movement = 0.5 * om * dx2 + 0.5 * dy2 / om;
  const double eta_bar = inter > 0.0 ? movement / inter : INFINITY;
  const double first = (1.0 - step_factor(tab, 0, c->attempts, p->step_reduction)) * eta_bar;
  const double second = (1.0 + step_factor(tab, 1, c->attempts, p->step_growth)) * eta;
  const double eta_next = second < first ? second : first;
  c->last_eta_bar = eta_bar;
  if (eta <= eta_bar) {
    const bool learn = p->lr > 0.0 && (c->k % p->phi) == 0;
    c->eta_acc = eta;
    c->w += eta;
    c->k += 1;
    c->t += 1;
    c->cur ^= 1;
    c->eta = eta_next;
    c->retries = 0;
    if (learn) {
      c->learn_pending = 1;
      c->g2 = g2;
      c->r2 = r2;
      c->gp2 = gp2;
      c->gd2 = gd2;
      if (p->schedule == 1) {  // AdaGrad on the norm: H += |G / scale|^2 = |G|^2 / scale^2
        const bool np = p->normalize && !(g2 > 0.0);
        const bool nd = p->normalize && !(r2 > 0.0);
        const double sp = p->normalize ? g2 : 1.0;
        const double sd = p->normalize ? r2 : 1.0;
        if (!np) c->hp_norm = c->hp_norm + gp2 / (sp * sp);
        if (!nd) c->hd_norm = c->hd_norm + gd2 / (sd * sd);
      }
    }
    if (c->k % p->eval_every == 0 || c->k >= p->max_iter) c->need_eval = 1;
  } else {
    c->eta = eta_next;
    c->retries += 1;
    if (c->retries > p->max_retries || !(eta_next > 0.0 && isfinite(eta_next)))
      c->status = kNumError;
  }
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
  if (c->t > 0) {
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
        const double th = p->pw_smoothing;
        c->omega = exp(th * log(dyn / dxn) + (1.0 - th) * log(om));
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

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <typename V>
__global__ __launch_bounds__(kBlock) void k_init_products(const BatchDev* __restrict__ bd) {
  __shared__ RowAcc<V> s_long[4];
  const int nwork = bd->nwork_a;
  const double nodiv[1] = {0.0};
  for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const WorkItem it = bd->work_a[wi];
    const LpDev& lp = bd->lps[it.lp];
    const int cur = lp.ctl->cur;
    const Tile tile = lp.tiles_a[it.tile];
    V* Ax = static_cast<V*>(lp.Ax[cur]);
    const V* vecs[1] = {static_cast<const V*>(lp.x[cur])};
    tile_spmv<V, 1>(tile, lp.rp_a, lp.ci_a, static_cast<const V*>(lp.va_a), vecs, nodiv,
                    [&](int i, V (&acc)[1]) { Ax[i] = acc[0]; }, s_long);
  }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_primal(const BatchDev* __restrict__ bd, int force) {
  __shared__ DD s_red[4 * 3];
  __shared__ RowAcc<V> s_long[4];
  const int nwork = bd->nwork_t;
  const double nodiv[1] = {0.0};
  for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const WorkItem it = bd->work_t[wi];
    const LpDev& lp = bd->lps[it.lp];
    const Ctl* c = lp.ctl;
    if (!force && !attempt_guard(c)) continue;
    const int cur = c->cur, nxt = cur ^ 1;
    const double eta = c->eta, om = c->omega;
    const V tau = (V)(eta / om);
    const V etav = (V)eta;
    const bool learn = lp.prm->lr > 0.0 && (c->k % lp.prm->phi) == 0;
    const V* __restrict__ cc = static_cast<const V*>(lp.c);
    const V* __restrict__ lo = static_cast<const V*>(lp.l);
    const V* __restrict__ hi = static_cast<const V*>(lp.u);
    const V* __restrict__ T = static_cast<const V*>(lp.T);
    const V* __restrict__ x = static_cast<const V*>(lp.x[cur]);
    const V* __restrict__ xs = static_cast<const V*>(lp.xs[cur]);
    V* __restrict__ xn = static_cast<V*>(lp.x[nxt]);
    V* __restrict__ xsn = static_cast<V*>(lp.xs[nxt]);
    V* __restrict__ Gp = static_cast<V*>(lp.Gp);
    const V* vecs[1] = {static_cast<const V*>(lp.y[cur])};
    DD p[3] = {dd_zero(), dd_zero(), dd_zero()};
    const Tile tile = lp.tiles_t[it.tile];
    tile_spmv<V, 1>(
        tile, lp.rp_t, lp.ci_t, static_cast<const V*>(lp.va_t), vecs, nodiv,
        [&](int j, V (&acc)[1]) {
          const V g = cc[j] - acc[0];
          const V xj = x[j];
          const V xh = xj - (tau * T[j]) * g;
          const V lj = lo[j], uj = hi[j];
          const V xv = clampv(xh, lj, uj);
          xn[j] = xv;
          xsn[j] = xs[j] + etav * xv;
          const double dx = (double)xv - (double)xj;
          dd_add_prod(p[0], dx, dx);
          dd_add_prod(p[1], (double)g, (double)g);
          if (learn) {
            const bool ind = (xh >= lj) && (xh <= uj);
            const V gp = ind ? -((tau * g) * g) : V(0);
            Gp[j] = gp;
            dd_add_prod(p[2], (double)gp, (double)gp);
          }
        },
        s_long);
    block_sum<3>(p, s_red);
    store_partials<3>(lp.part_t + (size_t)it.tile * kPartStride, p);
  }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_dual(const BatchDev* __restrict__ bd) {
  __shared__ DD s_red[4 * 4];
  __shared__ RowAcc<V> s_long[4];
  __shared__ int s_flag;
  const int nwork = bd->nwork_a;
  const double nodiv[1] = {0.0};
  for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const WorkItem it = bd->work_a[wi];
    const LpDev& lp = bd->lps[it.lp];
    Ctl* c = lp.ctl;
    if (!attempt_guard(c)) continue;
    const int cur = c->cur, nxt = cur ^ 1;
    const double eta = c->eta, om = c->omega;
    const V sig = (V)(eta * om);
    const V etav = (V)eta;
    const bool learn = lp.prm->lr > 0.0 && (c->k % lp.prm->phi) == 0;
    const V* __restrict__ b = static_cast<const V*>(lp.b);
    const V* __restrict__ S = static_cast<const V*>(lp.S);
    const V* __restrict__ y = static_cast<const V*>(lp.y[cur]);
    const V* __restrict__ ys = static_cast<const V*>(lp.ys[cur]);
    const V* __restrict__ Ax = static_cast<const V*>(lp.Ax[cur]);
    V* __restrict__ yn = static_cast<V*>(lp.y[nxt]);
    V* __restrict__ ysn = static_cast<V*>(lp.ys[nxt]);
    V* __restrict__ Axn = static_cast<V*>(lp.Ax[nxt]);
    V* __restrict__ Gd = static_cast<V*>(lp.Gd);
    const int8_t* __restrict__ sense = lp.sense;
    const V* vecs[1] = {static_cast<const V*>(lp.x[nxt])};
    DD p[4] = {dd_zero(), dd_zero(), dd_zero(), dd_zero()};
    const Tile tile = lp.tiles_a[it.tile];
    tile_spmv<V, 1>(
        tile, lp.rp_a, lp.ci_a, static_cast<const V*>(lp.va_a), vecs, nodiv,
        [&](int i, V (&acc)[1]) {
          const V axn = acc[0];
          const V ax = Ax[i];
          const V axbar = V(2) * axn - ax;
          const V bi = b[i];
          const V rt = bi - axbar;
          const V yi = y[i];
          const V yh = yi + (sig * S[i]) * rt;
          const bool ineq = sense[i] != 0;
          const V yv = (ineq && yh < V(0)) ? V(0) : yh;
          yn[i] = yv;
          Axn[i] = axn;
          ysn[i] = ys[i] + etav * yv;
          const double dy = (double)yv - (double)yi;
          dd_add_prod(p[0], dy, dy);
          dd_add_prod(p[1], dy, (double)axn - (double)ax);
          const V r = bi - ax;
          dd_add_prod(p[2], (double)r, (double)r);
          if (learn) {
            const bool ind = !ineq || yh >= V(0);
            const V gd = ind ? -((sig * r) * rt) : V(0);
            Gd[i] = gd;
            dd_add_prod(p[3], (double)gd, (double)gd);
          }
        },
        s_long);
    block_sum<4>(p, s_red);
    store_partials<4>(lp.part_a + (size_t)it.tile * kPartStride, p);
    if (last_tile(&c->cnt_dual, lp.ntiles_a, &s_flag)) {
      double st[3], sa[4];
      sum_partials<3>(lp.part_t, lp.ntiles_t, st, s_red);
      sum_partials<4>(lp.part_a, lp.ntiles_a, sa, s_red);
      if (threadIdx.x == 0) {
        const double s[7] = {st[0], st[1], st[2], sa[0], sa[1], sa[2], sa[3]};
        decide_step(c, lp.prm, lp.pow_tab, s);
        c->cnt_dual = 0;
        __threadfence();
      }
      __syncthreads();
    }
  }
}

template <typename V>
__device__ __forceinline__ void ogd_update(V* __restrict__ P, V* __restrict__ H,
                                           const V* __restrict__ G, int r0, int r1,
                                           double scale, const DevParams* p, double hnorm) {
  const V lr = (V)p->lr;
  const V fl = (V)p->floor;
  for (int r = r0 + threadIdx.x; r < r1; r += kBlock) {
    const V gv = (V)((double)G[r] / scale);
    V step;
    if (p->schedule == 0) {
      const V h = H[r] + gv * gv;
      H[r] = h;
      step = h > V(0) ? gv / sqrt(h) : V(0);
    } else if (p->schedule == 1) {
      step = hnorm > 0.0 ? (V)((double)gv / sqrt(hnorm)) : V(0);
    } else {
      step = gv;
    }
    const V pv = P[r] - lr * step;
    P[r] = pv < fl ? fl : pv;
  }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_learn(const BatchDev* __restrict__ bd) {
  __shared__ int s_flag;
  const int nt = bd->nwork_t;
  const int nwork = nt + bd->nwork_a;
  for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const bool tside = wi < nt;
    const WorkItem it = tside ? bd->work_t[wi] : bd->work_a[wi - nt];
    const LpDev& lp = bd->lps[it.lp];
    Ctl* c = lp.ctl;
    if (!c->learn_pending) continue;
    const DevParams* p = lp.prm;
    const Tile tile = tside ? lp.tiles_t[it.tile] : lp.tiles_a[it.tile];
    const double nrm = tside ? c->g2 : c->r2;
    const bool skip = p->normalize && !(nrm > 0.0);
    const double scale = p->normalize ? nrm : 1.0;
    if (!skip) {
      if (tside)
        ogd_update<V>(static_cast<V*>(lp.T), static_cast<V*>(lp.Hp),
                      static_cast<const V*>(lp.Gp), tile.rb, tile.re, scale, p, c->hp_norm);
      else
        ogd_update<V>(static_cast<V*>(lp.S), static_cast<V*>(lp.Hd),
                      static_cast<const V*>(lp.Gd), tile.rb, tile.re, scale, p, c->hd_norm);
    }
    if (last_tile(&c->cnt_learn, lp.ntiles_t + lp.ntiles_a, &s_flag)) {
      if (threadIdx.x == 0) {
        c->learn_pending = 0;
        c->cnt_learn = 0;
        __threadfence();
      }
      __syncthreads();
    }
  }
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

template <typename V>
__global__ __launch_bounds__(kBlock) void k_eval_t(const BatchDev* __restrict__ bd) {
  __shared__ DD s_red[4 * 2 * kEvT];
  __shared__ RowAcc<V> s_long[4 * 2];
  const int nwork = bd->nwork_t;
  for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const WorkItem it = bd->work_t[wi];
    const LpDev& lp = bd->lps[it.lp];
    const Ctl* c = lp.ctl;
    if (!eval_guard(c)) continue;
    const int cur = c->cur;
    const double w = c->w;
    const bool has_avg = w > 0.0;
    const V* __restrict__ cc = static_cast<const V*>(lp.c);
    const V* __restrict__ lo = static_cast<const V*>(lp.l);
    const V* __restrict__ hi = static_cast<const V*>(lp.u);
    const V* __restrict__ x = static_cast<const V*>(lp.x[cur]);
    const V* __restrict__ xs = static_cast<const V*>(lp.xs[cur]);
    const V* __restrict__ xa = static_cast<const V*>(lp.xa);
    const double* __restrict__ dc = lp.dc;
    const int8_t* __restrict__ bfin = lp.bfin;
    const V* vecs[2] = {static_cast<const V*>(lp.y[cur]), static_cast<const V*>(lp.ys[cur])};
    const double divs[2] = {0.0, has_avg ? w : 0.0};
    DD p[2 * kEvT];
#pragma unroll
    for (int q = 0; q < 2 * kEvT; ++q) p[q] = dd_zero();
    const Tile tile = lp.tiles_t[it.tile];
    tile_spmv<V, 2>(
        tile, lp.rp_t, lp.ci_t, static_cast<const V*>(lp.va_t), vecs, divs,
        [&](int j, V (&acc)[2]) {
          const double cj = (double)cc[j];
          const int8_t bf = bfin[j];
          const double lj = (double)lo[j], uj = (double)hi[j];
          const double xaj = (double)xa[j];
          for (int z = 0; z < (has_avg ? 2 : 1); ++z) {
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
        },
        s_long);
    block_sum<2 * kEvT>(p, s_red);
    store_partials<2 * kEvT>(lp.part_t + (size_t)it.tile * kPartStride, p);
  }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_eval_a(const BatchDev* __restrict__ bd) {
  __shared__ DD s_red[4 * 2 * kEvT];
  __shared__ RowAcc<V> s_long[4];
  __shared__ int s_flag;
  const int nwork = bd->nwork_a;
  for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const WorkItem it = bd->work_a[wi];
    const LpDev& lp = bd->lps[it.lp];
    Ctl* c = lp.ctl;
    if (!eval_guard(c)) continue;
    const int cur = c->cur;
    const double w = c->w;
    const bool has_avg = w > 0.0;
    const V* __restrict__ b = static_cast<const V*>(lp.b);
    const V* __restrict__ y = static_cast<const V*>(lp.y[cur]);
    const V* __restrict__ ys = static_cast<const V*>(lp.ys[cur]);
    const V* __restrict__ ya = static_cast<const V*>(lp.ya);
    const V* __restrict__ Ax = static_cast<const V*>(lp.Ax[cur]);
    V* __restrict__ Axa = static_cast<V*>(lp.Axa);
    const double* __restrict__ dr = lp.dr;
    const int8_t* __restrict__ sense = lp.sense;
    const V* vecs[1] = {static_cast<const V*>(lp.xs[cur])};
    const double divs[1] = {has_avg ? w : 0.0};
    DD p[2 * kEvA];
#pragma unroll
    for (int q = 0; q < 2 * kEvA; ++q) p[q] = dd_zero();
    const Tile tile = lp.tiles_a[it.tile];
    tile_spmv<V, 1>(
        tile, lp.rp_a, lp.ci_a, static_cast<const V*>(lp.va_a), vecs, divs,
        [&](int i, V (&acc)[1]) {
          const double bi = (double)b[i];
          const bool ineq = sense[i] != 0;
          const double yai = (double)ya[i];
          if (has_avg) Axa[i] = acc[0];
          for (int z = 0; z < (has_avg ? 2 : 1); ++z) {
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
        },
        s_long);
    block_sum<2 * kEvA>(p, s_red);
    store_partials<2 * kEvA>(lp.part_a + (size_t)it.tile * kPartStride, p);
    if (last_tile(&c->cnt_eval, lp.ntiles_a, &s_flag)) {
      double st[2 * kEvT], sa[2 * kEvA];
      sum_partials<2 * kEvT>(lp.part_t, lp.ntiles_t, st, s_red);
      sum_partials<2 * kEvA>(lp.part_a, lp.ntiles_a, sa, s_red);
      if (threadIdx.x == 0) {
        decide_eval(c, lp.prm, st, sa);
        c->cnt_eval = 0;
        __threadfence();
      }
      __syncthreads();
    }
  }
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_apply(const BatchDev* __restrict__ bd) {
  __shared__ int s_flag;
  const int nt = bd->nwork_t;
  const int nwork = nt + bd->nwork_a;
  for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const bool tside = wi < nt;
    const WorkItem it = tside ? bd->work_t[wi] : bd->work_a[wi - nt];
    const LpDev& lp = bd->lps[it.lp];
    Ctl* c = lp.ctl;
    const bool restart = c->restart_pending != 0;
    const bool fin = c->finalize_avg != 0;
    if (!restart && !fin) continue;
    const int cur = c->cur;
    const bool to_avg = restart ? (c->restart_avg != 0) : true;
    const double w = c->restart_w;
    const Tile tile = tside ? lp.tiles_t[it.tile] : lp.tiles_a[it.tile];
    if (tside) {
      V* x = static_cast<V*>(lp.x[cur]);
      V* xs = static_cast<V*>(lp.xs[cur]);
      V* xa = static_cast<V*>(lp.xa);
      for (int j = tile.rb + threadIdx.x; j < tile.re; j += kBlock) {
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
      for (int i = tile.rb + threadIdx.x; i < tile.re; i += kBlock) {
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
    if (last_tile(&c->cnt_apply, lp.ntiles_t + lp.ntiles_a, &s_flag)) {
      if (threadIdx.x == 0) {
        c->restart_pending = 0;
        c->finalize_avg = 0;
        c->cnt_apply = 0;
        __threadfence();
      }
      __syncthreads();
    }
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

template <typename V>
int Kernels<V>::init_products(const LaunchCfg& c, void* stream) {
  hipLaunchKernelGGL(k_init_products<V>, dim3(c.grid_a), dim3(kBlock), 0,
                     (hipStream_t)stream, c.bd);
  return launched();
}

template <typename V>
int Kernels<V>::primal(const LaunchCfg& c, void* stream, int force) {
  hipLaunchKernelGGL(k_primal<V>, dim3(c.grid_t), dim3(kBlock), 0, (hipStream_t)stream, c.bd,
                     force);
  return launched();
}

template <typename V>
int Kernels<V>::dual(const LaunchCfg& c, void* stream) {
  hipLaunchKernelGGL(k_dual<V>, dim3(c.grid_a), dim3(kBlock), 0, (hipStream_t)stream, c.bd);
  return launched();
}

template <typename V>
int Kernels<V>::learn(const LaunchCfg& c, void* stream) {
  hipLaunchKernelGGL(k_learn<V>, dim3(c.grid_ta), dim3(kBlock), 0, (hipStream_t)stream, c.bd);
  return launched();
}

template <typename V>
int Kernels<V>::eval_t(const LaunchCfg& c, void* stream) {
  hipLaunchKernelGGL(k_eval_t<V>, dim3(c.grid_t), dim3(kBlock), 0, (hipStream_t)stream, c.bd);
  return launched();
}

template <typename V>
int Kernels<V>::eval_a(const LaunchCfg& c, void* stream) {
  hipLaunchKernelGGL(k_eval_a<V>, dim3(c.grid_a), dim3(kBlock), 0, (hipStream_t)stream, c.bd);
  return launched();
}

template <typename V>
int Kernels<V>::apply(const LaunchCfg& c, void* stream) {
  hipLaunchKernelGGL(k_apply<V>, dim3(c.grid_ta), dim3(kBlock), 0, (hipStream_t)stream, c.bd);
  return launched();
}

template struct Kernels<double>;
template struct Kernels<float>;

}  // namespace opdhg
