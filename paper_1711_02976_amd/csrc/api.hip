// C ABI of librpyfmm: plan construction, the matvec launch sequence and
// tree export.  See include/rpyfmm.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rpyfmm.h"
#include "fmm.h"

namespace {

// Detail of the last failure on this thread: a fixed buffer (trivially
// destructible, so no thread-exit or process-exit handler is registered).
thread_local char g_last_error[512];

void set_error(const std::string& msg) {
  const size_t k = std::min(msg.size(), sizeof(g_last_error) - 1);
  std::memcpy(g_last_error, msg.data(), k);
  g_last_error[k] = 0;
}

rpy_status fail(rpy_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

// Smallest expansion order whose measured relative L2 error against the
// direct sum stays below eps/2 on calibration inputs (the accuracy-to-order
// map is not given in the paper; Sec. 4.3 reports 3, 6 and 9 digits with
// refinement limits 80, 100 and 120).  Level-uniform trees (no W/X lists)
// converge faster than adaptive ones, whose W and X interactions have a
// worse separation ratio: measured on a uniform cube, p = 7 gives 2.2e-4 and
// p = 16 gives 4.0e-7; on 20k beads in Gaussian blobs p = 12, 16, 20 give
// 3.2e-5, 2.6e-6 and 2.8e-7, and on 4M beads in 2,000 blobs (depth 11-13)
// p = 20 gives 1.0e-6 and p = 21 gives 6.8e-7.  Below 1e-8 (the paper's
// 9-digit setting) the order is the highest built, 27: on 20k beads in a
// uniform cube p = 21, 24, 27 give 3.3e-8, 9.0e-9, 2.6e-9, and on 20k
// clustered beads (adaptive tree) 1.3e-7, 3.1e-8, 7.5e-9.
// Highest order at which the library picks the polynomial evaluation.
constexpr int EVAL_POLY_AUTO_MAX = 10;

int order_for_eps(double eps, bool adaptive) {
  static const double tol[] = {1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7,
                               3e-8, 1e-8};
  static const int ord[] = {2, 3, 4, 6, 7, 8, 10, 11, 13, 14, 16, 17, 19, 20, 21};
  int p = rpy::MAX_ORDER;
  for (int i = 0; i < (int)(sizeof(tol) / sizeof(tol[0])); ++i)
    if (eps >= tol[i]) {
      p = ord[i];
      break;
    }
  if (adaptive) p += (p - 3) / 3 + 1;
  return std::min(p, rpy::MAX_ORDER);
}

// ---- leaf-size choice ------------------------------------------------------
// Modelled time of one matvec with nrhs right-hand sides on a built tree, from
// its interaction counts and per-unit kernel times measured on MI355X for this
// library (uniform cube, sphere surface, Gaussian blobs and batched systems,
// p = 16 and 21):
//   * P2P and the direct W sums per ordered bead pair, with targets padded to
//     whole 64-bead waves (a wave with no target in its 128-bead tile skips
//     the pair loop); a pass of 4 right-hand sides costs about 2.3x a pass
//     of one;
//   * per density (4 per right-hand side): M2L per V pair (O(p^3)), upward
//     and downward translations per box (O(p^4)), S->M and evaluation sets
//     per leaf, S->L per (bead, X box) and W-multipole evaluation per
//     (target bead, W box) (O(p^2)).
// The overlap correction is not modelled: trial trees have no O list.  Also
// returns the range of refinement limits that produce this same tree.
// Right-hand sides of the near-field group with `left` still to do and
// groups of at most nrn: 16 on the matrix cores, else 8, 4, 2 or 1 on the
// vector units.  In the FP64 form the group of 16 also takes x = 1, 2, 4 or
// 8 more on the vector units of the same launch (unless 32 or more remain,
// so that more of them reach the matrix cores): on cube-15M, 16 + 4 run in
// 1.22 s against 0.95 + 0.36 s as two launches.  In the mixed form the
// extra registers halve the matrix-core kernel's occupancy and 16 + 4 take
// 0.82 s against 0.51 + 0.20 s, so its groups of 16 stay alone.
static int vec_group(int m) {
  int c = 1;
  while (2 * c <= std::min(m, rpy::NEAR_VEC_RHS)) c *= 2;
  return c;
}
static int near_group(int left, int nrn, bool mixed) {
  const int m = std::min(left, nrn);
  if (m < rpy::NEAR_MC_RHS) return vec_group(m);
  if (mixed || m == rpy::NEAR_MC_RHS || left >= 2 * rpy::NEAR_MC_RHS) return rpy::NEAR_MC_RHS;
  return rpy::NEAR_MC_RHS + vec_group(m - rpy::NEAR_MC_RHS);
}
// The largest group of a matvec of nrhs right-hand sides (its workspace).
static int near_group_max(int nrhs, bool mixed) {
  int g = 1;
  for (int left = nrhs; left > 0; left -= near_group(left, rpy::NEAR_MAX_RHS, mixed))
    g = std::max(g, near_group(left, rpy::NEAR_MAX_RHS, mixed));
  return g;
}

struct TreeCost {
  double ns = 0;
  double near_ns = 0;  // the P2P and direct-W part of ns
  int same_lo = 0;     // largest leaf that a larger limit could not split
  int same_hi = 0;     // smallest count among split boxes: limits below it keep every split
  bool adaptive = false;
};

static int model_tree(const rpy::Built& B, int order, double eps, bool mixed, int max_depth, int nrhs, int wd_opt,
                      TreeCost* out) {
  const rpy::Tree& t = B.tree;
  const int nbox = t.nbox;
  std::vector<int> beg(nbox), end(nbox), child(nbox), lev(nbox);
  auto get = [&](std::vector<int>& h, const int* d, size_t n) {
    return n == 0 || hipMemcpy(h.data(), d, sizeof(int) * n, hipMemcpyDeviceToHost) == hipSuccess;
  };
  if (!get(beg, t.begin, nbox) || !get(end, t.end, nbox) || !get(child, t.child, nbox) || !get(lev, t.level, nbox))
    return -4;
  const rpy::List& U = B.lists[rpy::LU];
  const rpy::List& W = B.lists[rpy::LW];
  const rpy::List& X = B.lists[rpy::LX];
  std::vector<int> uo(nbox + 1), ue(U.len), wo(nbox + 1), we(W.len), xo(nbox + 1), xe(X.len);
  if (!get(uo, U.off, nbox + 1) || !get(ue, U.ent, U.len) || !get(wo, W.off, nbox + 1) || !get(we, W.ent, W.len) ||
      !get(xo, X.off, nbox + 1) || !get(xe, X.ent, X.len))
    return -4;
  const bool adaptive = W.len > 0 || X.len > 0;
  const int p = order ? order : order_for_eps(eps, adaptive);
  const int wmax = wd_opt == 0 ? rpy::wdirect_default(p) : wd_opt;
  double pairs = 0, weval = 0, xpairs = 0, nleaf = 0;
  int lo = 0, hi = 0x7fffffff;
  for (int b = 0; b < nbox; ++b) {
    const int nb = end[b] - beg[b];
    if (child[b] < 0) {
      if (lev[b] < max_depth) lo = std::max(lo, nb);
      nleaf += 1;
      const double padded = 64.0 * ((nb + 63) / 64);
      double src = 0;
      for (int k = uo[b]; k < uo[b + 1]; ++k) src += end[ue[k]] - beg[ue[k]];
      for (int k = wo[b]; k < wo[b + 1]; ++k) {
        const int nc = end[we[k]] - beg[we[k]];
        if (wmax < 0 || nc > wmax) weval += nb;
        else src += nc;
      }
      pairs += padded * src;
    } else {
      hi = std::min(hi, nb);
    }
    for (int k = xo[b]; k < xo[b + 1]; ++k) xpairs += end[xe[k]] - beg[xe[k]];
  }
  const double S = (p + 1.0) * (p + 2.0) * (2.0 * p + 3.0) / 6.0, T = (p + 1.0) * (p + 2.0) / 2.0;
  const double S16 = 1785.0, S21 = 3795.0, T21 = 253.0;
  // ns per unit (one density unless stated)
  const double c_pair = mixed ? 0.53e-3 : 0.98e-3;  // per padded pair, one right-hand side
  // the FP32 rotation M2L up to p = 16 fits two blocks per CU; the FP64 one
  // above p = 16 takes 32 columns per batch
  // up to p = 16 the M->L per (V pair, density) is affine in S: a part
  // that does not shrink with the order (gathers, phases, column sums,
  // barriers) equal to 655 units of S (cube-15M, FP32: 0.70 ns at p = 16,
  // 0.25 ns at p = 7)
  double c_v = p > 16 ? 2.55 * S / S21 : 0.94 * (655.0 + S) / (655.0 + S16);
  if (!mixed) c_v *= p > 16 ? 2.15 : 1.65;
  const double c_box = 30.0 * (T / T21) * (T / T21);
  const double c_leaf = 27.0 * T / T21;
  const double c_x = 0.075 * T / T21, c_w = 0.09 * T / T21;
  const double far = B.lists[rpy::LV].len * c_v + nbox * c_box + nleaf * c_leaf + xpairs * c_x + weval * c_w;
  // near-field groups as rpy_matvec runs them, in units of a one-rhs launch
  // (measured on cube-15M: 16 rhs on the matrix cores 5.5, 16 + 4 in the
  // FP64 form 7.1; on the vector units 8 rhs 3.9, 4 rhs 2.3, 2 rhs 1.5)
  const int r = std::max(nrhs, 1);
  double near_passes = 0.0;
  for (int left = r; left > 0;) {
    const int g = near_group(left, rpy::NEAR_MAX_RHS, mixed);
    const int x = g >= rpy::NEAR_MC_RHS ? g - rpy::NEAR_MC_RHS : g;
    const double vec = x == 8 ? 3.9 : x == 4 ? 2.3 : x == 2 ? 1.5 : x == 1 ? 1.0 : 0.0;
    near_passes += g >= rpy::NEAR_MC_RHS ? 5.5 + 0.65 * vec : vec;
    left -= g;
  }
  out->near_ns = pairs * c_pair * near_passes;
  out->ns = out->near_ns + 4.0 * r * far;
  out->same_lo = lo;
  out->same_hi = hi;
  out->adaptive = adaptive;
  return 0;
}

}  // namespace

// Matvec workspace for the right-hand sides of one pass.
struct Work {
  double2* M = nullptr;   // multipoles [nbox][4 nrc][T]
  double2* L = nullptr;   // local expansions [nbox][4 nrc][T]
  double* sF = nullptr;   // forces, tree order [nrc][3][n]
  double* u = nullptr;    // near-field velocities, tree order
  double* uf = nullptr;   // far-field velocities, tree order
  double* Q = nullptr;    // per-bead charges for S->M / S->L [n + 64][4 nrc]
  double2* DL = nullptr;  // evaluation sets (local expansions of the leaves)
  double2* DW = nullptr;  // evaluation sets (evaluated W-list multipoles)
  double2* XP = nullptr;  // S->L partial sums of boxes split over several work items
  double* PV = nullptr;   // polynomial evaluation: the leaves' density polynomials
  float2* M32 = nullptr;  // mixed form: multipoles as the FP32 M->L reads them
};
constexpr int WS_N = 11;  // arrays of Work, in the order above

struct rpy_plan_s {
  rpy::Built B;
  rpy::Tables tb{};
  rpy::Tiles tiles{};
  rpy::EvalPlan ep{};
  int p = 0, leaf_size = 0, max_depth = 14, precision = 0, m2l_mode = 2;
  int wd = 0;         // W-list boxes of at most wd beads are summed directly (< 0: none)
  int eval_mode = 0;  // rpy::EVAL_SETS or rpy::EVAL_POLY
  int inject = -1;    // phase at which the next pass reports a HIP error (tests)
  int tuned = 0, tune_hit = 0;       // autotuned; choice taken from the cache
  double tune_err = 0.0;             // measured error of the tuned choice
  int device = 0;     // device current when the plan was built
  double a = 0, eta = 0, eps = 0;
  hipStream_t stream = nullptr;
  // The near field (P2P, overlap and direct W sums) runs on a second stream
  // of the plan, concurrently with the far-field chain on `stream`, into a
  // separate velocity buffer; events order the two, and the result is
  // combined on `stream`.
  hipStream_t near = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // M->L of the deepest level (sources need only S->M) runs on a third
  // stream while the upward pass continues on `stream`
  hipStream_t far2 = nullptr;
  hipEvent_t ev_p2m = nullptr, ev_m2l0 = nullptr;
  int sticky = 0;
  // matvec workspace, sized for `ws_nrc` right-hand sides per pass
  int ws_nrc = 0;   // right-hand sides per far-field pass the workspace holds
  int ws_nrn = 0;   // and per near-field group
  Work ws{};
  int64_t ws_bytes = 0;
  // Krylov workspace (rpy_sqrt_matvec), grown on demand
  double* kbuf = nullptr;
  int64_t kbuf_doubles = 0;
  double plan_ms = 0;
  // bead passes of the first tree built (bounding cubes, keys, sort, gather)
  double bead_pass_ms = 0;
  int sort_passes = 0;
  // per-phase timing
  int timing = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;  // (phase, start, stop)
  rpy_timings_t acc{};
};

// Bytes of each Work array for nrc right-hand sides per far-field pass and
// nrn per near-field group (sF and u hold a group).  Q carries 64 rows past
// the last bead that the S->M/S->L kernels may read (with zero weight); they
// must hold finite values (zeros).
static void ws_sizes(const rpy_plan_t* P, int nrc, int nrn, size_t sz[WS_N]) {
  const int64_t T = rpy::ncoef(P->p);
  const int64_t nbox = std::max(P->B.tree.nbox, 1);
  const int64_t n = std::max<int64_t>(P->B.n, 1);
  const size_t ex = sizeof(double2) * nbox * 4 * nrc * T;
  const size_t vb = sizeof(double) * 3 * nrc * n;
  int64_t dwb = 0, pvb = 0;
  const size_t dlb = (size_t)rpy::eval_sets_bytes(&P->B, P->ep, P->p, nrc, &dwb, &pvb);
  sz[0] = sz[1] = ex;
  sz[2] = sz[3] = sizeof(double) * 3 * std::max(nrc, nrn) * n;
  sz[4] = vb;
  sz[5] = sizeof(double) * 4 * nrc * (n + 64);
  sz[6] = dlb;
  sz[7] = (size_t)dwb;
  sz[8] = sizeof(double2) * std::max<int64_t>(P->B.nxshared, 1) * 4 * nrc * T;
  sz[9] = (size_t)pvb;
  sz[10] = P->precision == RPY_PREC_MIXED ? sizeof(float2) * nbox * 4 * nrc * T : 256;
}

static hipEvent_t get_event(rpy_plan_t* P) {
  if (!P->ev_pool.empty()) {
    hipEvent_t e = P->ev_pool.back();
    P->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs one phase, bracketed by events on its stream when timing is on.
// mc > 0: the step is a P2P launch on the matrix cores carrying mc
// right-hand sides, also accumulated on its own (events keyed phase +
// TIMED_MC)
constexpr int TIMED_MC = 0x100;
template <class F>
static hipError_t timed(rpy_plan_t* P, int phase, int launches, hipStream_t st, F&& f, int mc = 0) {
  if (!P->timing) return f();
  hipEvent_t a = get_event(P), b = get_event(P);
  if (a) (void)hipEventRecord(a, st);
  hipError_t e = f();
  if (b) (void)hipEventRecord(b, st);
  if (a && b) P->ev_pending.push_back({phase + (mc ? TIMED_MC : 0), {a, b}});
  P->acc.launches[phase] += launches;
  if (mc) {
    P->acc.p2p_mc_launches += launches;
    P->acc.p2p_mc_rhs += (int64_t)launches * mc;
  }
  return e;
}

static void fold_events(rpy_plan_t* P) {
  for (auto& pe : P->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      P->acc.ms[pe.first & (TIMED_MC - 1)] += ms;
      if (pe.first & TIMED_MC) P->acc.p2p_mc_ms += ms;
    }
    P->ev_pool.push_back(pe.second.first);
    P->ev_pool.push_back(pe.second.second);
  }
  P->ev_pending.clear();
}

static void free_ws(rpy_plan_t* P) {
  Work& w = P->ws;
  void* ps[] = {w.M, w.L, w.sF, w.u, w.uf, w.Q, w.DL, w.DW, w.XP, w.PV, w.M32};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  w = Work{};
  P->ws_nrc = 0;
  P->ws_nrn = 0;
  P->ws_bytes = 0;
}

static int alloc_ws(rpy_plan_t* P, int nrc, int nrn) {
  if (P->ws_nrc >= nrc && P->ws_nrn >= nrn) return 0;
  nrc = std::max(nrc, P->ws_nrc);
  nrn = std::max(nrn, P->ws_nrn);
  free_ws(P);
  size_t sz[WS_N];
  ws_sizes(P, nrc, nrn, sz);
  Work& w = P->ws;
  void** dst[WS_N] = {(void**)&w.M, (void**)&w.L, (void**)&w.sF, (void**)&w.u, (void**)&w.uf,
                      (void**)&w.Q, (void**)&w.DL, (void**)&w.DW, (void**)&w.XP, (void**)&w.PV,
                      (void**)&w.M32};
  int64_t tot = 0;
  // an injected allocation failure (rpy_plan_inject_error) hits half-way,
  // after some arrays are allocated, like a device that runs out of memory
  const int fail_at = P->inject == RPY_INJECT_ALLOC ? WS_N / 2 : WS_N;
  if (fail_at < WS_N) P->inject = -1;
  for (int k = 0; k < WS_N; ++k) {
    if (k == fail_at || hipMalloc(dst[k], sz[k]) != hipSuccess) {
      (void)hipGetLastError();
      *dst[k] = nullptr;
      free_ws(P);
      return -1;
    }
    tot += sz[k];
  }
  // zeroed once so that every row of Q, including the padding, is finite
  if (hipMemset(w.Q, 0, sz[5]) != hipSuccess) {
    free_ws(P);
    return -1;
  }
  P->ws_nrc = nrc;
  P->ws_nrn = nrn;
  P->ws_bytes = tot;
  return 0;
}

// One matvec group over right-hand sides r0 .. r0 + cn - 1: the near field
// (P2P, overlap correction, direct W sums) for the whole group on the second
// stream, the far field in passes of at most nrc right-hand sides on the
// plan stream, each pass combined with the group's near-field velocities as
// it finishes.  Every step runs only if all earlier ones were issued without
// error; the first error is returned and nothing after it is issued.
static hipError_t matvec_group(rpy_plan_t* P, const rpy::Launch& l, const Work& w, const double* forces, int nrhs,
                               int r0, int cn, int nrc, int mixed, double* velocities, bool untimed = false) {
  const rpy::Built& B = P->B;
  const int nlev = B.depth;
  const int64_t n3 = 3 * B.n;
  const bool haveO = B.lists[rpy::LO].len > 0, haveX = B.lists[rpy::LX].len > 0, haveW = B.lists[rpy::LW].len > 0;
  // timing mode 2 runs the near field on the plan stream too, so that each
  // phase's events measure that phase alone
  const bool fork = P->near && P->timing != 2;
  const hipStream_t s0 = P->stream, s1 = fork ? P->near : P->stream;
  rpy::Launch ln = l;
  ln.s = s1;
  // a phase named by rpy_plan_inject_error reports an error instead of running
  auto step = [&](int phase, int launches, hipStream_t st, auto&& f, int mc = 0) -> hipError_t {
    if (P->inject == phase) {
      P->inject = -1;
      return hipErrorLaunchFailure;
    }
    if (untimed) return f();
    return timed(P, phase, launches, st, f, mc);
  };
  hipError_t he = step(RPY_PH_PERMUTE, 1, s0, [&] { return rpy::permute_forces(l, forces, nrhs, r0, cn, w.sF); });
  // near field on s1, after the permute
  if (he == hipSuccess && fork) {
    he = hipEventRecord(P->ev_fork, s0);
    if (he == hipSuccess) he = hipStreamWaitEvent(s1, P->ev_fork, 0);
  }
  if (he == hipSuccess)
    he = step(RPY_PH_P2P, 1, s1, [&] { return rpy::run_p2p(ln, P->tiles, cn, w.sF, w.u, mixed); },
              cn >= rpy::NEAR_MC_RHS ? cn : 0);
  if (he == hipSuccess && haveO)
    he = step(RPY_PH_OVERLAP, 1, s1, [&] { return rpy::run_overlap(ln, P->tiles, cn, w.sF, w.u, mixed); });
  if (he == hipSuccess && haveW)
    he = step(RPY_PH_OVERLAP, 1, s1, [&] { return rpy::run_wdirect(ln, P->tiles, cn, w.sF, w.u, mixed); });
  if (he == hipSuccess && fork) he = hipEventRecord(P->ev_join, s1);
  // far field on s0, pass by pass over slices of the group's forces
  bool joined = !fork;
  for (int q0 = 0; he == hipSuccess && q0 < cn;) {
    const int c = cn - q0 >= nrc ? nrc : (cn - q0 >= 2 && nrc >= 2 ? 2 : 1);
    const double* sFq = w.sF + q0 * n3;
    const rpy::Exp e{w.M, w.L, w.Q, w.DL, w.DW, w.XP, w.PV, w.M32};
    he = step(RPY_PH_P2M, 1, s0, [&] { return rpy::run_p2m(l, c, sFq, e); });
    // the deepest level's M->L needs only S->M: on a third stream, beside
    // the upward pass (it writes L of other boxes than the second part)
    const bool split = fork && P->far2 && P->m2l_mode != 1;
    if (he == hipSuccess && split) {
      rpy::Launch l2 = l;
      l2.s = P->far2;
      he = hipEventRecord(P->ev_p2m, s0);
      if (he == hipSuccess) he = hipStreamWaitEvent(P->far2, P->ev_p2m, 0);
      if (he == hipSuccess) he = step(RPY_PH_M2L, 1, P->far2, [&] { return rpy::run_m2l_rot(l2, c, e, mixed, 0); });
      if (he == hipSuccess) he = hipEventRecord(P->ev_m2l0, P->far2);
    }
    if (he == hipSuccess) he = step(RPY_PH_M2M, nlev > 2 ? nlev - 2 : 0, s0, [&] { return rpy::run_m2m(l, c, e); });
    if (he == hipSuccess) he = step(RPY_PH_M2L, 1, s0, [&] {
      if (P->m2l_mode == 1) return rpy::run_m2l(l, c, e);
      return rpy::run_m2l_rot(l, c, e, mixed, split ? 1 : -1);
    });
    if (he == hipSuccess && split) he = hipStreamWaitEvent(s0, P->ev_m2l0, 0);
    if (he == hipSuccess && haveX) he = step(RPY_PH_P2L, 1, s0, [&] { return rpy::run_p2l(l, c, sFq, e); });
    if (he == hipSuccess) he = step(RPY_PH_L2L, nlev > 2 ? nlev - 2 : 0, s0, [&] { return rpy::run_l2l(l, c, e); });
    if (he == hipSuccess) he = step(RPY_PH_EVAL, 1, s0, [&] { return rpy::run_eval(l, P->ep, c, e, w.uf); });
    // join once, then near + far of this pass back to caller order
    if (he == hipSuccess && !joined) {
      he = hipStreamWaitEvent(s0, P->ev_join, 0);
      joined = true;
    }
    if (he == hipSuccess)
      he = step(RPY_PH_UNPERMUTE, 1, s0,
                [&] { return rpy::unpermute_velocities(l, w.u + q0 * n3, w.uf, r0 + q0, c, velocities); });
    if (P->timing && !untimed) P->acc.passes += 1;
    q0 += c;
  }
  return he;
}

// ---- fixed workspace of the allocation-free matvec ----------------------
// rpy_matvec_noalloc runs the matvec with its workspace in this file-scope
// device array instead of plan-owned allocations.  Each device that loads
// the library holds its own copy for the life of the process.  Host code
// never passes the array's name to a kernel: it resolves the device address
// with hipGetSymbolAddress, once per device, and uses that pointer.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES];  // device address of `scratch`, per device

// Address of `scratch` on the current device (resolved on first use).
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t he = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (he != hipSuccess) return he;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

__global__ void k_zero(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

// ---- measured autotuning (rpy_options.tune = 1) ---------------------------
// Candidate plans are built on the caller's beads and timed on random forces;
// each is accepted only if its measured relative L2 error at sampled targets,
// against the library's own FP64 direct sum there (run_direct_sample), is at
// most eps/2 (the margin the order table was calibrated with).  The fastest
// accepted candidate wins.  Candidates: the cost model's refinement limit s0
// and its ladder neighbours s0/1.5 and 1.5 s0; for each, orders from the
// table's down while the gate holds; for the fastest, both evaluation
// approaches.  Choices are cached for the life of the process, keyed by
// (bead-count bucket, uniform or adaptive tree, eps, precision, right-hand
// sides, systems); a repeated plan of the same class reuses them.
namespace {

struct TuneKey {
  int nbucket;    // round(4 log2 n)
  int adaptive;   // W/X lists present in the model's tree
  double eps;
  int precision;
  int nrhs;
  int nsys;
};
struct TuneEntry {
  TuneKey key;
  int leaf_size, order, eval_mode;
  double ms, err;
};
constexpr int TUNE_CACHE = 64;
std::mutex g_tune_mu;
TuneEntry g_tune[TUNE_CACHE];  // plain data: nothing runs at process exit
int g_ntune = 0;

bool same_key(const TuneKey& a, const TuneKey& b) {
  return a.nbucket == b.nbucket && a.adaptive == b.adaptive && a.eps == b.eps && a.precision == b.precision &&
         a.nrhs == b.nrhs && a.nsys == b.nsys;
}

// Standard normal numbers from a counter-based generator: splitmix64 of
// (seed, index) gives two uniforms, Box-Muller gives one normal.
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}
__global__ void k_fill_normal(double* x, int64_t m, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t h1 = splitmix64(seed ^ (2 * (uint64_t)i)), h2 = splitmix64(seed ^ (2 * (uint64_t)i + 1));
  const double u1 = ((h1 >> 11) + 1.0) * 0x1.0p-53, u2 = (h2 >> 11) * 0x1.0p-53;
  x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}
__global__ void k_gather_rows(const double* U, const int* idx, int k, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * k) return;
  out[i] = U[(int64_t)idx[i / 3] * 3 + i % 3];
}

struct TuneRun {
  double ms = 0, err = 0;
  bool ok = false;
};

}  // namespace

// Builds a plan with fixed parameters, times nrhs matvecs (best of two after a
// warm-up) and measures the error of right-hand side 0 at the sampled caller
// indices cidx against ref [k][3].
static rpy_status tune_try(int32_t nsys, const int64_t* counts, const double* positions, double a, double eta,
                           double eps, rpy_options o, const double* F, double* U, int nrhs, const int* cidx_d, int k,
                           const std::vector<double>& ref, double* gath_d, TuneRun* out, rpy_plan_t** keep) {
  o.tune = 0;
  rpy_plan_t* P = nullptr;
  rpy_status st = rpy_plan_batched(&P, nsys, counts, positions, a, eta, eps, &o);
  if (st != RPY_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = 1e300;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  for (int it = 0; he == hipSuccess && it < 3; ++it) {
    if (he == hipSuccess) he = hipEventRecord(e0, P->stream);
    st = rpy_matvec(P, nrhs, F, U);
    if (st != RPY_OK) break;
    if (he == hipSuccess) he = hipEventRecord(e1, P->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (it > 0) best = std::min(best, (double)ms);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  std::vector<double> got(3 * (size_t)k);
  if (st == RPY_OK && he == hipSuccess) {
    k_gather_rows<<<(3 * k + 255) / 256, 256, 0, P->stream>>>(U, cidx_d, k, gath_d);
    he = hipGetLastError();
    if (he == hipSuccess) he = hipMemcpyAsync(got.data(), gath_d, sizeof(double) * got.size(), hipMemcpyDeviceToHost,
                                              P->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(P->stream);
  }
  if (st == RPY_OK && he != hipSuccess) st = fail(RPY_EDEVICE, std::string("autotuning: ") + hipGetErrorString(he));
  if (st == RPY_OK) {
    double num = 0, den = 0;
    for (size_t i = 0; i < got.size(); ++i) {
      num += (got[i] - ref[i]) * (got[i] - ref[i]);
      den += ref[i] * ref[i];
    }
    out->ms = best;
    out->err = den > 0 ? std::sqrt(num / den) : 0.0;
    out->ok = std::isfinite(out->err) && out->err <= 0.5 * eps;
  }
  if (keep && st == RPY_OK) *keep = P;
  else rpy_plan_free(P);
  return st;
}

// Chooses leaf size, order and evaluation approach for o by measurement (or
// from the cache); fills o->leaf_size, o->order, o->eval_mode.
static rpy_status autotune(int32_t nsys, const int64_t* counts, const double* positions, double a, double eta,
                           double eps, rpy_options* o, int* cache_hit, double* tune_err) {
  int64_t n = 0;
  for (int s = 0; s < nsys; ++s) n += counts[s];
  *cache_hit = 0;
  *tune_err = 0;
  const int nrhs = std::max(1, o->nrhs);
  // the model's plan: its refinement limit, tree class and table order
  rpy_options om = *o;
  om.tune = 0;
  rpy_plan_t* P0 = nullptr;
  rpy_status st = rpy_plan_batched(&P0, nsys, counts, positions, a, eta, eps, &om);
  if (st != RPY_OK) return st;
  const int s0 = P0->leaf_size, p0 = P0->p;
  const int adaptive = P0->B.lists[rpy::LW].len > 0 || P0->B.lists[rpy::LX].len > 0;
  const TuneKey key{(int)std::lround(4.0 * std::log2((double)std::max<int64_t>(n, 1))), adaptive, eps, o->precision,
                    nrhs, nsys};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int i = 0; i < g_ntune; ++i)
      if (same_key(g_tune[i].key, key)) {
        o->leaf_size = g_tune[i].leaf_size;
        o->order = g_tune[i].order;
        o->eval_mode = g_tune[i].eval_mode;
        *cache_hit = 1;
        *tune_err = g_tune[i].err;
        rpy_plan_free(P0);
        return RPY_OK;
      }
  }
  if (n == 0) {
    rpy_plan_free(P0);
    return RPY_OK;
  }
  // random forces, sampled targets (spread over the tree order) and their
  // exact velocities (right-hand side 0)
  const int k = (int)std::min<int64_t>(n, 256);
  double *F = nullptr, *U = nullptr, *sF = nullptr, *refd = nullptr, *gath = nullptr;
  int *tidx = nullptr, *cidx = nullptr;
  std::vector<int> ht(k), hc(k), perm(n);
  std::vector<double> ref(3 * (size_t)k);
  hipStream_t s = P0->stream;
  hipError_t he = hipMalloc(&F, sizeof(double) * 3 * nrhs * n);
  if (he == hipSuccess) he = hipMalloc(&U, sizeof(double) * 3 * nrhs * n);
  if (he == hipSuccess) he = hipMalloc(&sF, sizeof(double) * 3 * n);
  if (he == hipSuccess) he = hipMalloc(&refd, sizeof(double) * 3 * k);
  if (he == hipSuccess) he = hipMalloc(&gath, sizeof(double) * 3 * k);
  if (he == hipSuccess) he = hipMalloc(&tidx, sizeof(int) * k);
  if (he == hipSuccess) he = hipMalloc(&cidx, sizeof(int) * k);
  if (he == hipSuccess) {
    const int64_t m = 3 * (int64_t)nrhs * n;
    k_fill_normal<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(F, m, 0x5eed5eedull);
    he = hipGetLastError();
  }
  if (he == hipSuccess) he = hipMemcpyAsync(perm.data(), P0->B.perm, sizeof(int) * n, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he == hipSuccess) {
    for (int i = 0; i < k; ++i) {
      ht[i] = (int)(((int64_t)i * n) / k);
      hc[i] = perm[ht[i]];
    }
    he = hipMemcpyAsync(tidx, ht.data(), sizeof(int) * k, hipMemcpyHostToDevice, s);
  }
  if (he == hipSuccess) he = hipMemcpyAsync(cidx, hc.data(), sizeof(int) * k, hipMemcpyHostToDevice, s);
  rpy::Launch l{&P0->B, &P0->tb, P0->p, a, eta, s, P0->wd};
  if (he == hipSuccess) he = rpy::permute_forces(l, F, nrhs, 0, 1, sF);
  if (he == hipSuccess) he = rpy::run_direct_sample(l, tidx, k, 1, sF, refd);
  if (he == hipSuccess) he = hipMemcpyAsync(ref.data(), refd, sizeof(double) * 3 * k, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  rpy_plan_free(P0);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    st = fail(RPY_ENOMEM, std::string("autotuning workspace: ") + hipGetErrorString(he));
  }
  int best_s = s0, best_p = p0, best_e = 0;
  double best_ms = 1e300, best_err = 0;
  auto consider = [&](int sl, int p, int ev, const TuneRun& r) {
    if (r.ok && r.ms < best_ms) {
      best_ms = r.ms;
      best_s = sl;
      best_p = p;
      best_e = ev;
      best_err = r.err;
    }
  };
  const int ladder[3] = {std::max(8, (int)(s0 / 1.5)), s0, (int)(s0 * 1.5)};
  for (int li = 0; st == RPY_OK && li < 3; ++li) {
    // orders from the table's value down while the gate holds
    for (int p = p0; st == RPY_OK && p >= 1; --p) {
      rpy_options oc = *o;
      oc.leaf_size = ladder[li];
      oc.order = p;
      oc.eval_mode = 0;
      TuneRun r;
      st = tune_try(nsys, counts, positions, a, eta, eps, oc, F, U, nrhs, cidx, k, ref, gath, &r, nullptr);
      if (st != RPY_OK) break;
      consider(ladder[li], p, 0, r);
      if (!r.ok) break;
    }
  }
  // the other evaluation approach for the winner
  if (st == RPY_OK && best_ms < 1e300 && best_p <= rpy::EVAL_POLY_MAX_ORDER) {
    for (int ev = 1; ev <= 2; ++ev) {
      rpy_options oc = *o;
      oc.leaf_size = best_s;
      oc.order = best_p;
      oc.eval_mode = ev;
      TuneRun r;
      st = tune_try(nsys, counts, positions, a, eta, eps, oc, F, U, nrhs, cidx, k, ref, gath, &r, nullptr);
      if (st != RPY_OK) break;
      if (r.ok && r.ms < best_ms) {
        best_ms = r.ms;
        best_e = ev;
        best_err = r.err;
      }
    }
  }
  void* bufs[] = {F, U, sF, refd, gath, tidx, cidx};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (st != RPY_OK) return st;
  if (best_ms >= 1e300) {
    // no candidate met the gate: the model's choice with the table's order
    best_s = s0;
    best_p = p0;
    best_e = 0;
  }
  o->leaf_size = best_s;
  o->order = best_p;
  o->eval_mode = best_e;
  *tune_err = best_err;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  TuneEntry& e = g_tune[g_ntune < TUNE_CACHE ? g_ntune++ : (TUNE_CACHE - 1)];
  e = TuneEntry{key, best_s, best_p, best_e, best_ms, best_err};
  return RPY_OK;
}

extern "C" {

void rpy_default_options(rpy_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->struct_size = sizeof(rpy_options);
  opt->precision = RPY_PREC_FP64;
  opt->max_depth = 14;
}

const char* rpy_status_string(rpy_status s) {
  switch (s) {
    case RPY_OK: return "ok";
    case RPY_EINVAL: return "invalid argument";
    case RPY_ENONFINITE: return "non-finite position";
    case RPY_ENOMEM: return "out of device memory";
    case RPY_EDEVICE: return "HIP error";
    case RPY_EUNSUPPORTED: return "unsupported option";
  }
  return "unknown status";
}

const char* rpy_last_error(void) { return g_last_error; }

rpy_status rpy_plan_batched(rpy_plan_t** out, int32_t nsys, const int64_t* counts, const double* positions,
                            double a, double eta, double eps, const rpy_options* opt) {
  auto t0 = std::chrono::steady_clock::now();
  if (!out) return fail(RPY_EINVAL, "out is NULL");
  *out = nullptr;
  if (nsys < 1 || !counts) return fail(RPY_EINVAL, "nsys < 1 or counts is NULL");
  int64_t n = 0;
  for (int s = 0; s < nsys; ++s) {
    if (counts[s] < 0) return fail(RPY_EINVAL, "negative bead count");
    n += counts[s];
  }
  if (n > 0x7fffffffLL - 1) return fail(RPY_EINVAL, "too many beads (limit 2^31 - 2)");
  if (n > 0 && !positions) return fail(RPY_EINVAL, "positions is NULL");
  if (!(a > 0) || !std::isfinite(a)) return fail(RPY_EINVAL, "radius a must be finite and > 0");
  if (!(eta > 0) || !std::isfinite(eta)) return fail(RPY_EINVAL, "viscosity eta must be finite and > 0");
  if (!(eps >= 1e-12 && eps <= 1e-1)) return fail(RPY_EINVAL, "eps must lie in [1e-12, 1e-1]");
  rpy_options o;
  rpy_default_options(&o);
  if (opt) {
    if (opt->struct_size < offsetof(rpy_options, stream) + sizeof(void*))
      return fail(RPY_EINVAL, "options.struct_size too small");
    // fields past the caller's struct_size keep their defaults
    std::memcpy(&o, opt, std::min<size_t>(opt->struct_size, sizeof(rpy_options)));
    o.struct_size = sizeof(rpy_options);
  }
  if (o.precision != RPY_PREC_FP64 && o.precision != RPY_PREC_MIXED)
    return fail(RPY_EINVAL, "unknown precision");
  if (o.order < 0 || o.order > rpy::MAX_ORDER) return fail(RPY_EINVAL, "order must be 0..27");
  if (o.leaf_size < 0) return fail(RPY_EINVAL, "leaf_size must be >= 0");
  if (o.max_depth == 0) o.max_depth = 14;
  if (o.max_depth < 1 || o.max_depth > 21) return fail(RPY_EINVAL, "max_depth must be 1..21");
  if (o.nrhs < 0) return fail(RPY_EINVAL, "nrhs must be >= 0");
  if (o.m2l_mode < 0 || o.m2l_mode > 2) return fail(RPY_EINVAL, "m2l_mode must be 0, 1 or 2");
  if (o.w_direct < -1) return fail(RPY_EINVAL, "w_direct must be -1, 0 or a bead count");
  if (o.eval_mode < 0 || o.eval_mode > 2) return fail(RPY_EINVAL, "eval_mode must be 0, 1 or 2");
  if (o.eval_mode == 2 && o.order > rpy::EVAL_POLY_MAX_ORDER)
    return fail(RPY_EUNSUPPORTED, "polynomial evaluation is built up to order 21");
  if (o.tune < 0 || o.tune > 1) return fail(RPY_EINVAL, "tune must be 0 or 1");
  int tuned = 0, tune_hit = 0;
  double tune_err = 0.0;
  if (o.tune == 1 && o.leaf_size == 0 && o.order == 0) {
    const rpy_status ts = autotune(nsys, counts, positions, a, eta, eps, &o, &tune_hit, &tune_err);
    if (ts != RPY_OK) return ts;
    tuned = 1;
  }

  rpy_plan_t* P = new rpy_plan_t();
  if (hipGetDevice(&P->device) != hipSuccess) {
    (void)hipGetLastError();
    delete P;
    return fail(RPY_EDEVICE, "hipGetDevice failed");
  }
  P->a = a;
  P->eta = eta;
  P->eps = eps;
  P->precision = o.precision;
  P->stream = (hipStream_t)o.stream;
  P->p = o.order;
  P->leaf_size = o.leaf_size;
  P->max_depth = o.max_depth;
  // library choice: the rotation operator (measured 5x faster than the dense
  // one at p = 16 in FP64); the mixed form runs it in FP32.
  P->m2l_mode = o.m2l_mode != 0 ? o.m2l_mode : 2;
  P->wd = o.w_direct;
  P->eval_mode = o.eval_mode;

  std::vector<int64_t> sb(nsys + 1, 0);
  for (int s = 0; s < nsys; ++s) sb[s + 1] = sb[s] + counts[s];
  rpy::Error err{0, ""};
  int rc = 0;
  if (o.leaf_size > 0) {
    rpy::BuildArgs ba{n, nsys, sb.data(), positions, P->leaf_size, P->max_depth, a, P->stream};
    rc = rpy::build_tree(ba, &P->B, &err);
    P->bead_pass_ms = P->B.bead_pass_ms;
    P->sort_passes = P->B.sort_passes;
  } else {
    // Refinement limit chosen by the cost model over a ladder of limits
    // (64 * 1.5^k) up to the largest system; limits that provably give the
    // tree already built are skipped, so only distinct trees are built.  The
    // modelled time is not unimodal in the limit (partly refined trees in
    // between need a higher order), so the ladder is climbed until a tree's
    // near field alone, which only grows as the tree coarsens, costs more
    // than the best whole matvec.
    // Every trial tree after the first copies the bounding cubes, Morton
    // keys and sorted order of the best one so far (they do not depend on
    // the limit), into the bead arrays of the last discarded tree when there
    // is one.  Trial trees are built without the O list: the overlapping
    // bead pairs are fixed by the geometry, not by the tree, and dense
    // clusters with small leaves make that list very long.  The chosen tree
    // is rebuilt with it when some leaf is smaller than 2a.
    int64_t nmax = 1;
    for (int s = 0; s < nsys; ++s) nmax = std::max<int64_t>(nmax, counts[s]);
    double best = 0, sl = 64;
    bool need_o = false;
    rpy::Spare spare;  // bead arrays of the last discarded tree
    for (;;) {
      const int cand = (int)sl;
      rpy::Built Bc;
      rpy::BuildArgs ba{n, nsys, sb.data(), positions, cand, P->max_depth, a, P->stream};
      ba.skip_o = true;
      ba.presorted = P->leaf_size != 0 ? &P->B : nullptr;
      ba.spare = &spare;
      rc = rpy::build_tree(ba, &Bc, &err);
      if (!ba.presorted) {
        P->bead_pass_ms = Bc.bead_pass_ms;
        P->sort_passes = Bc.sort_passes;
      }
      TreeCost tc;
      if (rc == 0)
        rc = model_tree(Bc, o.order, eps, o.precision == RPY_PREC_MIXED, P->max_depth, o.nrhs, o.w_direct, &tc);
      if (rc != 0) {
        rpy::free_built(&Bc);
        break;
      }
      const bool first = P->leaf_size == 0;
      if (first || tc.ns < best) {
        if (!first) rpy::retire_built(&P->B, &spare);
        P->B = Bc;
        P->leaf_size = cand;
        best = tc.ns;
        need_o = false;
        for (int s = 0; s < nsys; ++s)
          if (ldexp(P->B.side[s], -P->B.depth) < 2.0 * a) need_o = true;
      } else {
        rpy::retire_built(&Bc, &spare);
      }
      if (cand >= nmax || tc.same_hi > nmax) break;  // one leaf per system from here on
      // coarser trees only add near-field pairs: once this tree's near field
      // alone costs more than the best whole matvec, no larger limit can win
      if (tc.near_ns > best) break;
      do sl *= 1.5;
      while ((int64_t)sl < tc.same_hi);
    }
    if (rc == 0 && need_o) {
      rpy::Built Bo;
      rpy::BuildArgs ba{n, nsys, sb.data(), positions, P->leaf_size, P->max_depth, a, P->stream};
      ba.presorted = &P->B;
      ba.spare = &spare;
      rc = rpy::build_tree(ba, &Bo, &err);
      rpy::free_built(&P->B);
      P->B = Bo;
    }
    rpy::free_spare(&spare);
  }
  if (rc == 0 && P->p == 0)
    P->p = order_for_eps(eps, P->B.lists[rpy::LW].len > 0 || P->B.lists[rpy::LX].len > 0);
  if (P->wd == 0) P->wd = rpy::wdirect_default(P->p);
  if (rc == 0 && P->eval_mode == 2 && P->p > rpy::EVAL_POLY_MAX_ORDER) {
    rpy_plan_free(P);
    return fail(RPY_EUNSUPPORTED, "polynomial evaluation is built up to order 21");
  }
  // library choice: the component polynomials at low orders (fewer
  // operations per target), the derivative sets above
  if (P->eval_mode == 0) P->eval_mode = P->p <= EVAL_POLY_AUTO_MAX ? rpy::EVAL_POLY : rpy::EVAL_SETS;
  if (rc == 0) rc = rpy::make_tables(P->p, &P->tb, P->stream, &err);
  if (rc == 0) rc = rpy::make_tiles(&P->B, 128, &P->tiles, P->stream, &err);
  if (rc == 0) rc = rpy::make_eval_plan(&P->B, P->p, P->wd, P->eval_mode, &P->ep, P->stream, &err);
  if (rc == 0) rc = rpy::make_m2l_map(&P->B, P->stream, &err);
  if (rc == 0) rc = rpy::make_p2l_work(&P->B, P->stream, &err);
  if (rc == 0) {
    // default priority (no priority argument); without it the near field
    // runs on the plan's stream
    if (hipStreamCreateWithFlags(&P->near, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      if (P->near) (void)hipStreamDestroy(P->near);
      if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
      if (P->ev_join) (void)hipEventDestroy(P->ev_join);
      P->near = nullptr;
      P->ev_fork = P->ev_join = nullptr;
    }
    if (hipStreamCreateWithFlags(&P->far2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_p2m, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P->ev_m2l0, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      if (P->far2) (void)hipStreamDestroy(P->far2);
      if (P->ev_p2m) (void)hipEventDestroy(P->ev_p2m);
      if (P->ev_m2l0) (void)hipEventDestroy(P->ev_m2l0);
      P->far2 = nullptr;
      P->ev_p2m = P->ev_m2l0 = nullptr;
    }
  }

  if (rc != 0) {
    rpy_status st = rc == -2 ? RPY_ENONFINITE : rc == -3 ? RPY_ENOMEM : RPY_EDEVICE;
    set_error(err.msg);
    rpy_plan_free(P);
    return st;
  }
  P->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  P->tuned = tuned;
  P->tune_hit = tune_hit;
  P->tune_err = tune_err;
  *out = P;
  return RPY_OK;
}

rpy_status rpy_plan(rpy_plan_t** out, int64_t n, const double* positions, double a, double eta, double eps,
                    const rpy_options* opt) {
  if (n < 0) {
    if (out) *out = nullptr;
    return fail(RPY_EINVAL, "n < 0");
  }
  return rpy_plan_batched(out, 1, &n, positions, a, eta, eps, opt);
}

rpy_status rpy_matvec(rpy_plan_t* P, int32_t nrhs, const double* forces, double* velocities) {
  if (!P) return fail(RPY_EINVAL, "plan is NULL");
  if (P->sticky) return fail(RPY_EDEVICE, "plan is in an error state from an earlier HIP failure");
  if (nrhs < 1) return fail(RPY_EINVAL, "nrhs < 1");
  if (P->B.n == 0) return RPY_OK;
  if (!forces || !velocities) return fail(RPY_EINVAL, "forces or velocities is NULL");
  // right-hand sides per pass: 4, 2 or 1, limited by device memory
  const int64_t T = rpy::ncoef(P->p);
  int nrc = nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1);
  if (P->p > rpy::MAX_ORDER_MULTI) nrc = 1;  // the high-order kernels take one right-hand side
  while (nrc > 1 && 2.0 * P->B.tree.nbox * 4.0 * nrc * T * 16.0 > 64e9) nrc /= 2;
  // near-field groups: 16 (matrix cores) or up to 8 right-hand sides share each pair's geometry
  const int nrn = std::max(nrc, near_group_max(nrhs, P->precision == RPY_PREC_MIXED));
  if (alloc_ws(P, nrc, nrn) != 0) return fail(RPY_ENOMEM, "cannot allocate the matvec workspace");
  rpy::Launch l{&P->B, &P->tb, P->p, P->a, P->eta, P->stream, P->wd};
  const int mixed = P->precision == RPY_PREC_MIXED;
  for (int r0 = 0; r0 < nrhs;) {
    const int cn = near_group(nrhs - r0, nrn, mixed);
    const hipError_t he = matvec_group(P, l, P->ws, forces, nrhs, r0, cn, std::min(nrc, cn), mixed, velocities);
    if (he != hipSuccess) {
      P->sticky = 1;
      return fail(RPY_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(he));
    }
    r0 += cn;
  }
  return RPY_OK;
}

rpy_status rpy_matvec_noalloc(rpy_plan_t* P, int32_t nrhs, const double* forces, double* velocities) {
  if (!P) return fail(RPY_EINVAL, "plan is NULL");
  if (P->sticky) return fail(RPY_EDEVICE, "plan is in an error state from an earlier HIP failure");
  if (nrhs < 1) return fail(RPY_EINVAL, "nrhs < 1");
  if (P->B.n == 0) return RPY_OK;
  if (!forces || !velocities) return fail(RPY_EINVAL, "forces or velocities is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != P->device)
    return fail(RPY_EINVAL, "the plan's device must be the current device");
  if (dev < 0 || dev >= MAX_DEVICES) return fail(RPY_EUNSUPPORTED, "device ordinal beyond 63");
  // right-hand sides per far-field pass and near-field group as in
  // rpy_matvec, halved until the workspace fits the fixed scratch
  int nrc = nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1);
  if (P->p > rpy::MAX_ORDER_MULTI) nrc = 1;
  int nrn = std::max(nrc, near_group_max(nrhs, P->precision == RPY_PREC_MIXED));
  size_t sz[WS_N], tot = 0;
  for (;;) {
    ws_sizes(P, nrc, nrn, sz);
    tot = 0;
    for (int k = 0; k < WS_N; ++k) tot += align256(sz[k]);
    if (tot <= NOALLOC_SCRATCH_BYTES || nrn == 1) break;
    if (nrn > nrc) nrn /= 2;
    else nrc = nrn = nrc / 2;
  }
  if (tot > NOALLOC_SCRATCH_BYTES)
    return fail(RPY_ENOMEM, "the matvec workspace of this plan (" + std::to_string(tot) +
                                " bytes for one right-hand side per pass) exceeds the " +
                                std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte fixed scratch of rpy_matvec_noalloc");
  void* base = nullptr;
  hipError_t he = scratch_address(dev, &base);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    return fail(RPY_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(he));
  }
  Work w;
  {
    unsigned char* q = static_cast<unsigned char*>(base);
    void** dst[WS_N] = {(void**)&w.M, (void**)&w.L, (void**)&w.sF, (void**)&w.u, (void**)&w.uf,
                        (void**)&w.Q, (void**)&w.DL, (void**)&w.DW, (void**)&w.XP, (void**)&w.PV,
                        (void**)&w.M32};
    for (int k = 0; k < WS_N; ++k) {
      *dst[k] = q;
      q += align256(sz[k]);
    }
  }
  // the 64 charge rows past the last bead are read with zero weight and must
  // be finite: cleared by a kernel on every call (earlier calls leave other
  // contents in the scratch)
  const int64_t pad = (int64_t)64 * 4 * nrc;
  k_zero<<<(unsigned)((pad + 255) / 256), 256, 0, P->stream>>>(w.Q + P->B.n * 4 * nrc, pad);
  he = hipGetLastError();
  rpy::Launch l{&P->B, &P->tb, P->p, P->a, P->eta, P->stream, P->wd};
  const int mixed = P->precision == RPY_PREC_MIXED;
  for (int r0 = 0; he == hipSuccess && r0 < nrhs;) {
    const int cn = near_group(nrhs - r0, nrn, mixed);
    he = matvec_group(P, l, w, forces, nrhs, r0, cn, std::min(nrc, cn), mixed, velocities, true);
    r0 += cn;
  }
  if (he != hipSuccess) {
    P->sticky = 1;
    return fail(RPY_EDEVICE, std::string("kernel launch failed: ") + hipGetErrorString(he));
  }
  return RPY_OK;
}

rpy_status rpy_sqrt_matvec(rpy_plan_t* P, int32_t nrhs, const double* z, double* y, double tol, int32_t max_iter,
                           rpy_sqrt_info_t* info) {
  if (info) *info = rpy_sqrt_info_t{0, 0, 0.0, 0.0};
  if (!P) return fail(RPY_EINVAL, "plan is NULL");
  if (P->sticky) return fail(RPY_EDEVICE, "plan is in an error state from an earlier HIP failure");
  if (nrhs < 1 || nrhs > 65535) return fail(RPY_EINVAL, "nrhs must be 1..65535");
  if (!(tol > 0.0 && tol < 1.0)) return fail(RPY_EINVAL, "tol must be in (0, 1)");
  if (max_iter < 1 || max_iter > 100) return fail(RPY_EINVAL, "max_iter must be 1..100");
  if (P->B.n == 0) {
    if (info) info->converged = 1;
    return RPY_OK;
  }
  if (!z || !y) return fail(RPY_EINVAL, "z or y is NULL");
  if (z == y) return fail(RPY_EINVAL, "y may not alias z");
  const int64_t L = 3 * P->B.n;
  const int kcap = max_iter + 1;
  const int64_t set = (int64_t)nrhs * L;
  const int64_t npart = rpy::krylov_part_doubles(L, kcap, nrhs);
  // basis [kcap][nrhs][L], w [nrhs][L], partial sums, 3 coefficient blocks [nrhs][kcap], scales [nrhs]
  const int64_t need = kcap * set + set + npart + 3 * (int64_t)nrhs * kcap + nrhs;
  hipStream_t st = P->stream;
  if (P->kbuf_doubles < need) {
    if (P->kbuf) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(P->kbuf);
    }
    P->kbuf = nullptr;
    P->kbuf_doubles = 0;
    if (hipMalloc(&P->kbuf, sizeof(double) * need) != hipSuccess) {
      (void)hipGetLastError();
      P->kbuf = nullptr;
      return fail(RPY_ENOMEM, "cannot allocate the Krylov workspace");
    }
    P->kbuf_doubles = need;
  }
  double* V = P->kbuf;
  double* W = V + kcap * set;
  double* part = W + set;
  double* cA = part + npart;
  double* cB = cA + (int64_t)nrhs * kcap;
  double* cF = cB + (int64_t)nrhs * kcap;
  double* sc = cF + (int64_t)nrhs * kcap;
  auto dev = [&](hipError_t he) {
    if (he != hipSuccess) {
      (void)hipGetLastError();
      P->sticky = 1;
      return fail(RPY_EDEVICE, std::string("Krylov step failed: ") + hipGetErrorString(he));
    }
    return RPY_OK;
  };
  std::vector<double> hA((size_t)nrhs * kcap), hB((size_t)nrhs * kcap), hs(nrhs);
  auto fetch = [&](const double* d, std::vector<double>& h) {
    hipError_t he = hipMemcpyAsync(h.data(), d, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    return he;
  };
  // beta_0 = |z|, v_0 = z / beta_0
  rpy_status rs = dev(rpy::krylov_mdot(z, 0, 1, z, L, nrhs, kcap, part, cA, st));
  if (rs == RPY_OK) rs = dev(fetch(cA, hA));
  if (rs != RPY_OK) return rs;
  std::vector<double> beta0(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    beta0[r] = std::sqrt(std::max(hA[(size_t)r * kcap], 0.0));
    hs[r] = beta0[r] > 0.0 ? 1.0 / beta0[r] : 0.0;
  }
  rs = dev(hipMemcpyAsync(sc, hs.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
  if (rs == RPY_OK) rs = dev(rpy::krylov_comb(nullptr, 0, 0, kcap, cA, 1.0, z, 1.0, sc, L, nrhs, V, st));
  if (rs != RPY_OK) return rs;

  // per right-hand side: tridiagonal entries, coefficients of y in the basis
  std::vector<std::vector<double>> alpha(nrhs), beta(nrhs), f(nrhs);
  std::vector<int> done(nrhs, 0);
  std::vector<double> change(nrhs, 0.0), ritz(nrhs, 0.0);
  for (int r = 0; r < nrhs; ++r)
    if (beta0[r] == 0.0) done[r] = 1;  // y = 0
  int steps = 0, used = 1;
  for (int k = 0; k < max_iter; ++k) {
    bool all = true;
    for (int r = 0; r < nrhs; ++r) all = all && done[r];
    if (all) break;
    const double* vk = V + k * set;
    rs = rpy_matvec(P, nrhs, vk, W);
    if (rs != RPY_OK) return rs;
    steps = k + 1;
    // two passes of classical Gram-Schmidt against v_0..v_k
    rs = dev(rpy::krylov_mdot(V, set, k + 1, W, L, nrhs, kcap, part, cA, st));
    if (rs == RPY_OK) rs = dev(rpy::krylov_comb(V, set, k + 1, kcap, cA, -1.0, W, 1.0, nullptr, L, nrhs, W, st));
    if (rs == RPY_OK) rs = dev(rpy::krylov_mdot(V, set, k + 1, W, L, nrhs, kcap, part, cB, st));
    if (rs == RPY_OK) rs = dev(rpy::krylov_comb(V, set, k + 1, kcap, cB, -1.0, W, 1.0, nullptr, L, nrhs, W, st));
    if (rs == RPY_OK) rs = dev(fetch(cA, hA));
    if (rs == RPY_OK) rs = dev(fetch(cB, hB));
    // |w|^2 into cF's first column
    if (rs == RPY_OK) rs = dev(rpy::krylov_mdot(W, 0, 1, W, L, nrhs, kcap, part, cF, st));
    std::vector<double> hn((size_t)nrhs * kcap);
    if (rs == RPY_OK) rs = dev(fetch(cF, hn));
    if (rs != RPY_OK) return rs;
    for (int r = 0; r < nrhs; ++r) {
      if (done[r]) continue;
      const double a = hA[(size_t)r * kcap + k] + hB[(size_t)r * kcap + k];
      const double b = std::sqrt(std::max(hn[(size_t)r * kcap], 0.0));
      alpha[r].push_back(a);
      beta[r].push_back(b);
      // T_k = tridiag(beta_1..beta_k; alpha_0..alpha_k; beta_1..beta_k)
      const int m = k + 1;
      std::vector<double> lam, Q;
      rpy::tridiag_eig(m, alpha[r], beta[r], lam, Q);
      // y = beta_0 V Q sqrt(Lambda) Q^T e_1
      std::vector<double> g(m, 0.0);
      double lmin = lam[0], lmax = 0.0;
      for (int q = 0; q < m; ++q) {
        lmin = std::min(lmin, lam[q]);
        lmax = std::max(lmax, std::fabs(lam[q]));
        const double w = std::sqrt(std::max(lam[q], 0.0)) * Q[q];  // Q[0][q] = e_1 . column q
        for (int i = 0; i < m; ++i) g[i] += Q[(size_t)i * m + q] * w;
      }
      double dn = 0.0, gn = 0.0;
      for (int i = 0; i < m; ++i) {
        g[i] *= beta0[r];
        const double prev = i < (int)f[r].size() ? f[r][i] : 0.0;
        dn += (g[i] - prev) * (g[i] - prev);
        gn += g[i] * g[i];
      }
      change[r] = k == 0 ? 1.0 : (gn > 0.0 ? std::sqrt(dn / gn) : 0.0);
      ritz[r] = lmin;
      f[r] = g;
      used = std::max(used, m);
      // converged, or the Krylov space is exhausted (D v_k lies in the span)
      if ((k > 0 && change[r] <= tol) || b <= 1e-14 * std::max(lmax, 1e-300)) done[r] = 1;
    }
    bool fin = true;
    for (int r = 0; r < nrhs; ++r) fin = fin && done[r];
    if (fin || k + 1 == max_iter) break;
    // v_{k+1} = w / beta_{k+1} (zero for the right-hand sides that are done)
    for (int r = 0; r < nrhs; ++r) {
      const double b = beta[r].empty() ? 0.0 : beta[r].back();
      hs[r] = (!done[r] && b > 0.0) ? 1.0 / b : 0.0;
    }
    rs = dev(hipMemcpyAsync(sc, hs.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
    if (rs == RPY_OK) rs = dev(rpy::krylov_comb(nullptr, 0, 0, kcap, cA, 1.0, W, 1.0, sc, L, nrhs, V + (k + 1) * set, st));
    if (rs == RPY_OK) rs = dev(hipStreamSynchronize(st));  // hs is reused next step
    if (rs != RPY_OK) return rs;
  }
  // y = sum_j f_j v_j
  std::vector<double> hf((size_t)nrhs * kcap, 0.0);
  for (int r = 0; r < nrhs; ++r)
    for (size_t i = 0; i < f[r].size(); ++i) hf[(size_t)r * kcap + i] = f[r][i];
  rs = dev(hipMemcpyAsync(cF, hf.data(), sizeof(double) * hf.size(), hipMemcpyHostToDevice, st));
  if (rs == RPY_OK) rs = dev(rpy::krylov_comb(V, set, used, kcap, cF, 1.0, nullptr, 0.0, nullptr, L, nrhs, y, st));
  if (rs == RPY_OK) rs = dev(hipStreamSynchronize(st));
  if (rs != RPY_OK) return rs;
  if (info) {
    info->iterations = steps;
    int conv = 1;
    double ch = 0.0, rm = 0.0;
    bool first = true;
    for (int r = 0; r < nrhs; ++r) {
      if (beta0[r] == 0.0) continue;
      conv = conv && done[r];
      ch = std::max(ch, change[r]);
      rm = first ? ritz[r] : std::min(rm, ritz[r]);
      first = false;
    }
    info->converged = conv;
    info->rel_change = ch;
    info->min_ritz = rm;
  }
  return RPY_OK;
}

rpy_status rpy_plan_stats(const rpy_plan_t* P, rpy_plan_stats_t* out) {
  if (!P || !out) return fail(RPY_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->n = P->B.n;
  out->nsys = P->B.nsys;
  out->order = P->p;
  out->leaf_size = P->leaf_size;
  out->depth = P->B.depth;
  out->precision = P->precision;
  out->m2l_mode = P->m2l_mode;
  out->nbox = P->B.tree.nbox;
  out->nleaf = P->B.nleaf;
  for (int L = 0; L < 5; ++L) out->list_len[L] = P->B.lists[L].len;
  out->device_bytes = P->B.bytes + P->tb.bytes + P->ws_bytes + (int64_t)(sizeof(int4) + 6 * sizeof(double)) * P->tiles.n;
  out->plan_ms = P->plan_ms;
  out->w_direct = P->wd;
  out->eval_mode = P->eval_mode;
  out->tuned = P->tuned ? (P->tune_hit ? 2 : 1) : 0;
  out->tune_err = P->tune_err;
  out->p2l_items = P->B.nxwork;
  out->p2l_split_boxes = P->B.nxred;
  out->bead_pass_ms = P->bead_pass_ms;
  out->sort_passes = P->sort_passes;
  return RPY_OK;
}

rpy_status rpy_plan_inject_error(rpy_plan_t* P, int32_t phase) {
  if (!P) return fail(RPY_EINVAL, "plan is NULL");
  if ((phase < -1 || phase >= RPY_NPHASE) && phase != RPY_INJECT_ALLOC)
    return fail(RPY_EINVAL, "phase must be -1, a rpy_phase or RPY_INJECT_ALLOC");
  P->inject = phase;
  return RPY_OK;
}

rpy_status rpy_plan_export(const rpy_plan_t* P, int64_t* perm, uint64_t* keys, int64_t* boxes, int64_t* offsets,
                           int64_t* entries) {
  if (!P) return fail(RPY_EINVAL, "plan is NULL");
  const rpy::Built& B = P->B;
  const int64_t n = B.n;
  const int nbox = B.tree.nbox;
  if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(RPY_EDEVICE, "stream synchronisation failed");
  auto d2h_int = [&](const int* src, int64_t cnt, std::vector<int>& dst) -> bool {
    dst.resize(std::max<int64_t>(cnt, 1));
    if (cnt == 0) return true;
    return hipMemcpy(dst.data(), src, sizeof(int) * cnt, hipMemcpyDeviceToHost) == hipSuccess;
  };
  std::vector<int> tmp;
  if (perm && n) {
    if (!d2h_int(B.perm, n, tmp)) return fail(RPY_EDEVICE, "copy failed");
    for (int64_t i = 0; i < n; ++i) perm[i] = tmp[i];
  }
  if (keys && n)
    if (hipMemcpy(keys, B.keys, sizeof(uint64_t) * n, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(RPY_EDEVICE, "copy failed");
  if (boxes && nbox) {
    const int* f[8] = {B.tree.level, B.tree.ax, B.tree.ay, B.tree.az, B.tree.begin, B.tree.end, B.tree.parent,
                       B.tree.child};
    for (int k = 0; k < 8; ++k) {
      if (!d2h_int(f[k], nbox, tmp)) return fail(RPY_EDEVICE, "copy failed");
      for (int b = 0; b < nbox; ++b) boxes[(int64_t)b * 8 + k] = tmp[b];
    }
  }
  int64_t e = 0;
  for (int L = 0; L < 5; ++L) {
    if (offsets) {
      if (!d2h_int(B.lists[L].off, nbox + 1, tmp)) return fail(RPY_EDEVICE, "copy failed");
      for (int b = 0; b <= nbox; ++b) offsets[(int64_t)L * (nbox + 1) + b] = tmp[b];
    }
    if (entries) {
      if (!d2h_int(B.lists[L].ent, B.lists[L].len, tmp)) return fail(RPY_EDEVICE, "copy failed");
      for (int64_t i = 0; i < B.lists[L].len; ++i) entries[e + i] = tmp[i];
    }
    e += B.lists[L].len;
  }
  return RPY_OK;
}

rpy_status rpy_plan_set_timing(rpy_plan_t* P, int32_t enable) {
  if (!P) return fail(RPY_EINVAL, "plan is NULL");
  if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(RPY_EDEVICE, "stream synchronisation failed");
  fold_events(P);
  P->acc = rpy_timings_t{};
  if (enable < 0 || enable > 2) return fail(RPY_EINVAL, "timing mode must be 0, 1 or 2");
  P->timing = enable;
  return RPY_OK;
}

rpy_status rpy_plan_timings(rpy_plan_t* P, rpy_timings_t* out) {
  if (!P || !out) return fail(RPY_EINVAL, "NULL argument");
  if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(RPY_EDEVICE, "stream synchronisation failed");
  fold_events(P);
  *out = P->acc;
  return RPY_OK;
}

void rpy_plan_free(rpy_plan_t* P) {
  if (!P) return;
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  else (void)hipDeviceSynchronize();
  if (P->near) (void)hipStreamSynchronize(P->near);
  if (P->far2) (void)hipStreamSynchronize(P->far2);
  fold_events(P);
  if (P->far2) (void)hipStreamDestroy(P->far2);
  if (P->ev_p2m) (void)hipEventDestroy(P->ev_p2m);
  if (P->ev_m2l0) (void)hipEventDestroy(P->ev_m2l0);
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  if (P->near) (void)hipStreamDestroy(P->near);
  for (hipEvent_t e : P->ev_pool) (void)hipEventDestroy(e);
  free_ws(P);
  if (P->kbuf) (void)hipFree(P->kbuf);
  rpy::free_tables(&P->tb);
  if (P->tiles.t) (void)hipFree(P->tiles.t);
  if (P->tiles.box) (void)hipFree(P->tiles.box);
  rpy::free_eval_plan(&P->ep);
  rpy::free_built(&P->B);
  delete P;
}

}  // extern "C"
