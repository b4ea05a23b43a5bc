// Declarations of the matvec kernels' launchers (fmm.hip, nearfield.hip).
#pragma once
#include "common.h"

namespace rpy {

// Expansion storage: for every box, ND = 4*nrc densities (F_x, F_y, F_z and
// the box-centred fourth charge F.(r - c), per right-hand side), each with
// ncoef(p) complex coefficients for 0 <= m <= n <= p.  Internally the
// coefficients use solid harmonics normalised so that translations are
// plain convolutions, R_n^m = r^n P_n^m(cos t) e^{im phi}/(n+m)! and
// I_n^m = (n-m)! P_n^m(cos t) e^{im phi}/r^{n+1}, and they are scaled by the
// box side h: a box's multipole is M_n^m/h^n and its local expansion
// L_n^m h^{n+1}, so every translation operator depends only on offsets in
// box units.  The paper's coefficients (Sec. 2) are these times (or divided
// by) sqrt((n-m)!(n+m)!) and the matching power of h.
struct Exp {
  double2* M;
  double2* L;
  double* Q;  // per-bead charges [n][4 nrc] for S->M and S->L (written by run_p2m)
  double2* DL;  // evaluation sets of the leaves' local expansions (eval.hip)
  double2* DW;  // evaluation sets of the W-list multipoles that are evaluated
  double2* XP;  // S->L partial sums of split boxes [Built::nxshared][4 nrc][T]
  double* PV;   // EVAL_POLY: monomial coefficients of the leaves' local expansions
  float2* M32;  // FP32 M->L: multipoles in the paper's normalisation, [nbox][4 nrc][T]
};

// Per wave and pass of the S->M / S->L kernels (p2e.hip): bit k of `start`
// marks a step that begins a column (order m, the next 5-bit field of
// mhi:mlo), steps k < nvalid produce a coefficient, the rest pad with zero.
struct P2EPass {
  uint32_t start;
  int32_t nvalid;
  uint32_t mlo, mhi;
};
// A schedule with K steps per wave and pass and P passes (P = 0: none): per
// wave (8) and pass a P2EPass, and per slot (P x 8K) the coefficient it
// holds (-1: padding) with its factor 1/((n-m)!(n+m)!).
struct P2ESched {
  P2EPass* desc;
  int* slot;
  double* scale;
  int K, P;
};

struct Tables {
  int p;
  double2* oct;    // [8][(p+1)^2] R_j^mu(d/h_parent), d = child - parent centre
  double2* itab;   // [343][(2p+1)^2] I_j^mu(t), t integer offset in box units
  // Rotation-based M->L, FP64 and FP32 copies.  rot: per degree n, the
  // +90 degree rotation about y as (n+1) rows of n+1 slots holding the
  // nonzero real-split entries (A+ on real parts, then A- on imaginary
  // parts; the two are checkerboard-sparse).  zt: per order l the
  // z-translation matrix H_l ((p-l+1)^2, rows = output degree).  geo: per
  // integer offset slot, e^{-i(pi/2-phi)}, e^{i theta}, 1/|t| (8 doubles).
  double* rot64;
  float* rot32;
  double* zt64;
  float* zt32;
  double* geo;
  double* sfac;    // [ncoef(p)] sqrt((n-m)!(n+m)!)
  double* rscale;  // [ncoef(p)] 1/((n-m)!(n+m)!)
  // S->M / S->L schedules (K = 8 and K = 16 steps per wave and pass) and
  // the diagonal constants (-1)^m (2m-1)!!.
  P2ESched p2e[2];
  double* p2e_dk;
  int rot_len;     // sum_n (n+1)^2
  int zt_len;      // sum_l (p-l+1)^2
  int64_t bytes;
};

int make_tables(int p, Tables* tb, hipStream_t s, Error* err);
int make_p2e_tables(int p, Tables* tb, Error* err);  // p2e.hip; called by make_tables

// Host helpers (fmm.hip): paper-normalised Y_n^m for 0 <= m <= n <= p at
// (cos theta, phi); the rotation by +90 degrees about y on degree-n sets,
// D[(m'+n)(2n+1) + (m+n)].
void host_ynm(int p, double ct, double phi, std::vector<double2>& y, int nlo = 0);
void host_rot90(int n, std::vector<double>& D);
void free_tables(Tables* tb);

struct Launch {
  const Built* B;
  const Tables* tb;
  int p;
  double a, eta;
  hipStream_t s;
  int wd;  // W-list boxes of at most wd beads are summed directly (wd < 0: none)
};

// Forces (caller order, [nrhs][n][3]) -> sorted SoA [nrc][3][n] for rhs r0..r0+nrc-1.
hipError_t permute_forces(const Launch& l, const double* F, int nrhs_total, int r0, int nrc, double* sF);
// Near- plus far-field velocities (sorted SoA) -> caller order output.
hipError_t unpermute_velocities(const Launch& l, const double* u, const double* uf, int r0, int nrc, double* out);

hipError_t run_p2m(const Launch& l, int nrc, const double* sF, Exp e);
hipError_t run_m2m(const Launch& l, int nrc, Exp e);
hipError_t run_m2l(const Launch& l, int nrc, Exp e);       // dense O(p^4)
// rotation, O(p^3); part 0: target boxes of the deepest level, 1: the
// others, -1: all
hipError_t run_m2l_rot(const Launch& l, int nrc, Exp e, int fp32, int part = -1);
// Fills B->m2l_map / m2l_part, which run_m2l_rot needs (m2l_rot.hip).
int make_m2l_map(Built* B, hipStream_t s, Error* err);
// Fills B->xwork / xchunks / nxwork, which run_p2l needs (p2e.hip).
int make_p2l_work(Built* B, hipStream_t s, Error* err);
hipError_t run_p2l(const Launch& l, int nrc, const double* sF, Exp e);
hipError_t run_l2l(const Launch& l, int nrc, Exp e);

// Near field.  `tiles` lists (leaf, first bead, count) work items.
struct Tiles {
  int n;
  int4* t;
  double* box;  // [n][6] bounding box of each tile's beads (lo xyz, hi xyz)
};
int make_tiles(const Built* B, int tile, Tiles* out, hipStream_t s, Error* err);
// The near-field kernels take 1, 2, 4 or 8 right-hand sides per launch on
// the vector units (NEAR_VEC_RHS), or 16 + x with x in {0, 1, 2, 4, 8} (x > 0
// in the FP64 form only): the P2P then runs 16 of them on the matrix cores
// (NEAR_MC_RHS) and x on the vector units of the same launch, and the
// overlap and direct W sums as launches of 8 and the rest; sF and u are
// [nrc][3][n].
constexpr int NEAR_VEC_RHS = 8;
constexpr int NEAR_MC_RHS = 16;
constexpr int NEAR_MAX_RHS = NEAR_MC_RHS + NEAR_VEC_RHS;
hipError_t run_p2p(const Launch& l, const Tiles& tiles, int nrc, const double* sF, double* u, int mixed);
hipError_t run_overlap(const Launch& l, const Tiles& tiles, int nrc, const double* sF, double* u, int mixed);
// W-list boxes of at most Launch::wd beads are summed directly (far
// formula) by run_wdirect; the target evaluation uses the multipoles of the
// others only.  Per target and right-hand side the multipole route costs
// about 12 sets x (p+3)(p+4)/2 coefficients, the direct route a few tens of
// operations per source bead, so the library's default threshold is
// wdirect_default(p) = 2 (p+1)(p+2)/2 beads.
__host__ __device__ constexpr int wdirect_default(int p) { return (p + 1) * (p + 2); }
hipError_t run_wdirect(const Launch& l, const Tiles& tiles, int nrc, const double* sF, double* u, int mixed);
// Exact FP64 RPY sums (Sec. 1) at k sampled targets tgt (tree order) over all
// beads of each target's system: out [k][nrc][3].  The autotuner's reference.
hipError_t run_direct_sample(const Launch& l, const int* tgt, int k, int nrc, const double* sF, double* out);

// Target evaluation (eval.hip).  tiles: up to 64 beads of one leaf each
// (.w = leaf ordinal); widx[box] = row of the box's evaluation sets among
// the nwbig W-list multipoles that are evaluated (wbig lists those boxes),
// -1 for the others.
// Evaluation of the leaves' local expansions at the targets (Sec. 2 names
// two approaches): EVAL_SETS differentiates each Laplace expansion in
// coefficient space (12 harmonic sets per leaf and right-hand side) and
// combines the sums at each target; EVAL_POLY pre-assembles each velocity
// component into one polynomial per leaf and evaluates it (orders <= 21).
enum { EVAL_SETS = 1, EVAL_POLY = 2 };
constexpr int EVAL_POLY_MAX_ORDER = 21;
struct EvalPlan {
  Tiles tiles{};
  int* widx = nullptr;
  int* wbig = nullptr;
  int nwbig = 0;
  int mode = EVAL_SETS;
  double* kct = nullptr;  // EVAL_POLY: monomial table of the regular harmonics
};
int make_eval_plan(const Built* B, int p, int wd, int mode, EvalPlan* out, hipStream_t s, Error* err);
void free_eval_plan(EvalPlan* ep);
// Bytes of the evaluation-set arrays for nrc right-hand sides: returns the
// leaves' (Exp::DL), stores the W multipoles' (Exp::DW) in *dw_bytes.
int64_t eval_sets_bytes(const Built* B, const EvalPlan& ep, int p, int nrc, int64_t* dw_bytes, int64_t* pv_bytes);
// Writes the far-field velocities of every bead (assigns; sorted SoA).
hipError_t run_eval(const Launch& l, const EvalPlan& ep, int nrc, Exp e, double* u);

// Krylov building blocks (krylov.hip).  Vector sets are [nrhs][L]; the j-th
// of a family of sets starts at V + j * vstride.  krylov_mdot writes
// out[r * kcap + j] = V_j[r] . w[r] for j < k (deterministic order; part
// holds krylov_part_doubles(L, kcap, nrhs) doubles).  krylov_comb writes
// out[r] = s[r] * (a w[r] + sgn sum_{j<k} coef[r * kcap + j] V_j[r]) (s may
// be null = 1, w may be null, out may alias w).
int64_t krylov_part_doubles(int64_t L, int kcap, int nrhs);
hipError_t krylov_mdot(const double* V, int64_t vstride, int k, const double* w, int64_t L, int nrhs, int kcap,
                       double* part, double* out, hipStream_t st);
hipError_t krylov_comb(const double* V, int64_t vstride, int k, int kcap, const double* coef, double sgn,
                       const double* w, double a, const double* s, int64_t L, int nrhs, double* out, hipStream_t st);
// Eigen-decomposition of a symmetric tridiagonal matrix (host, implicit QL):
// diagonal d[0..m), off-diagonal e[0..m-1); Q column q = eigenvector q.
void tridiag_eig(int m, const std::vector<double>& d, const std::vector<double>& e, std::vector<double>& lam,
                 std::vector<double>& Q);

}  // namespace rpy
