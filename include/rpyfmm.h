/*
 * rpyfmm.h -- C ABI of the MI355X (gfx950) RPY-FMM library.
 *
 * The library evaluates the Rotne-Prager-Yamakawa (RPY) mobility
 * matrix-vector product over N beads of one radius a in a fluid of viscosity
 * eta (Guan et al., arXiv:1711.02976, Sec. 1, the three RPY block equations;
 * kB*T = 1, so the self block is I/(6 pi eta a)):
 *
 *     u_i = sum_j M(r_i - r_j; a, eta) F_j ,   j = i included (self term),
 *
 * by splitting the far field into four Laplace potentials (Sec. 2, L1..L4,
 * L_C and eq. (2.8)) evaluated with an adaptive fast multipole method, plus
 * the exact near field and an overlap correction for pairs closer than 2a
 * that the far field treats with the r >= 2a formula.
 *
 * Conventions common to every entry point
 *   - Pointers marked "device" must be HIP device (or managed) memory on the
 *     current device.  Pointers marked "host" are ordinary host memory.
 *   - Arrays are dense, row-major, FP64.  positions [n][3] = (x, y, z) per
 *     bead; forces and velocities [nrhs][n][3], in the caller's bead order.
 *   - Every entry point returns an rpy_status; negative values are errors.
 *     No exception crosses the ABI.  rpy_last_error() gives a thread-local
 *     human-readable detail of the last failure on the calling thread.
 *   - A plan is used by one host thread at a time; distinct plans are
 *     independent.  Work is issued on the plan's stream (options.stream, or
 *     the null stream) and rpy_matvec returns before the GPU finishes.
 */
#ifndef RPYFMM_H
#define RPYFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RPY_OK = 0,
  RPY_EINVAL = -1,       /* invalid argument (sizes, radius, viscosity, eps, NULL) */
  RPY_ENONFINITE = -2,   /* a position is NaN or infinite */
  RPY_ENOMEM = -3,       /* device allocation failed */
  RPY_EDEVICE = -4,      /* a HIP call failed; sticky on the plan */
  RPY_EUNSUPPORTED = -5  /* option combination not built (polynomial
                            evaluation above order 21) */
} rpy_status;

typedef enum {
  RPY_PREC_FP64 = 0,   /* every kernel in FP64 */
  RPY_PREC_MIXED = 1   /* P2P, the direct W sums, the overlap correction's
                          pair terms and M2L in FP32 (pair differences,
                          expansion storage and every sum across kernels in
                          FP64) */
} rpy_precision;

typedef struct {
  uint32_t struct_size;  /* sizeof(rpy_options); lets the struct grow */
  int32_t precision;     /* rpy_precision */
  int32_t leaf_size;     /* refinement limit: max beads per leaf (Sec. 4.2
                            "threshold"); 0 = chosen by the library: trees
                            are built for limits 64 * 1.5^k and the one with
                            the lowest modelled matvec time is kept */
  int32_t order;         /* expansion order p, 0..27; 0 = chosen from eps.
                            Above 21 each pass carries one right-hand side */
  int32_t max_depth;     /* deepest tree level, 1..21; 0 = 14 */
  int32_t m2l_mode;      /* multipole-to-local operator: 0 = library choice
                            (rotation), 1 = dense O(p^4) translation,
                            2 = rotation to the z axis, O(p^3) */
  void* stream;          /* hipStream_t for all work; NULL = null stream */
  int32_t nrhs;          /* right-hand sides per rpy_matvec call that the
                            library's leaf-size choice is tuned for (passes of
                            4 make the near field cheaper per right-hand side,
                            so larger leaves pay); 0 = 1.  Any nrhs may still
                            be passed to rpy_matvec.  Callers built against a
                            struct_size that ends at `stream` get 0. */
  int32_t w_direct;      /* W-list evaluation (adaptive trees): a W box's
                            contribution is the far formula summed over its
                            beads, which its multipole approximates (Theorem
                            1).  W boxes with at most w_direct beads are
                            summed directly, the others through their
                            multipoles.  0 = library choice, (p+1)(p+2);
                            -1 = every W box through its multipole.  Callers
                            whose struct_size ends before it get 0. */
  int32_t eval_mode;     /* evaluation of the leaves' local expansions at the
                            targets, the two approaches of Sec. 2 (after
                            Theorem 2): 1 = differentiate each Laplace
                            expansion (derivative sets), then assemble eq.
                            (2.8) per target; 2 = pre-assemble each velocity
                            component into one polynomial per leaf, then
                            evaluate it (orders <= 21; RPY_EUNSUPPORTED
                            above); 0 = library choice (2 up to order 10,
                            else 1).  Both give the same result to rounding.
                            Callers whose struct_size ends before it get 0. */
  int32_t tune;          /* 0 = refinement limit from a cost model and order
                            from an accuracy table; 1 = measured: when
                            leaf_size and order are both 0, candidate plans
                            (the model's limit and its neighbours, orders
                            downward from the table's, both evaluation
                            approaches) are built and timed on random forces,
                            and the fastest whose measured relative L2 error
                            at 256 sampled targets, against an FP64 direct
                            sum there, is at most eps/2 is kept.  Choices are
                            cached per process by (bead-count bucket, uniform
                            or adaptive tree, eps, precision, nrhs, systems).
                            Planning then takes seconds to minutes. */
} rpy_options;

typedef struct rpy_plan_s rpy_plan_t;

typedef struct {
  int64_t n;             /* beads (all systems) */
  int32_t nsys;          /* independent systems in the plan */
  int32_t order;         /* expansion order p in use */
  int32_t leaf_size;     /* refinement limit in use */
  int32_t depth;         /* deepest level present */
  int32_t precision;     /* rpy_precision in use */
  int32_t m2l_mode;      /* multipole-to-local operator in use: 1 dense, 2 rotation */
  int64_t nbox;          /* boxes (all systems) */
  int64_t nleaf;
  int64_t list_len[5];   /* entries of the U, V, W, X, O lists */
  int64_t device_bytes;  /* device memory held by the plan */
  double plan_ms;        /* wall time of rpy_plan / rpy_plan_batched */
  int32_t w_direct;      /* W boxes of at most this many beads are summed
                            directly (-1: none) */
  int32_t p2l_items;     /* S->L work items (a box's X list may be split) */
  int32_t p2l_split_boxes; /* boxes whose S->L work is split over several
                            items (their shares are added in a fixed order) */
  int32_t sort_passes;   /* radix-sort passes of the bead sort */
  double bead_pass_ms;   /* GPU time of the bead passes of the plan's first
                            tree: bounding cubes, Morton keys, radix sort,
                            position gather */
  int32_t eval_mode;     /* evaluation approach in use (1 or 2, see options) */
  int32_t tuned;         /* 0 model choice, 1 measured by the autotuner,
                            2 taken from the autotuner's cache */
  double tune_err;       /* measured relative L2 error of the tuned choice */
} rpy_plan_stats_t;

/* Fills *opt with the defaults (FP64, automatic leaf size and order,
 * max_depth 14, null stream). */
void rpy_default_options(rpy_options* opt);

/* Build a plan for one system of n beads.
 *   positions  device [n][3] FP64; copied, may be freed after return.
 *   a, eta     bead radius and solvent viscosity, both > 0.
 *   eps        requested relative L2 accuracy of the far field, in
 *              [1e-12, 1e-1]; selects the expansion order when
 *              opt->order == 0 (Sec. 4.3 uses 3, 6 and 9 digits; below
 *              1e-8 the order is the highest built, 27, which reaches
 *              about 3e-9 on uniform beads).
 *   opt        nullable; NULL means rpy_default_options.
 * Builds, on the GPU: the bounding cube and 63-bit Morton keys, a stable
 * radix sort, the adaptive octree (refine while more than leaf_size beads,
 * Sec. 4.2) and the U, V, W, X and O interaction lists.  n == 0 is valid
 * (every matvec is then a no-op).  On failure *out is set to NULL. */
rpy_status rpy_plan(rpy_plan_t** out, int64_t n, const double* positions, double a, double eta,
                    double eps, const rpy_options* opt);

/* Build one plan for nsys independent systems whose beads are concatenated
 * in positions (device [sum counts][3]); counts is host [nsys].  Systems do
 * not interact; each gets its own bounding cube and tree, and one launch of
 * each kernel serves all of them.  Each system is the paper's problem
 * (Sec. 4.2: sources = targets, one radius per evaluation); the batch serves
 * callers with many such systems, such as independent Brownian trajectories
 * (Sec. 1).  Validation and errors as for rpy_plan; counts may contain
 * zeros, and n = sum counts must be below 2^31 - 1. */
rpy_status rpy_plan_batched(rpy_plan_t** out, int32_t nsys, const int64_t* counts,
                            const double* positions, double a, double eta, double eps,
                            const rpy_options* opt);

/* velocities = M forces for nrhs right-hand sides.
 *   forces      device [nrhs][n][3] FP64, caller bead order; read only.
 *   velocities  device [nrhs][n][3] FP64; overwritten (not accumulated).
 * Asynchronous on the plan's stream; the buffers must stay valid until the
 * stream reaches this call's end. */
rpy_status rpy_matvec(rpy_plan_t* plan, int32_t nrhs, const double* forces, double* velocities);

/* rpy_matvec for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, result and errors as rpy_matvec, and the same kernels,
 * but the matvec workspace (expansions, staged forces, partial velocities,
 * charges, evaluation sets) lives in a fixed device array of 128 MiB that
 * the library holds on each device from load until the process ends; the
 * call issues no hipMalloc, hipFree or other allocating routine.
 *   - The plan's device must be current (RPY_EINVAL otherwise).
 *   - Right-hand sides per pass are chosen as in rpy_matvec and halved
 *     until the workspace fits; if one right-hand side per pass does not
 *     fit (roughly above a few hundred thousand beads at p = 16) the call
 *     returns RPY_ENOMEM and writes nothing.
 *   - Every call on a device shares that device's array and leaves its
 *     contents behind: calls that overlap in time on one device (plans on
 *     different streams, or different host threads) race and give wrong
 *     results; order them on one stream or synchronise between them.
 *   - Per-phase timing (rpy_plan_set_timing) does not record these calls. */
rpy_status rpy_matvec_noalloc(rpy_plan_t* plan, int32_t nrhs, const double* forces, double* velocities);

/* Brownian displacement vectors (Sec. 1, the Ermak-McCammon step): the
 * random displacements have covariance 2 D dt, so each is sqrt(2 dt) D^{1/2} z
 * for a standard normal z.  This computes y = D^{1/2} z, D the plan's
 * mobility (kB T = 1), by the Lanczos approximation from the Krylov space
 * {D^k z} (Sec. 1: D^{1/2} z approximated from the vectors D^k z), using only
 * rpy_matvec:
 *   beta_0 = |z|, v_0 = z / beta_0; per step k: w = D v_k, orthogonalised
 *   against v_0..v_k twice (classical Gram-Schmidt), alpha_k the v_k
 *   component, beta_{k+1} = |w|, v_{k+1} = w / beta_{k+1};
 *   y_k = beta_0 V_k T_k^{1/2} e_1, T_k the tridiagonal (alpha, beta) matrix,
 *   its square root from its eigen-decomposition (negative Ritz values,
 *   possible only through far-field error, are taken as 0).
 * No preconditioner is applied.  A right-hand side stops when
 * |y_k - y_{k-1}| <= tol |y_k| (the basis is orthonormal, so this is read off
 * the coefficients) or when beta_{k+1} vanishes; all right-hand sides share
 * the matvecs, nrhs at a time.
 *   z         device [nrhs][n][3] FP64, caller bead order; read only.
 *   y         device [nrhs][n][3] FP64; overwritten.  y may not alias z.
 *   tol       relative change at which to stop, in (0, 1).
 *   max_iter  most matvecs per right-hand side, 1..100.
 *   info      nullable host struct, filled on return.
 * Synchronous: it waits on the plan's stream after every step (a few
 * doubles cross to the host per step).  The plan keeps a workspace of
 * (max_iter + 2) nrhs 3n doubles after the first call (RPY_ENOMEM if it
 * cannot).  Not converging within max_iter is not an error: info says so. */
typedef struct {
  int32_t iterations;  /* matvecs applied (steps of the recurrence) */
  int32_t converged;   /* 1 if every right-hand side met tol */
  double rel_change;   /* largest last relative change over the right-hand sides */
  double min_ritz;     /* smallest Ritz value at the last step over the right-hand sides */
} rpy_sqrt_info_t;

rpy_status rpy_sqrt_matvec(rpy_plan_t* plan, int32_t nrhs, const double* z, double* y, double tol,
                           int32_t max_iter, rpy_sqrt_info_t* info);

/* Sizes and settings of a plan (host struct *out, caller allocated): the
 * tree depth and refinement limit (Sec. 4.2 "threshold"), the expansion
 * order, the lengths of the adaptive FMM's U, V, W, X lists (Sec. 2, Fig. 1)
 * and of the O list, and device memory.  RPY_EINVAL for NULL. */
rpy_status rpy_plan_stats(const rpy_plan_t* plan, rpy_plan_stats_t* out);

/* Copy the tree out for inspection and tests: the adaptive octree of the
 * refinement limit (Sec. 4.2) and the interaction lists of Fig. 1's
 * operators (U: S->T, V: M->L, W: M->T, X: S->L).  All host arrays, caller
 * allocated and sized from rpy_plan_stats; any pointer may be NULL to skip
 * it.  Waits for the plan's stream; RPY_EDEVICE if a copy fails:
 *   perm     [n]          caller index of the k-th bead in tree order
 *   keys     [n]          63-bit Morton keys in tree order
 *   boxes    [nbox][8]    level, anchor x, y, z, begin, end, parent,
 *                         first child (-1 for a leaf); begin/end index the
 *                         tree order; per-system boxes are concatenated
 *   offsets  [5][nbox+1]  CSR offsets of the U, V, W, X, O lists
 *   entries  [sum list_len] the five lists' entries, concatenated in the
 *                         order U, V, W, X, O; each list sorted by box id
 * Box ids and list entries are global across systems. */
rpy_status rpy_plan_export(const rpy_plan_t* plan, int64_t* perm, uint64_t* keys, int64_t* boxes,
                           int64_t* offsets, int64_t* entries);

/* Phases of one matvec pass, in launch order. */
typedef enum {
  RPY_PH_PERMUTE = 0,  /* forces to tree order */
  RPY_PH_P2P,          /* near field over the U lists, self term included */
  RPY_PH_OVERLAP,      /* r < 2a correction over the O lists */
  RPY_PH_P2M,          /* S->M at leaves */
  RPY_PH_M2M,          /* M->M, one launch per level */
  RPY_PH_M2L,          /* M->L over the V lists */
  RPY_PH_P2L,          /* S->L over the X lists */
  RPY_PH_L2L,          /* L->L, one launch per level */
  RPY_PH_EVAL,         /* L->T, M->T (W lists) and eq. (2.8) */
  RPY_PH_UNPERMUTE,    /* velocities to caller order */
  RPY_NPHASE
} rpy_phase;

typedef struct {
  double ms[RPY_NPHASE];         /* accumulated GPU time per phase (HIP events) */
  int64_t launches[RPY_NPHASE];  /* kernel launches per phase */
  int64_t passes;                /* matvec passes (right-hand-side chunks) timed */
  double p2p_mc_ms;              /* part of ms[RPY_PH_P2P] spent in P2P launches on the matrix
                                    cores (near-field groups of 16 right-hand sides there; in
                                    the FP64 form plus up to 8 on the vector units of the same
                                    launch) */
  int64_t p2p_mc_launches;       /* those launches (also counted in launches[RPY_PH_P2P]) */
  int64_t p2p_mc_rhs;            /* right-hand sides those launches carried, summed */
} rpy_timings_t;

/* Per-phase timing with HIP events: 0 off, 1 on (phases keep their normal
 * concurrency: the near field runs on a second stream beside the far-field
 * chain, so concurrent phases share the GPU), 2 on with every phase run on
 * the plan's stream one after another (each phase's time is its own; the
 * matvec is slower).  Any call resets the accumulators.  Timing adds two
 * events per phase and pass and no synchronisation.  Other values:
 * RPY_EINVAL. */
rpy_status rpy_plan_set_timing(rpy_plan_t* plan, int32_t enable);

/* Waits for the plan's stream, folds all recorded events into *out. */
rpy_status rpy_plan_timings(rpy_plan_t* plan, rpy_timings_t* out);

/* Failure-path testing: the next matvec pass of the plan reports a HIP
 * error at `phase` (an rpy_phase) instead of issuing that phase, exactly as
 * a failed launch would: rpy_matvec returns RPY_EDEVICE, nothing after the
 * failed phase is issued, and the plan is in the sticky error state.
 * phase = RPY_INJECT_ALLOC instead makes the plan's next matvec-workspace
 * allocation fail part-way, as a failed hipMalloc would: rpy_matvec frees
 * what it had allocated and returns RPY_ENOMEM before issuing any work, the
 * velocities are not written, and the plan stays usable (the next call
 * allocates again).  A call that needs no new workspace leaves the injection
 * pending.  phase = -1 clears a pending injection.  Returns RPY_EINVAL for
 * other values.  No kernel is made to fail on the device. */
#define RPY_INJECT_ALLOC 100
rpy_status rpy_plan_inject_error(rpy_plan_t* plan, int32_t phase);

/* Release a plan and its device memory; NULL is a no-op.  Waits for the
 * plan's streams first.  The host images of the translation tables stay
 * cached per expansion order for the life of the process. */
void rpy_plan_free(rpy_plan_t* plan);

const char* rpy_status_string(rpy_status s);
const char* rpy_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RPYFMM_H */
