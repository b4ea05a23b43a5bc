// Multipole-to-local translation (M->L over V lists) by rotation: every
// V-list source multipole is rotated so that the translation vector lies on
// the z axis, translated along z (an O(p^3) operator that keeps the order m),
// and rotated back.  The paper's FMM diagonalises this step with exponential
// expansions (arXiv:1711.02976, Sec. 1 and 3.2); this kernel computes the
// same truncated operator as the dense M->L instead.
//
// Coefficients are handled in the paper's normalisation (Sec. 2: Y_n^m =
// sqrt((n-|m|)!/(n+|m|)!) P_n^|m| e^{i m phi}), where a rotation is a real
// orthogonal matrix per degree.  For the offset t = (rho, theta, phi) the
// whole M->L is
//   Phi(phi - pi/2) R^-1 Phi(theta) R Z(rho) R^-1 Phi(-theta) R Phi(pi/2 - phi)
// with Phi(a) = diag(e^{-i m a}), R the fixed rotation by +90 degrees about y
// (inverse S R S, S = diag((-1)^m)) and Z(rho) the translation along +z,
//   L'_k^l = rho^-(k+1) sum_n H_l[k][n] rho^-n M'_n^l,
//   H_l[k][n] = (-1)^{n+l} (n+k)! / (s_k^l s_n^l),  s_n^m = sqrt((n-m)!(n+m)!).
//
// GPU organisation.  One block of RW waves per target box (the block-to-box
// map balances the V-list work over the XCDs, see make_m2l_map); its V-list
// (source, density) pairs are the columns, taken NC (64; 60 or 32 when LDS
// is short) at a time into an LDS array X[coefficient][column].  Each batch
// runs four phases separated by barriers:
//   0. all threads gather the columns' multipoles into X;
//   1. per degree n: Phi(pi/2-phi), R, Phi(-theta), S R S;
//   2. per order l: the z translation;
//   3. per degree n: R, Phi(theta), S R S, Phi(phi - pi/2);
// then every thread sums the columns of the outputs it owns into FP64
// accumulators kept in registers across batches.  A wave processes whole
// degrees (or orders), one column per lane, so the rotation and translation
// matrices are the same for every lane: they are read as scalar operands,
// and each lane's coefficients of one degree stay in registers.  Degrees and
// orders are assigned to waves by a host-side longest-first schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "fmm.h"

namespace rpy {

namespace {

constexpr int RW = 8;          // waves per block
constexpr int RT = 64 * RW;    // threads per block
constexpr int MAXK = MAX_ORDER + 1;

template <class R> struct Cx;
template <> struct Cx<double> { using T = double2; };
template <> struct Cx<float> { using T = float2; };

// Degrees (phases 1 and 3) and orders (phase 2) handled by each wave.
struct RotSched {
  unsigned char deg[RW][MAXK];
  unsigned char ord[RW][MAXK];
  unsigned char ndeg[RW];
  unsigned char nord[RW];
};

// Per-column data of a batch, in LDS (structure of arrays, one slot per lane),
// in the kernel's precision.
template <class R>
struct ColData {
  int* src;  // source box, -1 for an empty column
  R* e1x;    // e^{-i(pi/2 - phi)}
  R* e1y;
  R* e2x;    // e^{i theta}
  R* e2y;
  R* rinv;   // 1/rho (box units)
  R* wx;     // source centre - target centre (re-centres the fourth density)
  R* wy;
  R* wz;
};

__host__ __device__ constexpr int rot_block(int n) { return n * (n + 1) * (2 * n + 1) / 6; }  // sum_{j<n} (j+1)^2

// One row of the real-split rotation of degree N whose A+ part uses the
// inputs of parity Q: yr = sum A+ Re x, yi = sum A- Im x over the nonzero
// entries, stored in that order in the row a.
template <int N, int Q, class R>
__device__ inline void rot_row(const R* __restrict__ a, const R* xr, const R* xi, R& yr, R& yi) {
  constexpr int NP = N >= Q ? (N - Q) / 2 + 1 : 0;
  constexpr int MS = Q == 1 ? 2 : 1;
  constexpr int NM = N >= MS ? (N - MS) / 2 + 1 : 0;
  R r = 0, i = 0;
#pragma unroll
  for (int j = 0; j < NP; ++j) r = fma(a[j], xr[Q + 2 * j], r);
#pragma unroll
  for (int j = 0; j < NM; ++j) i = fma(a[NP + j], xi[MS + 2 * j], i);
  yr = r;
  yi = i;
}

// Stores (SR yr + i SI yi) times e (if PH) to col[mp] and advances e by (bx, by).
// The phase e^{i m a} is advanced by recurrence in the kernel's precision: in
// FP32 its error grows like m ulp, and it multiplies coefficients of degree
// n >= m, which the V-list separation makes smaller by a factor of at least
// 0.43^n than the degree-0 term.
template <bool PH, int SR, int SI, class R>
__device__ inline void put_row(typename Cx<R>::T* col, int mp, int ld, R yr, R yi, R& fr, R& fi, R bx, R by) {
  typename Cx<R>::T o;
  if (SR < 0) yr = -yr;
  if (SI < 0) yi = -yi;
  if (PH) {
    o.x = yr * fr - yi * fi;
    o.y = yr * fi + yi * fr;
    const R tr = fr * bx - fi * by;
    fi = fr * by + fi * bx;
    fr = tr;
  } else {
    o.x = yr;
    o.y = yi;
  }
  col[mp * ld] = o;
}

// col[mp] = e^{mp} (SR Re(R x)_mp + i SI Im(R x)_mp) for mp = 0..N, with
// e = (bx, by) when PH (else 1); SR = SI = 1 gives R, SR = (-1)^N and
// SI = -(-1)^N give the inverse rotation S R S on the same table.
template <int N, bool PH, int SR, int SI, class R>
__device__ inline void rot_apply(const R* __restrict__ A, const R* xr, const R* xi, R bx, R by,
                                 typename Cx<R>::T* col, int ld) {
  constexpr int K = N + 1;
  R fr = 1, fi = 0;
#pragma unroll 1
  for (int mp = 0; mp < K - 1; mp += 2) {
    R yr, yi;
    rot_row<N, (N & 1), R>(A + mp * K, xr, xi, yr, yi);
    put_row<PH, SR, SI, R>(col, mp, ld, yr, yi, fr, fi, bx, by);
    rot_row<N, ((N + 1) & 1), R>(A + (mp + 1) * K, xr, xi, yr, yi);
    put_row<PH, SR, SI, R>(col, mp + 1, ld, yr, yi, fr, fi, bx, by);
  }
  if (K & 1) {
    R yr, yi;
    rot_row<N, (N & 1), R>(A + N * K, xr, xi, yr, yi);
    put_row<PH, SR, SI, R>(col, N, ld, yr, yi, fr, fi, bx, by);
  }
}

template <int N, class R>
__device__ inline void load_col(const typename Cx<R>::T* col, int ld, R* xr, R* xi) {
#pragma unroll
  for (int m = 0; m <= N; ++m) {
    const auto v = col[m * ld];
    xr[m] = v.x;
    xi[m] = v.y;
  }
}

// Phase 1 for degree N of column c (the column's coefficients are already in
// X, scaled to the paper's normalisation): Phi(pi/2 - phi), R, Phi(-theta),
// S R S.
template <int N, class R>
__device__ void first_half(int c, int ld, const ColData<R>& cd, const R* __restrict__ A, typename Cx<R>::T* X) {
  using C = typename Cx<R>::T;
  constexpr int K = N + 1, t0 = N * (N + 1) / 2;
  constexpr int SG = (N & 1) ? -1 : 1;
  C* col = X + t0 * ld + c;
  R xr[K], xi[K];
  {
    const R ax = (R)cd.e1x[c], ay = (R)cd.e1y[c];
    R er = 1, ei = 0;
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const C v = col[m * ld];
      xr[m] = v.x * er - v.y * ei;
      xi[m] = v.x * ei + v.y * er;
      const R tr = er * ax - ei * ay;
      ei = er * ay + ei * ax;
      er = tr;
    }
  }
  rot_apply<N, true, 1, 1, R>(A, xr, xi, (R)cd.e2x[c], (R)cd.e2y[c], col, ld);
  load_col<N, R>(col, ld, xr, xi);
  rot_apply<N, false, SG, -SG, R>(A, xr, xi, 0.0, 0.0, col, ld);
}

// Phase 2: z translation of order l (KK = p - l + 1 degrees) of column c.
template <int KK, class R>
__device__ void ztrans(int l, int c, int ld, const ColData<R>& cd, const R* __restrict__ H, typename Cx<R>::T* X) {
  using C = typename Cx<R>::T;
  const R ri = (R)cd.rinv[c];
  R s = 1;
  for (int j = 0; j < l; ++j) s *= ri;
  R vr[KK], vi[KK];
#pragma unroll
  for (int j = 0; j < KK; ++j) {
    const int n = l + j;
    C v = X[(n * (n + 1) / 2 + l) * ld + c];
    vr[j] = v.x * s;
    vi[j] = v.y * s;
    s *= ri;
  }
  R so = 1;
  for (int j = 0; j <= l; ++j) so *= ri;
#pragma unroll 2
  for (int kk = 0; kk < KK; ++kk) {
    const R* h = H + kk * KK;
    R ar = 0, ai = 0;
#pragma unroll
    for (int j = 0; j < KK; ++j) {
      ar = fma(h[j], vr[j], ar);
      ai = fma(h[j], vi[j], ai);
    }
    const int k = l + kk;
    C o;
    o.x = ar * so;
    o.y = ai * so;
    X[(k * (k + 1) / 2 + l) * ld + c] = o;
    so *= ri;
  }
}

// Phase 3 for degree N of column c: R, Phi(theta), S R S, Phi(phi - pi/2).
template <int N, class R>
__device__ void second_half(int c, int ld, const ColData<R>& cd, const R* __restrict__ A, typename Cx<R>::T* X) {
  using C = typename Cx<R>::T;
  constexpr int K = N + 1, t0 = N * (N + 1) / 2;
  constexpr int SG = (N & 1) ? -1 : 1;
  C* col = X + t0 * ld + c;
  R xr[K], xi[K];
  load_col<N, R>(col, ld, xr, xi);
  rot_apply<N, true, 1, 1, R>(A, xr, xi, (R)cd.e2x[c], -(R)cd.e2y[c], col, ld);
  load_col<N, R>(col, ld, xr, xi);
  rot_apply<N, true, SG, -SG, R>(A, xr, xi, (R)cd.e1x[c], -(R)cd.e1y[c], col, ld);
}

// Degree (order) cases compiled into a kernel: 0..16, plus 17..21 when the
// kernel is built for PM = 21, plus 22..27 for PM = 27.
#define RPY_DEG_CASES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
#define RPY_DEG_CASES_HI(X) X(17) X(18) X(19) X(20) X(21)
#define RPY_DEG_CASES_HI2(X) X(22) X(23) X(24) X(25) X(26) X(27)

}  // namespace

// PM: highest degree compiled in (16, 21 or 27).  MINW: waves per SIMD the
// register allocation must allow (4 lets two blocks share a CU when their
// LDS fits).  A block translates ND of the box's nd_all densities, starting
// at density ND * blockIdx.y.
template <int ND, class R, int PM, int MINW>
__global__ void __launch_bounds__(RT, MINW) k_m2l_rot(int p, int nc, int nd_all, Tree t, List V, RotSched sched,
                                                const R* __restrict__ rot, const R* __restrict__ zt, int rot_len,
                                                const double* __restrict__ geo, const double* __restrict__ sf,
                                                const double2* __restrict__ M, const float2* __restrict__ M32,
                                                double2* __restrict__ L, const int* __restrict__ bmap) {
  using C = typename Cx<R>::T;
  constexpr int NACC = (ND * ncoef(PM) + RT - 1) / RT;
  extern __shared__ double2 smem[];
  const int T = ncoef(p);
  const int ld = nc + 1;  // padded row: column-wise and row-wise LDS accesses both avoid bank conflicts
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int b = bmap[blockIdx.x];
  if (b < 0) return;  // whole block, before any barrier
  const int d0 = ND * blockIdx.y;
  C* X = reinterpret_cast<C*>(smem);
  ColData<R> cd;
  {
    R* dq = reinterpret_cast<R*>(X + (size_t)T * ld);
    cd.e1x = dq; dq += nc;
    cd.e1y = dq; dq += nc;
    cd.e2x = dq; dq += nc;
    cd.e2y = dq; dq += nc;
    cd.rinv = dq; dq += nc;
    cd.wx = dq; dq += nc;
    cd.wy = dq; dq += nc;
    cd.wz = dq; dq += nc;
    cd.src = reinterpret_cast<int*>(dq);
  }
  double2 acc[NACC];
#pragma unroll
  for (int r = 0; r < NACC; ++r) acc[r] = make_double2(0.0, 0.0);

  const int e0 = V.off[b], e1 = V.off[b + 1];
  const int ncols = (e1 - e0) * ND;
  const int bx = t.ax[b], by = t.ay[b], bz = t.az[b];
  const double cbx = t.cx[b], cby = t.cy[b], cbz = t.cz[b];

  for (int c0 = 0; c0 < ncols; c0 += nc) {
    if (tid < nc) {
      const int g = c0 + tid;
      int S = -1;
      double q0 = 1.0, q1 = 0.0, q2 = 1.0, q3 = 0.0, q4 = 0.5, w0 = 0.0, w1 = 0.0, w2 = 0.0;
      if (g < ncols) {
        S = V.ent[e0 + g / ND];
        const int o = (t.ax[S] - bx + 3) * 49 + (t.ay[S] - by + 3) * 7 + (t.az[S] - bz + 3);
        const double* gq = geo + (size_t)o * 8;
        q0 = gq[0];
        q1 = gq[1];
        q2 = gq[2];
        q3 = gq[3];
        q4 = gq[4];
        w0 = t.cx[S] - cbx;
        w1 = t.cy[S] - cby;
        w2 = t.cz[S] - cbz;
      }
      cd.src[tid] = S;
      cd.e1x[tid] = q0;
      cd.e1y[tid] = q1;
      cd.e2x[tid] = q2;
      cd.e2y[tid] = q3;
      cd.rinv[tid] = q4;
      cd.wx[tid] = w0;
      cd.wy[tid] = w1;
      cd.wz[tid] = w2;
    }
    __syncthreads();
    // phase 0: gather the batch's multipoles (coefficient-contiguous reads),
    // convert to the paper's normalisation (times s_n^m) and store them
    // column-wise.  A thread takes the four densities of one right-hand side
    // of one source at one coefficient, so the fourth density is re-centred
    // on this machine from registers: M4 + (c_S - c_B) . (M1, M2, M3).
    {
      const int ng = nc / 4;  // (source, rhs) groups in the batch
      for (int it = tid; it < ng * T; it += RT) {
        const int g = it / T, f = it - (it / T) * T;
        const int c = 4 * g, S = cd.src[c];
        C o[4];
        if (S >= 0 && sizeof(R) == 4) {
          // FP32: multipoles already scaled and rounded (k_m2l_prep)
          const float2* src = M32 + ((int64_t)S * nd_all + d0 + (c % ND)) * T + f;
          float2 v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] = src[k * T];
          const float w0 = (float)cd.wx[c], w1 = (float)cd.wy[c], w2 = (float)cd.wz[c];
          v[3].x += w0 * v[0].x + w1 * v[1].x + w2 * v[2].x;
          v[3].y += w0 * v[0].y + w1 * v[1].y + w2 * v[2].y;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            o[k].x = (R)v[k].x;
            o[k].y = (R)v[k].y;
          }
        } else if (S >= 0) {
          const double2* src = M + ((int64_t)S * nd_all + d0 + (c % ND)) * T + f;
          double2 v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] = src[k * T];
          const double w0 = cd.wx[c], w1 = cd.wy[c], w2 = cd.wz[c];
          v[3].x += w0 * v[0].x + w1 * v[1].x + w2 * v[2].x;
          v[3].y += w0 * v[0].y + w1 * v[1].y + w2 * v[2].y;
          const double s = sf[f];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            o[k].x = (R)(v[k].x * s);
            o[k].y = (R)(v[k].y * s);
          }
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) o[k].x = o[k].y = 0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) X[f * ld + c + k] = o[k];
      }
    }
    __syncthreads();
    if (lane < nc) {
      const int nd = sched.ndeg[wv];
      for (int i = 0; i < nd; ++i) {
        const int n = sched.deg[wv][i];
        const R* A = rot + rot_block(n);
        switch (n) {
#define RPY_P1(k) \
  case k: if (k <= PM) first_half<(k <= PM ? k : 0), R>(lane, ld, cd, A, X); break;
          RPY_DEG_CASES(RPY_P1)
          RPY_DEG_CASES_HI(RPY_P1)
          RPY_DEG_CASES_HI2(RPY_P1)
#undef RPY_P1
          default: break;
        }
      }
    }
    __syncthreads();
    if (lane < nc) {
      const int no = sched.nord[wv];
      for (int i = 0; i < no; ++i) {
        const int l = sched.ord[wv][i];
        const int kk = p - l + 1;
        // rows of orders below l: sum_{l' < l} (p - l' + 1)^2
        const int zo = (p + 1) * (p + 2) * (2 * p + 3) / 6 - kk * (kk + 1) * (2 * kk + 1) / 6;
        switch (kk) {
#define RPY_P2(k) \
  case k + 1: if (k <= PM) ztrans<(k <= PM ? k : 0) + 1, R>(l, lane, ld, cd, zt + zo, X); break;
          RPY_DEG_CASES(RPY_P2)
          RPY_DEG_CASES_HI(RPY_P2)
          RPY_DEG_CASES_HI2(RPY_P2)
#undef RPY_P2
          default: break;
        }
      }
    }
    __syncthreads();
    if (lane < nc) {
      const int nd = sched.ndeg[wv];
      for (int i = 0; i < nd; ++i) {
        const int n = sched.deg[wv][i];
        const R* A = rot + rot_block(n);
        switch (n) {
#define RPY_P3(k) \
  case k: if (k <= PM) second_half<(k <= PM ? k : 0), R>(lane, ld, cd, A, X); break;
          RPY_DEG_CASES(RPY_P3)
          RPY_DEG_CASES_HI(RPY_P3)
          RPY_DEG_CASES_HI2(RPY_P3)
#undef RPY_P3
          default: break;
        }
      }
    }
    __syncthreads();
    // sum the columns of each (coefficient, density) into the accumulators
#pragma unroll
    for (int r = 0; r < NACC; ++r) {
      const int i = tid + r * RT;
      if (i < ND * T) {
        const int d = i / T, f = i - d * T;  // lanes walk a column: one bank per lane
        const C* row = X + (size_t)f * ld + d;
        double sx = 0.0, sy = 0.0;
        for (int j = 0; j < nc; j += ND) {
          const C v = row[j];
          sx += (double)v.x;
          sy += (double)v.y;
        }
        acc[r].x += sx;
        acc[r].y += sy;
      }
    }
    __syncthreads();
  }
  // paper normalisation -> stored normalisation (times s_k^l)
  double2* Lb = L + ((int64_t)b * nd_all + d0) * T;
#pragma unroll
  for (int r = 0; r < NACC; ++r) {
    const int i = tid + r * RT;
    if (i < ND * T) {
      const int d = i / T, f = i - d * T;
      const double s = sf[f];
      Lb[(size_t)d * T + f] = make_double2(acc[r].x * s, acc[r].y * s);
    }
  }
}

// Longest-first assignment of degrees (cost (n+1)^2) and orders (cost
// (p-l+1)^2) to the block's waves.
static RotSched make_sched(int p) {
  RotSched s{};
  for (int pass = 0; pass < 2; ++pass) {
    long load[RW] = {0};
    for (int j = p; j >= 0; --j) {
      // items in decreasing cost: degree j, or order p - j
      const int item = pass == 0 ? j : p - j;
      int w = 0;
      for (int k = 1; k < RW; ++k)
        if (load[k] < load[w]) w = k;
      load[w] += (long)(j + 1) * (j + 1);
      if (pass == 0) s.deg[w][s.ndeg[w]++] = (unsigned char)item;
      else s.ord[w][s.nord[w]++] = (unsigned char)item;
    }
  }
  return s;
}

static size_t rot_smem_bytes(int p, int nc, size_t real) {
  return (size_t)ncoef(p) * (nc + 1) * 2 * real + (size_t)nc * (8 * real + sizeof(int));
}

// ND densities per block, nsplit blocks per target box (nsplit ND densities
// per box in M and L).
template <class R, int ND, int PM, int MINW>
static hipError_t launch_nd(const Launch& l, Exp e, int nc, size_t shm, const RotSched& sc, const R* rot,
                            const R* zt, int part, int nsplit = 1) {
  const Built* B = l.B;
  auto kern = k_m2l_rot<ND, R, PM, MINW>;
  hipError_t he = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (he != hipSuccess) return he;
  if (!B->m2l_map || B->m2l_part[2] < B->tree.nbox) return hipErrorInvalidValue;
  const int b0 = part == 1 ? B->m2l_part[1] : 0, b1 = part == 0 ? B->m2l_part[1] : B->m2l_part[2];
  if (b1 <= b0) return hipSuccess;
  // the map runs are whole multiples of 8 blocks, so every density group of
  // a box lands on the same XCD
  kern<<<dim3(b1 - b0, nsplit), RT, shm, l.s>>>(l.p, nc, ND * nsplit, B->tree, B->lists[LV], sc, rot, zt,
                                                 l.tb->rot_len, l.tb->geo, l.tb->sfac, e.M, e.M32, e.L,
                                                 B->m2l_map + b0);
  return hipGetLastError();
}

// The FP32 M->L reads the multipoles of its source boxes in the paper's
// normalisation, scaled and rounded once per pass here instead of per
// V-list entry: boxes [b0, b1), all nd densities.
__global__ void k_m2l_prep(int T, int nd, int64_t b0, int64_t b1, const double* __restrict__ sf,
                           const double2* __restrict__ M, float2* __restrict__ M32) {
  const int64_t i = b0 * nd * T + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= b1 * nd * T) return;
  const double s = sf[i % T];
  const double2 v = M[i];
  M32[i] = make_float2((float)(v.x * s), (float)(v.y * s));
}

template <class R>
static hipError_t launch_rot(const Launch& l, int nrc, Exp e, const R* rot, const R* zt, int part) {
  const int p = l.p;
  if (p < 0 || p > MAX_ORDER) return hipErrorInvalidValue;
  if (l.B->tree.nbox == 0) return hipSuccess;
  if (sizeof(R) == 4) {
    // sources of the deepest level's targets (part 0) are on that level, those
    // of the other targets (part 1) above it
    if (!e.M32) return hipErrorInvalidValue;
    const Built* B = l.B;
    const int64_t deep = B->level_start.empty() ? 0 : B->level_start[B->depth];
    const int64_t b0 = part == 1 ? 0 : (part == 0 ? deep : 0), b1 = part == 1 ? deep : B->tree.nbox;
    const int T = ncoef(p), nd = 4 * nrc;
    const int64_t cnt = (b1 - b0) * nd * T;
    if (cnt > 0)
      k_m2l_prep<<<(unsigned)((cnt + 255) / 256), 256, 0, l.s>>>(T, nd, b0, b1, l.tb->sfac, e.M, e.M32);
    const hipError_t he = hipGetLastError();
    if (he != hipSuccess) return he;
  }
  // 64 columns per batch (one per lane), halved while the LDS (160 KB per CU)
  // cannot hold them.  Up to degree 16 in FP32 two blocks share a CU (80 KB
  // each; registers are then capped for four waves per SIMD); each block
  // then takes the four densities of one right-hand side.
  const bool lo = p <= 16, two = lo && sizeof(R) == 4;
  int nc = 64;
  while (nc > 8 && rot_smem_bytes(p, nc, sizeof(R)) > 160 * 1024) nc /= 2;
  const size_t shm = rot_smem_bytes(p, nc, sizeof(R));
  if (shm > 160 * 1024) return hipErrorInvalidValue;
  const RotSched sc = make_sched(p);
  // orders above 21 (the 9-digit setting) run one right-hand side per pass
  if (p > MAX_ORDER_MULTI) return nrc == 1 ? launch_nd<R, 4, 27, 1>(l, e, nc, shm, sc, rot, zt, part) : hipErrorInvalidValue;
  if constexpr (sizeof(R) == 4)
    if (two && (nrc == 1 || nrc == 2 || nrc == 4)) return launch_nd<R, 4, 16, 4>(l, e, nc, shm, sc, rot, zt, part, nrc);
  switch (nrc) {
    case 1:
      return lo ? launch_nd<R, 4, 16, 1>(l, e, nc, shm, sc, rot, zt, part) : launch_nd<R, 4, 21, 1>(l, e, nc, shm, sc, rot, zt, part);
    case 2:
      return lo ? launch_nd<R, 8, 16, 1>(l, e, nc, shm, sc, rot, zt, part) : launch_nd<R, 8, 21, 1>(l, e, nc, shm, sc, rot, zt, part);
    case 4:
      return lo ? launch_nd<R, 16, 16, 1>(l, e, nc, shm, sc, rot, zt, part)
                : launch_nd<R, 16, 21, 1>(l, e, nc, shm, sc, rot, zt, part);
    default: return hipErrorInvalidValue;
  }
}

// Blocks are dealt to the 8 XCDs round-robin (block i to XCD i mod 8), and
// each XCD has its own L2.  Every XCD gets one contiguous run of target
// boxes, so that neighbouring targets share their V-list sources in one L2,
// and the runs are cut where the modelled work (V entries, plus the part
// batch and the store of L per box) splits evenly: with clustered beads the
// V lists are far from uniform along the box order, and equal box counts
// per XCD left some XCDs with twice the mean work.  Block 8k + x takes the
// k-th box of run x; blocks past the end of a shorter run take none.
// Map of the boxes [r0, r1) appended to map (8 K entries).
static void append_map(const std::vector<int>& off, int r0, int r1, std::vector<int>& map) {
  if (r1 <= r0) return;
  const int nb = r1 - r0;
  std::vector<double> pre(nb + 1, 0.0);
  for (int i = 0; i < nb; ++i) {
    const int v = off[r0 + i + 1] - off[r0 + i];
    pre[i + 1] = pre[i] + v + (v > 0 ? 1.0 : 0.0) + 0.25;
  }
  int cut[9];
  cut[0] = 0;
  cut[8] = nb;
  for (int x = 1; x < 8; ++x) {
    const double goal = pre[nb] * x / 8.0;
    cut[x] = (int)(std::lower_bound(pre.begin(), pre.end(), goal) - pre.begin());
    cut[x] = std::min(std::max(cut[x], cut[x - 1]), nb);
  }
  int K = 0;
  for (int x = 0; x < 8; ++x) K = std::max(K, cut[x + 1] - cut[x]);
  const size_t base = map.size();
  map.resize(base + (size_t)8 * K, -1);
  for (int x = 0; x < 8; ++x)
    for (int k = 0; k < cut[x + 1] - cut[x]; ++k) map[base + (size_t)8 * k + x] = r0 + cut[x] + k;
}

int make_m2l_map(Built* B, hipStream_t s, Error* err) {
  const int nbox = B->tree.nbox;
  if (B->m2l_map) {
    (void)hipFree(B->m2l_map);
    B->m2l_map = nullptr;
  }
  B->m2l_part[0] = B->m2l_part[1] = B->m2l_part[2] = 0;
  if (nbox == 0) return 0;
  std::vector<int> off(nbox + 1);
  RPY_HIP(hipMemcpyAsync(off.data(), B->lists[LV].off, sizeof(int) * (nbox + 1), hipMemcpyDeviceToHost, s));
  RPY_HIP(hipStreamSynchronize(s));
  // boxes are numbered by level: the deepest level is the last range
  const int deep = B->level_start.empty() ? 0 : B->level_start[B->depth];
  std::vector<int> map;
  append_map(off, deep, nbox, map);
  B->m2l_part[1] = (int)map.size();
  append_map(off, 0, deep, map);
  B->m2l_part[2] = (int)map.size();
  if (map.empty()) return 0;
  RPY_HIP(hipMalloc(&B->m2l_map, sizeof(int) * map.size()));
  RPY_HIP(hipMemcpy(B->m2l_map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice));
  B->bytes += (int64_t)sizeof(int) * map.size();
  return 0;
}

hipError_t run_m2l_rot(const Launch& l, int nrc, Exp e, int fp32, int part) {
  return fp32 ? launch_rot<float>(l, nrc, e, l.tb->rot32, l.tb->zt32, part)
              : launch_rot<double>(l, nrc, e, l.tb->rot64, l.tb->zt64, part);
}

}  // namespace rpy
