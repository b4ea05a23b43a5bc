// Near field of the RPY matvec: the exact RPY block (arXiv:1711.02976, Sec. 1,
// the three RPY block equations, kB*T = 1) summed over every bead of the
// U-list leaves of each target leaf (self term included), plus the overlap
// correction (M_overlap - M_far) F for pairs closer than 2a whose leaves are
// not adjacent (the far field treated them with the r >= 2a formula).
//
// One block of P2P_T threads per target tile (a leaf, or a P2P_T-bead slice
// of a large leaf); each lane owns one target and keeps 3 * nrc sums in
// registers; source beads of each U-list leaf are staged through LDS
// (positions and forces, SoA) and read back as wave-wide broadcasts.  With
// 16 right-hand sides (in the FP64 form plus up to 8 more on the vector units
// of the same launch) the P2P runs on the matrix cores instead (k_p2p_mfma, 16 targets
// per wave, the 3x3 pair blocks as product operands).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "fmm.h"

namespace rpy {

namespace {
constexpr double PI = 3.14159265358979323846;
constexpr int P2P_T = 128;
inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------- tiles ---
__global__ void k_tile_count(const int* leaves, int nleaf, Tree t, int tile, int* cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nleaf) return;
  int b = leaves[i];
  cnt[i] = (t.end[b] - t.begin[b] + tile - 1) / tile;
}

__global__ void k_tile_fill(const int* leaves, int nleaf, Tree t, int tile, const int* off, int4* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nleaf) return;
  int b = leaves[i];
  int o = off[i];
  for (int s = t.begin[b]; s < t.end[b]; s += tile) out[o++] = make_int4(b, s, min(tile, t.end[b] - s), i);
}

// Bounding box of each tile's beads: lo xyz, hi xyz.
__global__ void k_tile_box(const int4* tiles, int nt, const double* sx, const double* sy, const double* sz,
                           double* box) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const int4 tl = tiles[i];
  double lo[3] = {sx[tl.y], sy[tl.y], sz[tl.y]}, hi[3] = {lo[0], lo[1], lo[2]};
  for (int j = tl.y + 1; j < tl.y + tl.z; ++j) {
    const double v[3] = {sx[j], sy[j], sz[j]};
    for (int k = 0; k < 3; ++k) {
      lo[k] = fmin(lo[k], v[k]);
      hi[k] = fmax(hi[k], v[k]);
    }
  }
  for (int k = 0; k < 3; ++k) {
    box[6 * (int64_t)i + k] = lo[k];
    box[6 * (int64_t)i + 3 + k] = hi[k];
  }
}

int make_tiles(const Built* B, int tile, Tiles* out, hipStream_t s, Error* err) {
  out->n = 0;
  out->t = nullptr;
  out->box = nullptr;
  if (B->nleaf == 0) return 0;
  int *cnt = nullptr, *off = nullptr, *tmp = nullptr;
  RPY_HIP(hipMalloc(&cnt, sizeof(int) * B->nleaf));
  RPY_HIP(hipMalloc(&off, sizeof(int) * B->nleaf));
  RPY_HIP(hipMalloc(&tmp, sizeof(int) * scan_tmp_ints(B->nleaf)));
  k_tile_count<<<nblk(B->nleaf, 256), 256, 0, s>>>(B->leaf_ids, B->nleaf, B->tree, tile, cnt);
  RPY_HIP(scan_exclusive(cnt, off, B->nleaf, tmp, s));
  int last[2];
  RPY_HIP(hipMemcpyAsync(&last[0], off + B->nleaf - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  RPY_HIP(hipMemcpyAsync(&last[1], cnt + B->nleaf - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  RPY_HIP(hipStreamSynchronize(s));
  out->n = last[0] + last[1];
  RPY_HIP(hipMalloc(&out->t, sizeof(int4) * out->n));
  k_tile_fill<<<nblk(B->nleaf, 256), 256, 0, s>>>(B->leaf_ids, B->nleaf, B->tree, tile, off, out->t);
  RPY_HIP(hipGetLastError());
  RPY_HIP(hipMalloc(&out->box, sizeof(double) * 6 * std::max(out->n, 1)));
  if (out->n > 0) k_tile_box<<<nblk(out->n, 256), 256, 0, s>>>(out->t, out->n, B->sx, B->sy, B->sz, out->box);
  RPY_HIP(hipGetLastError());
  RPY_HIP(hipStreamSynchronize(s));
  (void)hipFree(cnt); (void)hipFree(off); (void)hipFree(tmp);
  return 0;
}

// ------------------------------------------------------------ pair math ---

// Pair coefficients of the P2P sum with the far prefactor c1 = 1/(8 pi eta)
// taken out of the sum (applied once per target):
//   far      A' = 1/r + (2a^2/3)/r^3,        B' = (1 - 2a^2/r^2)/r^3,
//   overlap  A' = (c0/c1)(1 - 9r/(32a)),     B' = (c0/c1)(3/(32a))/r,
// c0/c1 = 4/(3a).  The pair kernels work in units scaled by a power of two S
// chosen so that 2aS lies in [1, 2): positions are scaled by S (exactly),
// the constants are those of the radius aS, and the sums come out divided by
// S, which the prefactor c1 S restores.  Apart from overflow and underflow
// this is the same arithmetic rounded the same way, and it keeps every pair
// quantity of order one whatever the length unit.
template <class R>
struct PairK {
  R a3;       // 2a^2/3
  R a2;       // 2a^2
  R four_a2;  // (2a)^2
  R oc;       // c0/c1
  R ock9;     // (c0/c1) 9/(32a)
  R ob;       // (c0/c1) 3/(32a)
  R r2min;    // floor added to r^2 before the reciprocal square root (coincident beads)
  R i2a;      // 1/(2a)
};

// Power of two S with 2aS in [1, 2).
static double pair_scale(double a) { return std::ldexp(1.0, -std::ilogb(2.0 * a)); }

// Constants for the scaled radius as = a S.
template <class R>
static PairK<R> pair_const(double as) {
  const double oc = 4.0 / (3.0 * as);
  return PairK<R>{(R)(2.0 * as * as / 3.0), (R)(2.0 * as * as), (R)(4.0 * as * as), (R)oc,
                  (R)(oc * 9.0 / (32.0 * as)), (R)(oc * 3.0 / (32.0 * as)), (R)1e-30, (R)(0.5 / as)};
}

__device__ inline float rinv_of(float r2) { return __builtin_amdgcn_rsqf(r2); }
// single-precision estimate refined by one Newton step (relative error
// below 2^-44); r2 >= 1e-30 here (a normal FP32 number), so the estimate is
// finite
__device__ inline double rinv_of(double r2) {
  double y = (double)__builtin_amdgcn_rsqf((float)r2);
  return y * fma(-0.5 * r2, y * y, 1.5);
}

// --------------------------------------------------------------- P2P -----
// The overlap formula is evaluated only when some lane of the wave has a
// source closer than 2a (a wave-uniform branch), since such pairs are rare
// apart from each target's own bead.  For r = 0 (the bead itself, or a
// coincident bead) r^2 carries a floor of 1e-30 in the scaled units (added
// in the first FMA) before the reciprocal square root: the far values are
// then finite and discarded, and the overlap values give the r -> 0 limit
// A' = c0/c1, B' d = 0.  Since 2a >= 1 in these units, the floor changes
// r^2 by a relative amount below 1e-30 at every r >= 2a, where the far
// formula applies.
// Positions enter the pair arithmetic relative to the target leaf's centre
// (differences taken in FP64, scaled by S and rounded once); in the mixed
// form the pair arithmetic and per-source-leaf sums run in FP32.
// The FP32 launch of 4 right-hand sides (the rest of 20 after the
// matrix-core group) is held to 96 registers, five waves per SIMD instead of
// four (two registers spill; 192 instead of 196 ms on cube-15M).
template <int NRC, bool MIXED>
__global__ void __launch_bounds__(P2P_T, (NRC == 4 && MIXED) ? 5 : 1) k_p2p(const int4* tiles, Tree t, List U, const double* sx,
                                               const double* sy, const double* sz, const double* sF, int64_t n,
                                               PairK<typename std::conditional<MIXED, float, double>::type> k,
                                               double S, double c1, double* u) {
  using R = typename std::conditional<MIXED, float, double>::type;
  using V4 = typename std::conditional<MIXED, float4, double4>::type;
  __shared__ alignas(32) R xs[P2P_T];
  __shared__ alignas(32) R ys[P2P_T];
  __shared__ alignas(32) R zs[P2P_T];
  __shared__ alignas(32) R fs[NRC * 3][P2P_T];
  const int4 tl = tiles[xcd_run(blockIdx.x, gridDim.x)];
  const int b = tl.x;
  const bool valid = (int)threadIdx.x < tl.z;
  const bool wlive = (int)(threadIdx.x & ~63u) < tl.z;  // this wave holds a target of the tile
  const int i = tl.y + (valid ? threadIdx.x : 0);
  const double ox = t.cx[b], oy = t.cy[b], oz = t.cz[b];
  const R xi = (R)((sx[i] - ox) * S), yi = (R)((sy[i] - oy) * S), zi = (R)((sz[i] - oz) * S);
  double acc[NRC][3];
  for (int r = 0; r < NRC; ++r) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
  const int e0 = __builtin_amdgcn_readfirstlane(U.off[b]), e1 = __builtin_amdgcn_readfirstlane(U.off[b + 1]);
  for (int e = e0; e < e1; ++e) {
    const int C = __builtin_amdgcn_readfirstlane(U.ent[e]);
    const int j1 = __builtin_amdgcn_readfirstlane(t.end[C]);
    for (int jc = __builtin_amdgcn_readfirstlane(t.begin[C]); jc < j1; jc += P2P_T) {
      const int ns = min(P2P_T, j1 - jc);
      // the tile is padded to a multiple of 4 sources with inert ones: zero
      // force at 1e30, where 1/r, A' and B' all evaluate to exactly zero
      const int ns4 = (ns + 3) & ~3;
      __syncthreads();
      if ((int)threadIdx.x < ns) {
        int j = jc + threadIdx.x;
        xs[threadIdx.x] = (R)((sx[j] - ox) * S); ys[threadIdx.x] = (R)((sy[j] - oy) * S);
        zs[threadIdx.x] = (R)((sz[j] - oz) * S);
        for (int q = 0; q < NRC * 3; ++q) fs[q][threadIdx.x] = (R)sF[(int64_t)q * n + j];
      } else if ((int)threadIdx.x < ns4) {
        xs[threadIdx.x] = (R)1e30; ys[threadIdx.x] = (R)1e30; zs[threadIdx.x] = (R)1e30;
        for (int q = 0; q < NRC * 3; ++q) fs[q][threadIdx.x] = (R)0;
      }
      __syncthreads();
      R ar[NRC][3];
      for (int r = 0; r < NRC; ++r) ar[r][0] = ar[r][1] = ar[r][2] = (R)0;
      // four sources per trip, read as vectors; one wave-wide test for the
      // overlap branch per trip.  A wave with no target of the tile (the
      // second wave of a tile of 64 beads or fewer) stages and syncs only.
      for (int s0 = 0; s0 < (wlive ? ns4 : 0); s0 += 4) {
        const V4 X4 = *reinterpret_cast<const V4*>(xs + s0), Y4 = *reinterpret_cast<const V4*>(ys + s0),
                 Z4 = *reinterpret_cast<const V4*>(zs + s0);
        // padding sources: r^2 overflows to inf in FP32, 1/r = 0, A = B = 0
        const R dx[4] = {xi - X4.x, xi - X4.y, xi - X4.z, xi - X4.w};
        const R dy[4] = {yi - Y4.x, yi - Y4.y, yi - Y4.z, yi - Y4.w};
        const R dz[4] = {zi - Z4.x, zi - Z4.y, zi - Z4.z, zi - Z4.w};
        R r2[4], rinv[4], A[4], B[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // r^2 + r2min: the floor rides in the first FMA instead of a max
          r2[q] = fma(dx[q], dx[q], fma(dy[q], dy[q], fma(dz[q], dz[q], k.r2min)));
          rinv[q] = rinv_of(r2[q]);
          const R ri2 = rinv[q] * rinv[q], ri3 = ri2 * rinv[q];
          A[q] = fma(k.a3, ri3, rinv[q]);
          B[q] = ri3 * fma(-k.a2, ri2, (R)1);
        }
        const R r2lo = min(min(r2[0], r2[1]), min(r2[2], r2[3]));
        if (__builtin_expect(__any(r2lo < k.four_a2), 0)) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool ov = r2[q] < k.four_a2;
            // r from r^2 without the floor: exactly 0 for the bead itself
            const R Ao = fma(-k.ock9, (r2[q] - k.r2min) * rinv[q], k.oc), Bo = k.ob * rinv[q];
            A[q] = ov ? Ao : A[q];
            B[q] = ov ? Bo : B[q];
          }
        }
        // with several right-hand sides, B d is formed once per pair (3
        // multiplies) so that each right-hand side costs 9 operations:
        // t = d.F, u += A F + t (B d)
        R bdx[4], bdy[4], bdz[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bdx[q] = NRC >= 4 ? B[q] * dx[q] : dx[q];
          bdy[q] = NRC >= 4 ? B[q] * dy[q] : dy[q];
          bdz[q] = NRC >= 4 ? B[q] * dz[q] : dz[q];
        }
#pragma unroll
        for (int r = 0; r < NRC; ++r) {
          const V4 FX = *reinterpret_cast<const V4*>(&fs[3 * r][s0]), FY = *reinterpret_cast<const V4*>(&fs[3 * r + 1][s0]),
                   FZ = *reinterpret_cast<const V4*>(&fs[3 * r + 2][s0]);
          const R fx[4] = {FX.x, FX.y, FX.z, FX.w}, fy[4] = {FY.x, FY.y, FY.z, FY.w}, fz[4] = {FZ.x, FZ.y, FZ.z, FZ.w};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const R dF = fma(dx[q], fx[q], fma(dy[q], fy[q], dz[q] * fz[q]));
            const R t = NRC >= 4 ? dF : B[q] * dF;
            ar[r][0] = fma(A[q], fx[q], fma(t, bdx[q], ar[r][0]));
            ar[r][1] = fma(A[q], fy[q], fma(t, bdy[q], ar[r][1]));
            ar[r][2] = fma(A[q], fz[q], fma(t, bdz[q], ar[r][2]));
          }
        }
      }
      for (int r = 0; r < NRC; ++r)
        for (int c = 0; c < 3; ++c) acc[r][c] += (double)ar[r][c];
    }
  }
  if (valid)
    for (int r = 0; r < NRC; ++r)
      for (int c = 0; c < 3; ++c) u[((int64_t)r * 3 + c) * n + i] = c1 * acc[r][c];
}

// ------------------------------------------- P2P on the matrix cores ----
// With 16 right-hand sides the P2P of a target tile is a product
//   U[3 x targets][16] += M[3 x targets][3 x sources] F[3 x sources][16]
// whose 3x3 blocks M_ij = A_ij I + B_ij d d^T (the RPY block of Sec. 1, with
// the overlap branch for r < 2a) are formed on the fly.  A wave owns 16
// targets; per step of 4 sources each lane forms one pair (target lane % 16,
// source lane / 16) and the six distinct entries of its block, which are
// exactly the A operands of 16x16x4 matrix-core products in that lane:
// D_a += M_ab F_b for a, b in {x, y, z}, nine products per step, with F_b
// (source, right-hand side) as the B operand.  The FP32 form uses
// v_mfma_f32_16x16x4f32 and adds D into FP64 sums after each staged chunk of
// sources (as the vector kernel does); the FP64 form uses
// v_mfma_f64_16x16x4f64 and keeps the sums in D.
// In the FP64 form XR = 1, 2, 4 or 8 further right-hand sides ride in the
// same launch on the vector units: each lane applies its pair block to them
// (nine multiply-adds per right-hand side), so the pair geometry is formed
// once for 16 + XR right-hand sides.  Their per-lane partial sums are added
// over the four source lanes of a target after each staged chunk, and lane
// (t, k) keeps the FP64 sums of the right-hand sides k, k + 4.  (The mixed
// form runs its extra right-hand sides in the vector kernel: there the
// registers they take cost the matrix-core loop more than the shared
// geometry saves.)
namespace {
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef double v4d_t __attribute__((ext_vector_type(4)));
constexpr int MF_W = 8;         // waves per block: 16 targets each, P2P_T per tile
constexpr int MF_R = NEAR_MC_RHS;  // right-hand sides on the matrix cores (the product's N)
__device__ inline v4f_t mfma16(float a, float b, v4f_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline v4d_t mfma16(double a, double b, v4d_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
// Row (target within the wave's 16) of item v of a 16x16 result in lane l;
// the column (right-hand side) is l % 16 in both forms.
__device__ inline int mf_row(float, int l, int v) { return 4 * (l >> 4) + v; }
__device__ inline int mf_row(double, int l, int v) { return 4 * v + (l >> 4); }
}  // namespace

template <bool MIXED, int XR>
__global__ void __launch_bounds__(64 * MF_W) k_p2p_mfma(const int4* tiles, Tree t, List U, const double* sx,
                                                       const double* sy, const double* sz, const double* sF,
                                                       int64_t n,
                                                       PairK<typename std::conditional<MIXED, float, double>::type> k,
                                                       double S, double c1, double* u) {
  using R = typename std::conditional<MIXED, float, double>::type;
  using R4 = typename std::conditional<MIXED, float4, double4>::type;
  using VD = typename std::conditional<MIXED, v4f_t, v4d_t>::type;
  constexpr int XS = XR > 0 ? XR : 1, XH = (XR + 3) / 4 > 0 ? (XR + 3) / 4 : 1;
  __shared__ R4 ps[P2P_T];          // positions (x, y, z, -)
  __shared__ R fs[3][P2P_T][MF_R];  // [component][source][right-hand side]
  __shared__ alignas(16) R fx[3][P2P_T][XS];  // the XR vector-unit right-hand sides
  const int4 tl = tiles[xcd_run(blockIdx.x, gridDim.x)];
  const int b = tl.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int t0 = 16 * __builtin_amdgcn_readfirstlane(tid >> 6);  // the wave's first target in the tile
  const bool wlive = t0 < tl.z;
  const int ti = lane & 15, sk = lane >> 4;  // lane's target row and source within a step
  // rows past the tile take its last target (finite values, never stored)
  const int i = tl.y + max(0, min(t0 + ti, tl.z - 1));
  const double ox = t.cx[b], oy = t.cy[b], oz = t.cz[b];
  const R xi = (R)((sx[i] - ox) * S), yi = (R)((sy[i] - oy) * S), zi = (R)((sz[i] - oz) * S);
  VD D[3];
  double acc[3][4];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    D[c] = VD{0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[c][v] = 0.0;
  }
  R xa[XS][3];      // this lane's pair sums of the vector-unit right-hand sides (one chunk)
  double xacc[XH][3];  // FP64 sums of right-hand sides sk + 4 h for target ti
#pragma unroll
  for (int h = 0; h < XH; ++h) xacc[h][0] = xacc[h][1] = xacc[h][2] = 0.0;
  const int e0 = __builtin_amdgcn_readfirstlane(U.off[b]), e1 = __builtin_amdgcn_readfirstlane(U.off[b + 1]);
  for (int e = e0; e < e1; ++e) {
    const int C = __builtin_amdgcn_readfirstlane(U.ent[e]);
    const int j1 = __builtin_amdgcn_readfirstlane(t.end[C]);
    for (int jc = __builtin_amdgcn_readfirstlane(t.begin[C]); jc < j1; jc += P2P_T) {
      const int ns = min(P2P_T, j1 - jc);
      // padded to a multiple of 4 sources with inert ones (zero force at 1e30)
      const int ns4 = (ns + 3) & ~3;
      __syncthreads();
      if (tid < ns) {
        const int j = jc + tid;
        ps[tid] = R4{(R)((sx[j] - ox) * S), (R)((sy[j] - oy) * S), (R)((sz[j] - oz) * S), (R)0};
      } else if (tid < ns4) {
        ps[tid] = R4{(R)1e30, (R)1e30, (R)1e30, (R)0};
      }
      // forces: sF row q = 3 r + c, read along the sources (coalesced)
      for (int q = tid; q < 3 * (MF_R + XR) * P2P_T; q += 64 * MF_W) {
        const int row = q / P2P_T, sj = q - row * P2P_T;
        if (sj < ns4) {
          const R v = sj < ns ? (R)sF[(int64_t)row * n + jc + sj] : (R)0;
          if (row < 3 * MF_R) fs[row % 3][sj][row / 3] = v;
          else fx[(row - 3 * MF_R) % 3][sj][(row - 3 * MF_R) / 3] = v;
        }
      }
      __syncthreads();
      if (wlive) {
        R m[6], f[3];
#pragma unroll
        for (int x = 0; x < XS; ++x) xa[x][0] = xa[x][1] = xa[x][2] = (R)0;
        for (int s0 = 0; s0 < ns4; s0 += 4) {
          const int j = s0 + sk;
          const R4 p = ps[j];
          {  // the pair block, as in k_p2p: six distinct entries xx, yy, zz, xy, xz, yz
            const R dx = xi - p.x, dy = yi - p.y, dz = zi - p.z;
            const R r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, k.r2min)));
            const R rinv = rinv_of(r2);
            const R ri2 = rinv * rinv, ri3 = ri2 * rinv;
            R A = fma(k.a3, ri3, rinv);
            R B = ri3 * fma(-k.a2, ri2, (R)1);
            if (__builtin_expect(__any(r2 < k.four_a2), 0)) {
              const bool ov = r2 < k.four_a2;
              const R Ao = fma(-k.ock9, (r2 - k.r2min) * rinv, k.oc), Bo = k.ob * rinv;
              A = ov ? Ao : A;
              B = ov ? Bo : B;
            }
            const R bx = B * dx, by = B * dy, bz = B * dz;
            m[0] = fma(bx, dx, A);
            m[1] = fma(by, dy, A);
            m[2] = fma(bz, dz, A);
            m[3] = bx * dy;
            m[4] = bx * dz;
            m[5] = by * dz;
          }
          f[0] = fs[0][j][ti];
          f[1] = fs[1][j][ti];
          f[2] = fs[2][j][ti];
          D[0] = mfma16(m[0], f[0], D[0]);
          D[1] = mfma16(m[3], f[0], D[1]);
          D[2] = mfma16(m[4], f[0], D[2]);
          D[0] = mfma16(m[3], f[1], D[0]);
          D[1] = mfma16(m[1], f[1], D[1]);
          D[2] = mfma16(m[5], f[1], D[2]);
          D[0] = mfma16(m[4], f[2], D[0]);
          D[1] = mfma16(m[5], f[2], D[1]);
          D[2] = mfma16(m[2], f[2], D[2]);
#pragma unroll
          for (int x = 0; x < XR; ++x) {
            const R gx = fx[0][j][x], gy = fx[1][j][x], gz = fx[2][j][x];
            xa[x][0] = fma(m[0], gx, fma(m[3], gy, fma(m[4], gz, xa[x][0])));
            xa[x][1] = fma(m[3], gx, fma(m[1], gy, fma(m[5], gz, xa[x][1])));
            xa[x][2] = fma(m[4], gx, fma(m[5], gy, fma(m[2], gz, xa[x][2])));
          }
        }
        if (MIXED) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[c][v] += (double)D[c][v];
            D[c] = VD{0, 0, 0, 0};
          }
        }
        // the chunk's sums over the four source lanes of each target; lane
        // sk keeps right-hand sides sk, sk + 4
#pragma unroll
        for (int x = 0; x < XR; ++x)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            R v = xa[x][c];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (sk == (x & 3)) xacc[x >> 2][c] += (double)v;
          }
      }
    }
  }
  if (!wlive) return;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = mf_row(R(0), lane, v);
      if (t0 + row < tl.z) {
        const double x = MIXED ? acc[c][v] : (double)D[c][v];
        u[((int64_t)ti * 3 + c) * n + tl.y + t0 + row] = c1 * x;
      }
    }
  if (t0 + ti < tl.z)
#pragma unroll
    for (int h = 0; h < XH; ++h) {
      const int x = sk + 4 * h;
      if (x < XR)
#pragma unroll
        for (int c = 0; c < 3; ++c) u[((int64_t)(MF_R + x) * 3 + c) * n + tl.y + t0 + ti] = c1 * xacc[h][c];
    }
}

// ---------------------------------------------------- W list, direct ----
// W-list boxes with few beads: their multipole evaluation at this leaf's
// targets (Theorem 1, order p + 2) costs more than summing their beads, so
// they are summed directly with the far formula, which is what the far field
// stands for (pairs closer than 2a are then corrected by the O list as
// before).  Boxes with more than wmax beads keep the multipole route.
template <int NRC, bool MIXED>
__global__ void __launch_bounds__(P2P_T) k_wdirect(const int4* tiles, Tree t, List W, int wmax, const double* sx,
                                                   const double* sy, const double* sz, const double* sF, int64_t n,
                                                   PairK<typename std::conditional<MIXED, float, double>::type> k,
                                                   double S, double c1, double* u) {
  using R = typename std::conditional<MIXED, float, double>::type;
  __shared__ R xs[P2P_T], ys[P2P_T], zs[P2P_T];
  __shared__ R fs[NRC * 3][P2P_T];
  const int4 tl = tiles[blockIdx.x];
  const int b = tl.x;
  const int e0 = __builtin_amdgcn_readfirstlane(W.off[b]), e1 = __builtin_amdgcn_readfirstlane(W.off[b + 1]);
  if (e0 == e1) return;
  const bool valid = (int)threadIdx.x < tl.z;
  const bool wlive = (int)(threadIdx.x & ~63u) < tl.z;  // this wave holds a target of the tile
  const int i = tl.y + (valid ? threadIdx.x : 0);
  const double ox = t.cx[b], oy = t.cy[b], oz = t.cz[b];  // positions relative to the target leaf
  const R xi = (R)((sx[i] - ox) * S), yi = (R)((sy[i] - oy) * S), zi = (R)((sz[i] - oz) * S);
  double acc[NRC][3];
  for (int r = 0; r < NRC; ++r) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
  bool any = false;
  for (int e = e0; e < e1; ++e) {
    const int C = __builtin_amdgcn_readfirstlane(W.ent[e]);
    const int j0 = __builtin_amdgcn_readfirstlane(t.begin[C]), j1 = __builtin_amdgcn_readfirstlane(t.end[C]);
    if (j1 - j0 > wmax) continue;
    any = true;
    for (int jc = j0; jc < j1; jc += P2P_T) {
      const int ns = min(P2P_T, j1 - jc);
      const int ns4 = (ns + 3) & ~3;
      __syncthreads();
      if ((int)threadIdx.x < ns) {
        int j = jc + threadIdx.x;
        xs[threadIdx.x] = (R)((sx[j] - ox) * S); ys[threadIdx.x] = (R)((sy[j] - oy) * S);
        zs[threadIdx.x] = (R)((sz[j] - oz) * S);
        for (int q = 0; q < NRC * 3; ++q) fs[q][threadIdx.x] = (R)sF[(int64_t)q * n + j];
      } else if ((int)threadIdx.x < ns4) {
        xs[threadIdx.x] = (R)1e30; ys[threadIdx.x] = (R)1e30; zs[threadIdx.x] = (R)1e30;
        for (int q = 0; q < NRC * 3; ++q) fs[q][threadIdx.x] = (R)0;
      }
      __syncthreads();
      R ar[NRC][3];
      for (int r = 0; r < NRC; ++r) ar[r][0] = ar[r][1] = ar[r][2] = (R)0;
      for (int s0 = 0; s0 < (wlive ? ns4 : 0); s0 += 4)
#pragma unroll
      for (int s = s0; s < s0 + 4; ++s) {
        const R dx = xi - xs[s], dy = yi - ys[s], dz = zi - zs[s];
        const R r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, k.r2min)));
        const R rinv = rinv_of(r2);
        const R ri2 = rinv * rinv, ri3 = ri2 * rinv;
        const R A = fma(k.a3, ri3, rinv), B = ri3 * fma(-k.a2, ri2, (R)1);
#pragma unroll
        for (int r = 0; r < NRC; ++r) {
          const R fx = fs[3 * r][s], fy = fs[3 * r + 1][s], fz = fs[3 * r + 2][s];
          const R sdf = B * fma(dx, fx, fma(dy, fy, dz * fz));
          ar[r][0] = fma(A, fx, fma(sdf, dx, ar[r][0]));
          ar[r][1] = fma(A, fy, fma(sdf, dy, ar[r][1]));
          ar[r][2] = fma(A, fz, fma(sdf, dz, ar[r][2]));
        }
      }
      for (int r = 0; r < NRC; ++r)
        for (int c = 0; c < 3; ++c) acc[r][c] += (double)ar[r][c];
    }
  }
  if (valid && any)
    for (int r = 0; r < NRC; ++r)
      for (int c = 0; c < 3; ++c) u[((int64_t)r * 3 + c) * n + i] += c1 * acc[r][c];
}

// ------------------------------------------------------- overlap (O) -----
// Pairs closer than 2a whose leaves are not adjacent: the far field treated
// them with the r >= 2a formula, so (M_overlap - M_far) F is added.  Same
// tiling as the P2P (padded, unrolled by 4); leaves of the O list are
// separated, so r > 0 and the far values are finite.  Pairs at r >= 2a get a
// zero coefficient (masked, no branch).  With the prefactor taken out and
// rho = r/(2a), the two branches' differences are
//   A' = oc (1 - 9r/(32a)) - 1/r - (2a^2/3)/r^3
//      = -(2a^2/3) (1 - rho)^2 (9 rho^2 + 2 rho + 1) / r^3,
//   B' = ob/r - (1 - 2a^2/r^2)/r^3 = 2a^2 (1 - rho)^2 (1 + rho)^2 / r^5,
// both with a double zero at r = 2a, where the branches meet.  In this
// factored form nothing cancels, so the mixed form evaluates it in FP32
// (rounding errors relative to the difference itself) and, as the P2P, adds
// each staged chunk's FP32 sums into FP64.  The FP64 form subtracts the two
// branches (fewer operations; the cancellation costs digits FP64 can spare).
// Most pairs of two such leaves are farther apart than 2a, so the staged
// sources are cut into groups of OV_G with bounding boxes, and a wave skips a
// group whose box is 2a or more from every one of the wave's targets.
constexpr int OV_G = 4;

template <int NRC, bool MIXED>
__global__ void __launch_bounds__(P2P_T) k_overlap(const int4* tiles, const double* tbox, Tree t, List O,
                                                   double four_a2, const double* sx,
                                                   const double* sy, const double* sz, const double* sF, int64_t n,
                                                   PairK<typename std::conditional<MIXED, float, double>::type> k,
                                                   double S, double c1, double* u) {
  using R = typename std::conditional<MIXED, float, double>::type;
  constexpr int NG = P2P_T / OV_G;
  __shared__ R xs[P2P_T], ys[P2P_T], zs[P2P_T];
  __shared__ R fs[NRC * 3][P2P_T];
  __shared__ R gbox[NG][6];  // per source group: lo xyz, hi xyz
  const int4 tl = tiles[blockIdx.x];
  const int b = tl.x;
  const int e0 = __builtin_amdgcn_readfirstlane(O.off[b]), e1 = __builtin_amdgcn_readfirstlane(O.off[b + 1]);
  if (e0 == e1) return;
  const bool valid = (int)threadIdx.x < tl.z;
  const bool wlive = (int)(threadIdx.x & ~63u) < tl.z;  // this wave holds a target of the tile
  const int i = tl.y + (valid ? threadIdx.x : 0);
  const double ox = t.cx[b], oy = t.cy[b], oz = t.cz[b];  // positions relative to the target leaf
  const R xi = (R)((sx[i] - ox) * S), yi = (R)((sy[i] - oy) * S), zi = (R)((sz[i] - oz) * S);
  // a group is skipped only when its box is clearly 2a away (rounding margin,
  // scaled units); idle lanes repeat the tile's first bead, so they add no
  // extra groups
  const R skip2 = k.four_a2 * (R)(1.0 + 1e-4);
  double acc[NRC][3];
  for (int r = 0; r < NRC; ++r) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
  double blo[3], bhi[3];
  for (int q = 0; q < 3; ++q) {
    blo[q] = tbox[6 * (int64_t)blockIdx.x + q];
    bhi[q] = tbox[6 * (int64_t)blockIdx.x + 3 + q];
  }
  for (int e = e0; e < e1; ++e) {
    const int C = __builtin_amdgcn_readfirstlane(O.ent[e]);
    // skip source leaves whose cube is 2a or more away from this tile's beads
    {
      const double hc = 0.5 * t.h[C], cc[3] = {t.cx[C], t.cy[C], t.cz[C]};
      double g2 = 0.0;
      for (int q = 0; q < 3; ++q) {
        const double g = fmax(0.0, fmax(cc[q] - hc - bhi[q], blo[q] - cc[q] - hc));
        g2 += g * g;
      }
      if (!(g2 < four_a2)) continue;
    }
    const int j1 = __builtin_amdgcn_readfirstlane(t.end[C]);
    for (int jc = __builtin_amdgcn_readfirstlane(t.begin[C]); jc < j1; jc += P2P_T) {
      const int ns = min(P2P_T, j1 - jc);
      const int ns4 = (ns + 3) & ~3;
      __syncthreads();
      if ((int)threadIdx.x < ns) {
        int j = jc + threadIdx.x;
        xs[threadIdx.x] = (R)((sx[j] - ox) * S); ys[threadIdx.x] = (R)((sy[j] - oy) * S);
        zs[threadIdx.x] = (R)((sz[j] - oz) * S);
        for (int q = 0; q < NRC * 3; ++q) fs[q][threadIdx.x] = (R)sF[(int64_t)q * n + j];
      } else if ((int)threadIdx.x < ns4) {
        xs[threadIdx.x] = (R)1e30; ys[threadIdx.x] = (R)1e30; zs[threadIdx.x] = (R)1e30;
        for (int q = 0; q < NRC * 3; ++q) fs[q][threadIdx.x] = (R)0;
      }
      __syncthreads();
      const int ng = (ns + OV_G - 1) / OV_G;
      if ((int)threadIdx.x < 3 * ng) {
        // box of the real sources of group g along one axis
        const int g = threadIdx.x / 3, q = threadIdx.x - 3 * g;
        const R* col = q == 0 ? xs : (q == 1 ? ys : zs);
        const int s1 = min(g * OV_G + OV_G, ns);
        R lo = col[g * OV_G], hi = lo;
        for (int s = g * OV_G + 1; s < s1; ++s) {
          lo = min(lo, col[s]);
          hi = max(hi, col[s]);
        }
        gbox[g][q] = lo;
        gbox[g][3 + q] = hi;
      }
      __syncthreads();
      R ar[NRC][3];
      for (int r = 0; r < NRC; ++r) ar[r][0] = ar[r][1] = ar[r][2] = (R)0;
      for (int g = 0; g < (wlive ? ng : 0); ++g) {
        // distance from this lane's target to the group's box; the wave
        // skips the group when no lane comes within 2a of it
        const R gx = max((R)0, max(gbox[g][0] - xi, xi - gbox[g][3]));
        const R gy = max((R)0, max(gbox[g][1] - yi, yi - gbox[g][4]));
        const R gz = max((R)0, max(gbox[g][2] - zi, zi - gbox[g][5]));
        const R g2 = fma(gx, gx, fma(gy, gy, gz * gz));
        if (!__any(g2 < skip2)) continue;  // wave-uniform
        const int s1 = min(g * OV_G + OV_G, ns4);
        for (int s0 = g * OV_G; s0 < s1; s0 += 4)
#pragma unroll
        for (int s = s0; s < s0 + 4; ++s) {
          const R dx = xi - xs[s], dy = yi - ys[s], dz = zi - zs[s];
          const R r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, k.r2min)));
          const R rinv = rinv_of(r2);
          const R ri2 = rinv * rinv, ri3 = ri2 * rinv;
          const bool ov = r2 < k.four_a2;
          R A, B;
          if constexpr (MIXED) {  // factored
            const R rho = (r2 - k.r2min) * rinv * k.i2a;
            const R om = (R)1 - rho, op = (R)1 + rho, w = om * om * ri3;
            A = ov ? -k.a3 * w * fma(fma((R)9, rho, (R)2), rho, (R)1) : (R)0;
            B = ov ? k.a2 * w * (op * op) * ri2 : (R)0;
          } else {  // the two branches and their difference (fewer operations)
            const R Af = fma(k.a3, ri3, rinv), Bf = ri3 * fma(-k.a2, ri2, (R)1);
            const R Ao = fma(-k.ock9, (r2 - k.r2min) * rinv, k.oc), Bo = k.ob * rinv;
            A = ov ? Ao - Af : (R)0;
            B = ov ? Bo - Bf : (R)0;
          }
#pragma unroll
          for (int r = 0; r < NRC; ++r) {
            const R fx = fs[3 * r][s], fy = fs[3 * r + 1][s], fz = fs[3 * r + 2][s];
            const R sdf = B * fma(dx, fx, fma(dy, fy, dz * fz));
            ar[r][0] = fma(A, fx, fma(sdf, dx, ar[r][0]));
            ar[r][1] = fma(A, fy, fma(sdf, dy, ar[r][1]));
            ar[r][2] = fma(A, fz, fma(sdf, dz, ar[r][2]));
          }
        }
      }
      for (int r = 0; r < NRC; ++r)
        for (int c = 0; c < 3; ++c) acc[r][c] += (double)ar[r][c];
    }
  }
  if (valid)
    for (int r = 0; r < NRC; ++r)
      for (int c = 0; c < 3; ++c) u[((int64_t)r * 3 + c) * n + i] += c1 * acc[r][c];
}

// Launch arguments shared by the pair kernels: the scale S (2aS in [1, 2)),
// the constants of the scaled radius in both precisions and the prefactor
// c1 S = S / (8 pi eta) that undoes the scaling of the sums.
struct PairLaunch {
  double S, c1S;
  PairK<float> kf;
  PairK<double> kd;
};

static PairLaunch pair_launch(double a, double eta) {
  PairLaunch q;
  q.S = pair_scale(a);
  q.c1S = q.S / (8.0 * PI * eta);
  q.kf = pair_const<float>(a * q.S);
  q.kd = pair_const<double>(a * q.S);
  return q;
}

hipError_t run_p2p(const Launch& l, const Tiles& tiles, int nrc, const double* sF, double* u, int mixed) {
  if (tiles.n == 0) return hipSuccess;
  const Built* B = l.B;
  const PairLaunch q = pair_launch(l.a, l.eta);
#define P2P_CASE(NR)                                                                                               \
  case NR:                                                                                                         \
    if (mixed)                                                                                                     \
      k_p2p<NR, true><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LU], B->sx, B->sy, B->sz, sF, B->n,     \
                                                  q.kf, q.S, q.c1S, u);                                            \
    else                                                                                                           \
      k_p2p<NR, false><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LU], B->sx, B->sy, B->sz, sF, B->n,    \
                                                   q.kd, q.S, q.c1S, u);                                           \
    break;
  switch (nrc) {
    P2P_CASE(1)
    P2P_CASE(2)
    P2P_CASE(4)
    P2P_CASE(8)
    case MF_R:
      if (mixed)
        k_p2p_mfma<true, 0><<<tiles.n, 64 * MF_W, 0, l.s>>>(tiles.t, B->tree, B->lists[LU], B->sx, B->sy, B->sz, sF,
                                                            B->n, q.kf, q.S, q.c1S, u);
      else
        k_p2p_mfma<false, 0><<<tiles.n, 64 * MF_W, 0, l.s>>>(tiles.t, B->tree, B->lists[LU], B->sx, B->sy, B->sz, sF,
                                                             B->n, q.kd, q.S, q.c1S, u);
      break;
    // 16 + XR: the FP64 form only
#define MF_CASE(XR)                                                                                                \
  case MF_R + XR:                                                                                                  \
    if (mixed) return hipErrorInvalidValue;                                                                        \
    k_p2p_mfma<false, XR><<<tiles.n, 64 * MF_W, 0, l.s>>>(tiles.t, B->tree, B->lists[LU], B->sx, B->sy, B->sz, sF,   \
                                                          B->n, q.kd, q.S, q.c1S, u);                              \
    break;
    MF_CASE(1)
    MF_CASE(2)
    MF_CASE(4)
    MF_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef P2P_CASE
#undef MF_CASE
  return hipGetLastError();
}

// The overlap correction: FP32 pair arithmetic (the factored differences)
// with FP64 sums per staged chunk in the mixed form, FP64 otherwise.
hipError_t run_overlap(const Launch& l, const Tiles& tiles, int nrc, const double* sF, double* u, int mixed) {
  const Built* B = l.B;
  if (tiles.n == 0 || B->lists[LO].len == 0) return hipSuccess;
  if (nrc > NEAR_VEC_RHS) {  // launches of 8 right-hand sides, then the rest
    const hipError_t he = run_overlap(l, tiles, NEAR_VEC_RHS, sF, u, mixed);
    const int64_t off = (int64_t)NEAR_VEC_RHS * 3 * B->n;
    return he != hipSuccess ? he : run_overlap(l, tiles, nrc - NEAR_VEC_RHS, sF + off, u + off, mixed);
  }
  const PairLaunch q = pair_launch(l.a, l.eta);
  const double four_a2 = 4.0 * l.a * l.a;
#define OV_CASE(NR)                                                                                                 \
  case NR:                                                                                                          \
    if (mixed)                                                                                                      \
      k_overlap<NR, true><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, tiles.box, B->tree, B->lists[LO], four_a2, B->sx,    \
                                                      B->sy, B->sz, sF, B->n, q.kf, q.S, q.c1S, u);                 \
    else                                                                                                            \
      k_overlap<NR, false><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, tiles.box, B->tree, B->lists[LO], four_a2, B->sx,   \
                                                       B->sy, B->sz, sF, B->n, q.kd, q.S, q.c1S, u);                \
    break;
  switch (nrc) {
    OV_CASE(1)
    OV_CASE(2)
    OV_CASE(4)
    OV_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef OV_CASE
  return hipGetLastError();
}

// The direct W sums are far-formula pair sums like the P2P: FP32 in the
// mixed form.
hipError_t run_wdirect(const Launch& l, const Tiles& tiles, int nrc, const double* sF, double* u, int mixed) {
  const Built* B = l.B;
  if (tiles.n == 0 || B->lists[LW].len == 0 || l.wd < 0) return hipSuccess;
  if (nrc > NEAR_VEC_RHS) {  // launches of 8 right-hand sides, then the rest
    const hipError_t he = run_wdirect(l, tiles, NEAR_VEC_RHS, sF, u, mixed);
    const int64_t off = (int64_t)NEAR_VEC_RHS * 3 * B->n;
    return he != hipSuccess ? he : run_wdirect(l, tiles, nrc - NEAR_VEC_RHS, sF + off, u + off, mixed);
  }
  const PairLaunch q = pair_launch(l.a, l.eta);
  const int wmax = l.wd;
#define WD_CASE(NR)                                                                                                 \
  case NR:                                                                                                          \
    if (mixed)                                                                                                      \
      k_wdirect<NR, true><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LW], wmax, B->sx, B->sy, B->sz, sF, \
                                                      B->n, q.kf, q.S, q.c1S, u);                                   \
    else                                                                                                            \
      k_wdirect<NR, false><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LW], wmax, B->sx, B->sy, B->sz,    \
                                                       sF, B->n, q.kd, q.S, q.c1S, u);                              \
    break;
  switch (nrc) {
    WD_CASE(1)
    WD_CASE(2)
    WD_CASE(4)
    WD_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef WD_CASE
  return hipGetLastError();
}


// ------------------------------------------------ sampled direct sums ---
// The exact RPY matvec (Sec. 1, all three blocks) at a few targets, summed
// over every bead of the target's system in FP64: the reference the
// autotuner measures candidate plans against.  One block per sampled
// target (tree order); threads stride over the sources and their partial
// sums are added in a fixed order.  sF is [nrc][3][n] in tree order; out is
// [k][nrc][3].
constexpr int DS_T = 256;
__global__ void __launch_bounds__(DS_T) k_direct_sample(const int* tgt, const int* sys_begin, int nsys,
                                                        const double* sx, const double* sy, const double* sz,
                                                        const double* sF, int64_t n, int nrc, double a, double eta,
                                                        double* out) {
  __shared__ double red[DS_T];
  const int i = tgt[blockIdx.x];
  // the target's system: sys_begin[s] <= i < sys_begin[s + 1] (binary search)
  int lo = 0, hi = nsys;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (sys_begin[mid] <= i) lo = mid;
    else hi = mid;
  }
  const int sy0 = sys_begin[lo], sy1 = sys_begin[lo + 1];
  const double xi = sx[i], yi = sy[i], zi = sz[i];
  const double c0 = 1.0 / (6.0 * PI * eta * a), c1 = 1.0 / (8.0 * PI * eta), four_a2 = 4.0 * a * a;
  for (int r = 0; r < nrc; ++r) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = sy0 + threadIdx.x; j < sy1; j += DS_T) {
      const double dx = xi - sx[j], dy = yi - sy[j], dz = zi - sz[j];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double fx = sF[((int64_t)r * 3 + 0) * n + j], fy = sF[((int64_t)r * 3 + 1) * n + j],
                   fz = sF[((int64_t)r * 3 + 2) * n + j];
      double A, B;
      if (r2 == 0.0) {
        A = c0;
        B = 0.0;
      } else if (r2 >= four_a2) {
        const double rr = sqrt(r2), cr = c1 / rr;
        A = cr * (1.0 + 2.0 * a * a / (3.0 * r2));
        B = cr * (1.0 - 2.0 * a * a / r2) / r2;
      } else {
        const double rr = sqrt(r2);
        A = c0 * (1.0 - 9.0 * rr / (32.0 * a));
        B = c0 * (3.0 / (32.0 * a)) / rr;
      }
      const double df = dx * fx + dy * fy + dz * fz;
      acc[0] += A * fx + B * df * dx;
      acc[1] += A * fy + B * df * dy;
      acc[2] += A * fz + B * df * dz;
    }
    for (int c = 0; c < 3; ++c) {
      red[threadIdx.x] = acc[c];
      __syncthreads();
      for (int w = DS_T / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
      }
      if (threadIdx.x == 0) out[((int64_t)blockIdx.x * nrc + r) * 3 + c] = red[0];
      __syncthreads();
    }
  }
}

hipError_t run_direct_sample(const Launch& l, const int* tgt, int k, int nrc, const double* sF, double* out) {
  const Built* B = l.B;
  if (k <= 0) return hipSuccess;
  k_direct_sample<<<k, DS_T, 0, l.s>>>(tgt, B->d_sys_begin, B->nsys, B->sx, B->sy, B->sz, sF, B->n, nrc, l.a,
                                       l.eta, out);
  return hipGetLastError();
}

}  // namespace rpy
