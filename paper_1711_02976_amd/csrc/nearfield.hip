// Near field of the RPY matvec: the exact RPY block (arXiv:1711.02976, Sec. 1,
// the three RPY block equations, kB*T = 1) summed over every bead of the
// U-list leaves of each target leaf (self term included), plus the overlap
// correction (M_overlap - M_far) F for pairs closer than 2a whose leaves are
// not adjacent (the far field treated them with the r >= 2a formula).
//
// One block of P2P_T threads per target tile (a leaf, or a P2P_T-bead slice
// of a large leaf); each lane owns one target and keeps 3 * nrc sums in
// registers; source beads of each U-list leaf are staged through LDS
// (positions and forces, SoA) and read back as wave-wide broadcasts.
#include <hip/hip_runtime.h>

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
  for (int s = t.begin[b]; s < t.end[b]; s += tile) out[o++] = make_int4(b, s, min(tile, t.end[b] - s), 0);
}

int make_tiles(const Built* B, int tile, Tiles* out, hipStream_t s, Error* err) {
  out->n = 0;
  out->t = nullptr;
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
  RPY_HIP(hipStreamSynchronize(s));
  (void)hipFree(cnt); (void)hipFree(off); (void)hipFree(tmp);
  return 0;
}

// ------------------------------------------------------------ pair math ---
// Coefficients of the RPY block M(d) = A I + B d d^T for one pair.
struct RpyConst {
  double c0;      // 1/(6 pi eta a): self mobility
  double c1;      // 1/(8 pi eta)
  double c1a3;    // c1 * 2a^2/3
  double c1a2;    // c1 * 2a^2
  double four_a2; // (2a)^2
  double k9;      // 9/(32a)
  double c0k3;    // c0 * 3/(32a)
};

// 1/r from the single-precision estimate refined by one Newton step
// (relative error below 2^-44); 0 for coincident beads (r^2 < 1e-30).
__device__ inline double rinv64(double r2) {
  double y = (double)__builtin_amdgcn_rsqf((float)r2);
  y = y * fma(-0.5 * r2, y * y, 1.5);
  return r2 < 1e-30 ? 0.0 : y;
}

// Far (r >= 2a) block: A = c1/r (1 + 2a^2/(3r^2)), B = c1/r^3 (1 - 2a^2/r^2).
__device__ inline void rpy_far(double rinv, const RpyConst& k, double& A, double& B) {
  const double ri2 = rinv * rinv, ri3 = ri2 * rinv;
  A = fma(k.c1a3, ri3, k.c1 * rinv);
  B = fma(-k.c1a2 * ri2, ri3, k.c1 * ri3);
}

// Overlap (r < 2a) block: A = c0 (1 - 9r/(32a)), B = c0 3/(32a) / r.
__device__ inline void rpy_overlap(double r2, double rinv, const RpyConst& k, double& A, double& B) {
  A = k.c0 * fma(-k.k9, r2 * rinv, 1.0);
  B = k.c0k3 * rinv;
}

struct RpyConstF {
  float c0, c1, c1a3, c1a2, four_a2, k9, c0k3;
};

// --------------------------------------------------------------- P2P -----
// The overlap formula is evaluated only when some lane of the wave has a
// source closer than 2a (a wave-uniform branch), since such pairs are rare.
template <int NRC, bool MIXED>
__global__ void __launch_bounds__(P2P_T) k_p2p(const int4* tiles, Tree t, List U, const double* sx,
                                               const double* sy, const double* sz, const double* sF, int64_t n,
                                               RpyConst k, RpyConstF kf, double* u) {
  __shared__ double xs[P2P_T], ys[P2P_T], zs[P2P_T];
  __shared__ double fs[NRC * 3][P2P_T];
  const int4 tl = tiles[blockIdx.x];
  const int b = tl.x;
  const bool valid = (int)threadIdx.x < tl.z;
  const int i = tl.y + (valid ? threadIdx.x : 0);
  const double xi = sx[i], yi = sy[i], zi = sz[i];
  double acc[NRC][3];
  for (int r = 0; r < NRC; ++r) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
  for (int e = U.off[b]; e < U.off[b + 1]; ++e) {
    const int C = U.ent[e];
    const int j1 = t.end[C];
    for (int jc = t.begin[C]; jc < j1; jc += P2P_T) {
      const int ns = min(P2P_T, j1 - jc);
      __syncthreads();
      if ((int)threadIdx.x < ns) {
        int j = jc + threadIdx.x;
        xs[threadIdx.x] = sx[j]; ys[threadIdx.x] = sy[j]; zs[threadIdx.x] = sz[j];
        for (int q = 0; q < NRC * 3; ++q) fs[q][threadIdx.x] = sF[(int64_t)q * n + j];
      }
      __syncthreads();
      if (MIXED) {
        float af[NRC][3];
        for (int r = 0; r < NRC; ++r) af[r][0] = af[r][1] = af[r][2] = 0.0f;
#pragma unroll 2
        for (int s = 0; s < ns; ++s) {
          const float dx = (float)(xi - xs[s]), dy = (float)(yi - ys[s]), dz = (float)(zi - zs[s]);
          const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          const float rinv = r2 < 1e-30f ? 0.0f : __builtin_amdgcn_rsqf(r2);
          const float ri2 = rinv * rinv, ri3 = ri2 * rinv;
          float A = fmaf(kf.c1a3, ri3, kf.c1 * rinv);
          float B = fmaf(-kf.c1a2 * ri2, ri3, kf.c1 * ri3);
          const bool ov = r2 < kf.four_a2;
          if (__builtin_expect(__any(ov), 0)) {
            const float Ao = kf.c0 * fmaf(-kf.k9, r2 * rinv, 1.0f), Bo = kf.c0k3 * rinv;
            A = ov ? Ao : A;
            B = ov ? Bo : B;
          }
#pragma unroll
          for (int r = 0; r < NRC; ++r) {
            const float fx = (float)fs[3 * r][s], fy = (float)fs[3 * r + 1][s], fz = (float)fs[3 * r + 2][s];
            const float sdf = B * fmaf(dx, fx, fmaf(dy, fy, dz * fz));
            af[r][0] = fmaf(A, fx, fmaf(sdf, dx, af[r][0]));
            af[r][1] = fmaf(A, fy, fmaf(sdf, dy, af[r][1]));
            af[r][2] = fmaf(A, fz, fmaf(sdf, dz, af[r][2]));
          }
        }
        for (int r = 0; r < NRC; ++r)
          for (int c = 0; c < 3; ++c) acc[r][c] += (double)af[r][c];
      } else {
#pragma unroll 2
        for (int s = 0; s < ns; ++s) {
          const double dx = xi - xs[s], dy = yi - ys[s], dz = zi - zs[s];
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          const double rinv = rinv64(r2);
          double A, B;
          rpy_far(rinv, k, A, B);
          const bool ov = r2 < k.four_a2;
          if (__builtin_expect(__any(ov), 0)) {
            double Ao, Bo;
            rpy_overlap(r2, rinv, k, Ao, Bo);
            A = ov ? Ao : A;
            B = ov ? Bo : B;
          }
#pragma unroll
          for (int r = 0; r < NRC; ++r) {
            const double fx = fs[3 * r][s], fy = fs[3 * r + 1][s], fz = fs[3 * r + 2][s];
            const double sdf = B * fma(dx, fx, fma(dy, fy, dz * fz));
            acc[r][0] = fma(A, fx, fma(sdf, dx, acc[r][0]));
            acc[r][1] = fma(A, fy, fma(sdf, dy, acc[r][1]));
            acc[r][2] = fma(A, fz, fma(sdf, dz, acc[r][2]));
          }
        }
      }
    }
  }
  if (valid)
    for (int r = 0; r < NRC; ++r)
      for (int c = 0; c < 3; ++c) u[((int64_t)r * 3 + c) * n + i] = acc[r][c];
}

// ------------------------------------------------------- overlap (O) -----
template <int NRC>
__global__ void __launch_bounds__(P2P_T) k_overlap(const int4* tiles, Tree t, List O, const double* sx,
                                                   const double* sy, const double* sz, const double* sF, int64_t n,
                                                   RpyConst k, double* u) {
  __shared__ double xs[P2P_T], ys[P2P_T], zs[P2P_T];
  __shared__ double fs[NRC * 3][P2P_T];
  const int4 tl = tiles[blockIdx.x];
  const int b = tl.x;
  if (O.off[b] == O.off[b + 1]) return;
  const bool valid = (int)threadIdx.x < tl.z;
  const int i = tl.y + (valid ? threadIdx.x : 0);
  const double xi = sx[i], yi = sy[i], zi = sz[i];
  double acc[NRC][3];
  for (int r = 0; r < NRC; ++r) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
  for (int e = O.off[b]; e < O.off[b + 1]; ++e) {
    const int C = O.ent[e];
    const int j1 = t.end[C];
    for (int jc = t.begin[C]; jc < j1; jc += P2P_T) {
      const int ns = min(P2P_T, j1 - jc);
      __syncthreads();
      if ((int)threadIdx.x < ns) {
        int j = jc + threadIdx.x;
        xs[threadIdx.x] = sx[j]; ys[threadIdx.x] = sy[j]; zs[threadIdx.x] = sz[j];
        for (int q = 0; q < NRC * 3; ++q) fs[q][threadIdx.x] = sF[(int64_t)q * n + j];
      }
      __syncthreads();
      for (int s = 0; s < ns; ++s) {
        const double dx = xi - xs[s], dy = yi - ys[s], dz = zi - zs[s];
        const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
        if (!(r2 < k.four_a2) || r2 < 1e-30) continue;
        const double rinv = 1.0 / sqrt(r2);
        double Af, Bf, Ao, Bo;
        rpy_far(rinv, k, Af, Bf);
        rpy_overlap(r2, rinv, k, Ao, Bo);
        const double A = Ao - Af, B = Bo - Bf;
        for (int r = 0; r < NRC; ++r) {
          const double fx = fs[3 * r][s], fy = fs[3 * r + 1][s], fz = fs[3 * r + 2][s];
          const double sdf = B * fma(dx, fx, fma(dy, fy, dz * fz));
          acc[r][0] = fma(A, fx, fma(sdf, dx, acc[r][0]));
          acc[r][1] = fma(A, fy, fma(sdf, dy, acc[r][1]));
          acc[r][2] = fma(A, fz, fma(sdf, dz, acc[r][2]));
        }
      }
    }
  }
  if (valid)
    for (int r = 0; r < NRC; ++r)
      for (int c = 0; c < 3; ++c) u[((int64_t)r * 3 + c) * n + i] += acc[r][c];
}

static RpyConst rpy_const(double a, double eta) {
  RpyConst k;
  k.c0 = 1.0 / (6.0 * PI * eta * a);
  k.c1 = 1.0 / (8.0 * PI * eta);
  k.c1a3 = k.c1 * 2.0 * a * a / 3.0;
  k.c1a2 = k.c1 * 2.0 * a * a;
  k.four_a2 = 4.0 * a * a;
  k.k9 = 9.0 / (32.0 * a);
  k.c0k3 = k.c0 * 3.0 / (32.0 * a);
  return k;
}

static RpyConstF rpy_const_f(const RpyConst& k) {
  return RpyConstF{(float)k.c0, (float)k.c1, (float)k.c1a3, (float)k.c1a2, (float)k.four_a2, (float)k.k9,
                   (float)k.c0k3};
}

hipError_t run_p2p(const Launch& l, const Tiles& tiles, int nrc, const double* sF, double* u, int mixed) {
  if (tiles.n == 0) return hipSuccess;
  const Built* B = l.B;
  RpyConst k = rpy_const(l.a, l.eta);
  RpyConstF kf = rpy_const_f(k);
#define P2P_CASE(NR)                                                                                            \
  case NR:                                                                                                      \
    if (mixed)                                                                                                  \
      k_p2p<NR, true><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LU], B->sx, B->sy, B->sz, sF, B->n, k, kf, u); \
    else                                                                                                        \
      k_p2p<NR, false><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LU], B->sx, B->sy, B->sz, sF, B->n, k, kf, u); \
    break;
  switch (nrc) {
    P2P_CASE(1)
    P2P_CASE(2)
    P2P_CASE(4)
    default: return hipErrorInvalidValue;
  }
#undef P2P_CASE
  return hipGetLastError();
}

hipError_t run_overlap(const Launch& l, const Tiles& tiles, int nrc, const double* sF, double* u) {
  const Built* B = l.B;
  if (tiles.n == 0 || B->lists[LO].len == 0) return hipSuccess;
  RpyConst k = rpy_const(l.a, l.eta);
  switch (nrc) {
    case 1: k_overlap<1><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LO], B->sx, B->sy, B->sz, sF, B->n, k, u); break;
    case 2: k_overlap<2><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LO], B->sx, B->sy, B->sz, sF, B->n, k, u); break;
    case 4: k_overlap<4><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LO], B->sx, B->sy, B->sz, sF, B->n, k, u); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace rpy
