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
  double twoa2_3; // 2a^2/3
  double twoa2;   // 2a^2
  double four_a2; // (2a)^2
  double k9;      // 9/(32a)
  double k3;      // 3/(32a)
};

__device__ inline void rpy_coef(double r2, const RpyConst& k, double& A, double& B) {
  // 1/r from a single-precision estimate refined by two Newton steps.
  float r2f = (float)r2;
  double y = (double)__builtin_amdgcn_rsqf(r2f);
  y = y * fma(-0.5 * r2, y * y, 1.5);
  y = y * fma(-0.5 * r2, y * y, 1.5);
  const bool coinc = r2 < 1e-30;
  const double rinv = coinc ? 0.0 : y;
  const double ri2 = rinv * rinv;
  const double Af = k.c1 * rinv * fma(k.twoa2_3, ri2, 1.0);
  const double Bf = k.c1 * rinv * ri2 * fma(-k.twoa2, ri2, 1.0);
  const double r = r2 * rinv;
  const double Ao = k.c0 * fma(-k.k9, r, 1.0);
  const double Bo = k.c0 * k.k3 * rinv;
  const bool ov = r2 < k.four_a2;
  A = ov ? Ao : Af;
  B = ov ? Bo : Bf;
}

__device__ inline void rpy_coef_f(float r2, float c0, float c1, float ta3, float ta, float fa2, float k9, float k3,
                                  float& A, float& B) {
  const bool coinc = r2 < 1e-30f;
  const float rinv = coinc ? 0.0f : __builtin_amdgcn_rsqf(r2);
  const float ri2 = rinv * rinv;
  const float Af = c1 * rinv * fmaf(ta3, ri2, 1.0f);
  const float Bf = c1 * rinv * ri2 * fmaf(-ta, ri2, 1.0f);
  const float r = r2 * rinv;
  const float Ao = c0 * fmaf(-k9, r, 1.0f);
  const float Bo = c0 * k3 * rinv;
  const bool ov = r2 < fa2;
  A = ov ? Ao : Af;
  B = ov ? Bo : Bf;
}

// --------------------------------------------------------------- P2P -----
template <int NRC, bool MIXED>
__global__ void __launch_bounds__(P2P_T) k_p2p(const int4* tiles, Tree t, List U, const double* sx,
                                               const double* sy, const double* sz, const double* sF, int64_t n,
                                               RpyConst k, double* u) {
  __shared__ double xs[P2P_T], ys[P2P_T], zs[P2P_T];
  __shared__ double fs[NRC * 3][P2P_T];
  const int4 tl = tiles[blockIdx.x];
  const int b = tl.x;
  const bool valid = (int)threadIdx.x < tl.z;
  const int i = tl.y + (valid ? threadIdx.x : 0);
  const double xi = sx[i], yi = sy[i], zi = sz[i];
  double acc[NRC][3];
  for (int r = 0; r < NRC; ++r) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
  const float c0f = (float)k.c0, c1f = (float)k.c1, ta3 = (float)k.twoa2_3, ta = (float)k.twoa2,
              fa2 = (float)k.four_a2, k9f = (float)k.k9, k3f = (float)k.k3;
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
        for (int s = 0; s < ns; ++s) {
          const float dx = (float)(xi - xs[s]), dy = (float)(yi - ys[s]), dz = (float)(zi - zs[s]);
          const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          float A, B;
          rpy_coef_f(r2, c0f, c1f, ta3, ta, fa2, k9f, k3f, A, B);
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
        for (int s = 0; s < ns; ++s) {
          const double dx = xi - xs[s], dy = yi - ys[s], dz = zi - zs[s];
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          double A, B;
          rpy_coef(r2, k, A, B);
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
        const double rinv = 1.0 / sqrt(r2), ri2 = rinv * rinv, r = r2 * rinv;
        const double A = k.c0 * fma(-k.k9, r, 1.0) - k.c1 * rinv * fma(k.twoa2_3, ri2, 1.0);
        const double B = k.c0 * k.k3 * rinv - k.c1 * rinv * ri2 * fma(-k.twoa2, ri2, 1.0);
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
  k.twoa2_3 = 2.0 * a * a / 3.0;
  k.twoa2 = 2.0 * a * a;
  k.four_a2 = 4.0 * a * a;
  k.k9 = 9.0 / (32.0 * a);
  k.k3 = 3.0 / (32.0 * a);
  return k;
}

hipError_t run_p2p(const Launch& l, const Tiles& tiles, int nrc, const double* sF, double* u, int mixed) {
  if (tiles.n == 0) return hipSuccess;
  const Built* B = l.B;
  RpyConst k = rpy_const(l.a, l.eta);
#define P2P_CASE(NR)                                                                                            \
  case NR:                                                                                                      \
    if (mixed)                                                                                                  \
      k_p2p<NR, true><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LU], B->sx, B->sy, B->sz, sF, B->n, k, u); \
    else                                                                                                        \
      k_p2p<NR, false><<<tiles.n, P2P_T, 0, l.s>>>(tiles.t, B->tree, B->lists[LU], B->sx, B->sy, B->sz, sF, B->n, k, u); \
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
