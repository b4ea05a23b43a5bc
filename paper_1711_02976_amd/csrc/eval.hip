// Target evaluation of the far field (arXiv:1711.02976, eq. (2.8) with
// Theorem 2 for a box's local expansion and Theorem 1 for the multipoles of
// its W list).
//
// Every expansion (four densities per right-hand side) is first turned into
// twelve real-symmetric coefficient sets
//   E_i  = C1 L_i + C1 d_i L4 - C2 d_i (d_x L1 + d_y L2 + d_z L3)
//   G_ik = d_i L_k                                   (i, k in x, y, z)
// so that at a target x with offset v = x - c from the expansion centre,
//   u_i = Re sum_c [E_i - C1 sum_k v_k G_ik]_c h_c(x)
// (h the regular or irregular harmonics).  This holds for any centre c as
// long as the fourth density was formed about the same c, so a W-list
// multipole is evaluated about its own box centre.
//
// Two kernels: one block per expansion builds its sets (in LDS) and writes
// them to a device array, coefficient-major in the order the evaluation
// walks them (order m, then degree n), with the factor 2 for m > 0 and, for
// local expansions, 1/((n-m)!(n+m)!) folded in; then one wave per tile of
// up to 64 beads of a leaf evaluates the leaf's sets and those of its W-list
// multipoles, with the coefficients read through scalar loads (uniform over
// the wave) and lane = target.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "fmm.h"

namespace rpy {

namespace {

constexpr double PI = 3.14159265358979323846;

// Coefficient C_n^m of a real-symmetric set stored for m >= 0 (C^{-m} =
// (-1)^m conj(C^m)); zero outside 0 <= n <= nmax, |m| <= n.
__device__ inline double2 getc(const double2* C, int n, int m, int nmax) {
  if (n < 0 || n > nmax || m > n || m < -n) return make_double2(0.0, 0.0);
  if (m >= 0) return C[tri(n) + m];
  double2 v = C[tri(n) - m];
  return (m & 1) ? make_double2(-v.x, v.y) : make_double2(v.x, -v.y);
}

// Derivative of a real-symmetric set in coefficient space.  Local (regular)
// sets: d_z C -> C_{n+1}^m, d_x -> (C_{n+1}^{m-1} - C_{n+1}^{m+1})/2,
// d_y -> -i (C_{n+1}^{m-1} + C_{n+1}^{m+1})/2.  Multipole (irregular) sets use
// n-1 in place of n+1 and d_z -> -C_{n-1}^m.
__device__ inline double2 dcoef(const double2* C, int nmax, int n, int m, int axis, bool mult) {
  int nn = mult ? n - 1 : n + 1;
  if (axis == 2) {
    double2 v = getc(C, nn, m, nmax);
    return mult ? make_double2(-v.x, -v.y) : v;
  }
  double2 a = getc(C, nn, m - 1, nmax), b = getc(C, nn, m + 1, nmax);
  if (axis == 0) return make_double2(0.5 * (a.x - b.x), 0.5 * (a.y - b.y));
  return make_double2(0.5 * (a.y + b.y), -0.5 * (a.x + b.x));
}

// Builds the 12 evaluation sets of one expansion in LDS (box side h):
//   D[3 + 3i + k] = h^-2 d_i L_k          (k, i = 0..2),
//   D[i]          = C1 h^-1 L_i + C1 h^-2 d_i L_4 - C2 h^-3 d_i L_C,
// with L_C = sum_k d_k L_k (degree <= nout; a multipole's sets have degree
// nin + 2).  G4 (3 sets) and LC are scratch.
__device__ void derived_sets(const double2* src, int nin, int nout, bool mult, double h, double C1, double C2,
                             double2* D, double2* G4, double2* LC) {
  const int To = ncoef(nout);
  const double ih = 1.0 / h, ih2 = ih * ih, ih3 = ih2 * ih;
  for (int w = threadIdx.x; w < 12 * To; w += blockDim.x) {
    const int k = w / (3 * To), rem = w - k * 3 * To, i = rem / To, c = rem - i * To;
    int n = 0;
    while (tri(n + 1) <= c) ++n;
    const int m = c - tri(n);
    const double2 g = dcoef(src + k * ncoef(nin), nin, n, m, i, mult);
    if (k < 3) D[(3 + 3 * i + k) * To + c] = make_double2(ih2 * g.x, ih2 * g.y);
    else G4[i * To + c] = g;
  }
  __syncthreads();
  const double h2 = h * h;
  for (int c = threadIdx.x; c < To; c += blockDim.x) {
    const double2 a = D[3 * To + c], b = D[7 * To + c], d = D[11 * To + c];
    LC[c] = make_double2(h2 * (a.x + b.x + d.x), h2 * (a.y + b.y + d.y));
  }
  __syncthreads();
  for (int w = threadIdx.x; w < 3 * To; w += blockDim.x) {
    const int i = w / To, c = w - i * To;
    int n = 0;
    while (tri(n + 1) <= c) ++n;
    const int m = c - tri(n);
    const double2 l = getc(src + i * ncoef(nin), n, m, nin);
    const double2 g4 = G4[i * To + c];
    const double2 dc = dcoef(LC, nout, n, m, i, mult);
    D[i * To + c] = make_double2(C1 * ih * l.x + C1 * ih2 * g4.x - C2 * ih3 * dc.x,
                                 C1 * ih * l.y + C1 * ih2 * g4.y - C2 * ih3 * dc.y);
  }
  __syncthreads();
}

constexpr int SETS_T = 256;

// One block per (expansion, right-hand side): the 12 sets of box boxes[i]'s
// expansion E (local: mult = false, degree p; multipole: degree p + 2),
// written as out[((i * NRC + r) * To + k) * 12 + e] for the m-major index k.
// rscale[tri(n)+m] = 1/((n-m)!(n+m)!) (local sets only).
template <int NRC>
__global__ void __launch_bounds__(SETS_T) k_eval_sets(int p, bool mult, const int* boxes, Tree t, const double2* E,
                                                      const double* __restrict__ rscale, double C1, double C2,
                                                      double2* out) {
  constexpr int ND = 4 * NRC;
  const int i = blockIdx.x, r = blockIdx.y;
  const int b = boxes[i];
  const int T = ncoef(p), nout = mult ? p + 2 : p, To = ncoef(nout);
  extern __shared__ double2 sm[];
  double2* D = sm;            // 12 * To
  double2* G4 = D + 12 * To;  // 3 * To
  double2* LC = G4 + 3 * To;  // To
  double2* src = LC + To;     // 4 * T
  const double2* in = E + ((int64_t)b * ND + 4 * r) * T;
  for (int x = threadIdx.x; x < 4 * T; x += SETS_T) src[x] = in[x];
  __syncthreads();
  derived_sets(src, p, nout, mult, t.h[b], C1, C2, D, G4, LC);
  double2* o = out + ((int64_t)i * NRC + r) * To * 12;
  for (int w = threadIdx.x; w < 12 * To; w += SETS_T) {
    const int k = w / 12, e = w - 12 * k;
    int m = 0, base = 0;
    while (base + (nout - m + 1) <= k) {
      base += nout - m + 1;
      ++m;
    }
    const int n = m + (k - base), c = tri(n) + m;
    double f = m ? 2.0 : 1.0;
    if (!mult) f *= rscale[c];
    const double2 v = D[e * To + c];
    o[w] = make_double2(f * v.x, f * v.y);
  }
}

// Adds the 12 sets at D (m-major, nmax) evaluated at this lane's target,
// offset (vx, vy, vz) from the expansion centre, box side h.  Harmonics:
// S_n^m = (n-m)!(n+m)! R_n^m (local; the factor is folded into the sets) or
// I_n^m (multipole), both by
//   h_m^m = -(2m-1) (x' + i y') h_{m-1}^{m-1},  h_0^0 = s',
//   h_n   = (2n-1) z' h_{n-1} - ((n-1)^2 - m^2) r' h_{n-2},
// (x', y', z', r', s') = (x, y, z, r^2, 1) or (x/r^2, y/r^2, z/r^2, 1/r^2, 1/r)
// in box units.
template <bool MULT>
__device__ inline void eval_sets(const double2* __restrict__ D, int nmax, double vx, double vy, double vz, double h,
                                 double C1, double* vel) {
  const double ih = 1.0 / h, x = vx * ih, y = vy * ih, z = vz * ih;
  const double r2 = x * x + y * y + z * z;
  double zz, rr, ux, uy, sc;
  if (MULT) {
    rr = 1.0 / r2;
    zz = z * rr;
    ux = x * rr;
    uy = y * rr;
    sc = sqrt(rr);
  } else {
    rr = r2;
    zz = z;
    ux = x;
    uy = y;
    sc = 1.0;
  }
  double s[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) s[e] = 0.0;
  auto acc = [&](double2 hv, const double2* d) {
#pragma unroll
    for (int e = 0; e < 12; ++e) s[e] = fma(d[e].x, hv.x, fma(-d[e].y, hv.y, s[e]));
  };
  double2 dg = make_double2(sc, 0.0);
  const double2* Dp = D;
  for (int m = 0; m <= nmax; ++m) {
    if (m > 0) {
      const double f = -(2.0 * m - 1.0);
      dg = make_double2(f * (ux * dg.x - uy * dg.y), f * (ux * dg.y + uy * dg.x));
    }
    double2 h0 = make_double2(0.0, 0.0), h1 = dg;
    double ca = 2.0 * m + 1.0, cb = 0.0;
    acc(h1, Dp);
    Dp += 12;
    int n = m + 1;
    // two degrees per trip, each overwriting the older of (h0, h1)
    for (; n + 1 <= nmax; n += 2) {
      double A = ca * zz, Bc = cb * rr;
      h0 = make_double2(A * h1.x - Bc * h0.x, A * h1.y - Bc * h0.y);
      cb += ca;
      ca += 2.0;
      acc(h0, Dp);
      A = ca * zz;
      Bc = cb * rr;
      h1 = make_double2(A * h0.x - Bc * h1.x, A * h0.y - Bc * h1.y);
      cb += ca;
      ca += 2.0;
      acc(h1, Dp + 12);
      Dp += 24;
    }
    if (n <= nmax) {
      const double A = ca * zz, Bc = cb * rr;
      acc(make_double2(A * h1.x - Bc * h0.x, A * h1.y - Bc * h0.y), Dp);
      Dp += 12;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) vel[i] += s[i] - C1 * (vx * s[3 + 3 * i] + vy * s[4 + 3 * i] + vz * s[5 + 3 * i]);
}

// One wave per tile (leaf box, first bead, count <= 64, leaf ordinal),
// EV_WAVES consecutive tiles per block.
constexpr int EV_WAVES = 4;
// Writes (assigns) the far-field velocity of every bead of the tile.
template <int NRC>
__global__ void __launch_bounds__(64 * EV_WAVES) k_eval_apply(int p, const int4* tiles, int ntiles, Tree t, List W,
                                                             const int* widx,
                                                   const double* sx, const double* sy, const double* sz, int64_t n,
                                                   const double2* __restrict__ DL, const double2* __restrict__ DW,
                                                   double C1, double* __restrict__ u) {
  // consecutive tiles (mostly of one leaf) share a block, hence a CU and its
  // scalar cache, and walk the same set coefficients at about the same time
  const int ti = blockIdx.x * EV_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (ti >= ntiles) return;
  const int4 tl = tiles[ti];
  const int b = tl.x, lane = threadIdx.x & 63;
  const int j = tl.y + min(lane, tl.z - 1);
  const double px = sx[j], py = sy[j], pz = sz[j];
  const int T = ncoef(p), To = ncoef(p + 2);
  const double cx = t.cx[b], cy = t.cy[b], cz = t.cz[b], h = t.h[b];
  const int w0 = W.off[b], w1 = W.off[b + 1];
  // all loads before the first store, so that the set arrays can be read
  // through the scalar cache
  double vel[NRC][3];
  for (int r = 0; r < NRC; ++r) {
    vel[r][0] = vel[r][1] = vel[r][2] = 0.0;
    eval_sets<false>(DL + ((int64_t)tl.w * NRC + r) * T * 12, p, px - cx, py - cy, pz - cz, h, C1, vel[r]);
    for (int e = w0; e < w1; ++e) {
      const int C = W.ent[e];
      const int wi = widx[C];
      if (wi < 0) continue;  // few beads: summed directly with the near field
      eval_sets<true>(DW + ((int64_t)wi * NRC + r) * To * 12, p + 2, px - t.cx[C], py - t.cy[C], pz - t.cz[C],
                      t.h[C], C1, vel[r]);
    }
  }
  if (lane < tl.z)
#pragma unroll
    for (int r = 0; r < NRC; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) u[((int64_t)r * 3 + k) * n + tl.y + lane] = vel[r][k];
}

// W-list boxes whose multipoles the evaluation uses: flag[C] = 1 for every
// W-list entry C with more than wd beads (every entry when wd < 0).
__global__ void k_wbig_flag(List W, Tree t, int wd, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W.len) return;
  const int C = W.ent[i];
  if (wd < 0 || t.end[C] - t.begin[C] > wd) flag[C] = 1;
}

__global__ void k_wbig_index(const int* flag, const int* off, int nbox, int* widx, int* wbig) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  widx[b] = flag[b] ? off[b] : -1;
  if (flag[b]) wbig[off[b]] = b;
}

template <int NRC>
hipError_t launch_eval(const Launch& l, const EvalPlan& ep, Exp e, double* u) {
  const Built* B = l.B;
  const int p = l.p;
  const double C1 = 1.0 / (8.0 * PI * l.eta), C2 = l.a * l.a / (12.0 * PI * l.eta);
  auto ks = k_eval_sets<NRC>;
  const size_t shm_l = sizeof(double2) * (16 * ncoef(p) + 4 * ncoef(p));
  const size_t shm_m = sizeof(double2) * (16 * ncoef(p + 2) + 4 * ncoef(p));
  hipError_t he = hipFuncSetAttribute(reinterpret_cast<const void*>(ks), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)shm_m);
  if (he != hipSuccess) return he;
  ks<<<dim3(B->nleaf, NRC), SETS_T, shm_l, l.s>>>(p, false, B->leaf_ids, B->tree, e.L, l.tb->rscale, C1, C2, e.DL);
  if (ep.nwbig > 0)
    ks<<<dim3(ep.nwbig, NRC), SETS_T, shm_m, l.s>>>(p, true, ep.wbig, B->tree, e.M, l.tb->rscale, C1, C2, e.DW);
  he = hipGetLastError();
  if (he != hipSuccess) return he;
  if (ep.tiles.n > 0)
    k_eval_apply<NRC><<<(ep.tiles.n + EV_WAVES - 1) / EV_WAVES, 64 * EV_WAVES, 0, l.s>>>(
        p, ep.tiles.t, ep.tiles.n, B->tree, B->lists[LW], ep.widx, B->sx, B->sy, B->sz,
                                                  B->n, e.DL, e.DW, C1, u);
  return hipGetLastError();
}

}  // namespace

int make_eval_plan(const Built* B, int p, int wd, EvalPlan* out, hipStream_t s, Error* err) {
  out->nwbig = 0;
  out->widx = out->wbig = nullptr;
  if (make_tiles(B, 64, &out->tiles, s, err) != 0) return -1;
  const int nbox = std::max(B->tree.nbox, 1);
  int *flag = nullptr, *off = nullptr, *tmp = nullptr;
  RPY_HIP(hipMalloc(&out->widx, sizeof(int) * nbox));
  RPY_HIP(hipMalloc(&flag, sizeof(int) * nbox));
  RPY_HIP(hipMalloc(&off, sizeof(int) * nbox));
  RPY_HIP(hipMalloc(&tmp, sizeof(int) * scan_tmp_ints(nbox)));
  RPY_HIP(hipMemsetAsync(flag, 0, sizeof(int) * nbox, s));
  const List& W = B->lists[LW];
  if (W.len > 0) k_wbig_flag<<<(unsigned)((W.len + 255) / 256), 256, 0, s>>>(W, B->tree, wd, flag);
  RPY_HIP(hipGetLastError());
  RPY_HIP(scan_exclusive(flag, off, nbox, tmp, s));
  int last[2] = {0, 0};
  RPY_HIP(hipMemcpyAsync(&last[0], off + nbox - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  RPY_HIP(hipMemcpyAsync(&last[1], flag + nbox - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  RPY_HIP(hipStreamSynchronize(s));
  out->nwbig = last[0] + last[1];
  RPY_HIP(hipMalloc(&out->wbig, sizeof(int) * std::max(out->nwbig, 1)));
  k_wbig_index<<<(nbox + 255) / 256, 256, 0, s>>>(flag, off, nbox, out->widx, out->wbig);
  RPY_HIP(hipGetLastError());
  RPY_HIP(hipStreamSynchronize(s));
  (void)hipFree(flag);
  (void)hipFree(off);
  (void)hipFree(tmp);
  return 0;
}

void free_eval_plan(EvalPlan* ep) {
  if (ep->tiles.t) (void)hipFree(ep->tiles.t);
  if (ep->tiles.box) (void)hipFree(ep->tiles.box);
  if (ep->widx) (void)hipFree(ep->widx);
  if (ep->wbig) (void)hipFree(ep->wbig);
  ep->tiles = Tiles{};
  ep->widx = ep->wbig = nullptr;
  ep->nwbig = 0;
}

int64_t eval_sets_bytes(const Built* B, const EvalPlan& ep, int p, int nrc, int64_t* dw_bytes) {
  const int64_t per = (int64_t)sizeof(double2) * 12 * nrc;
  *dw_bytes = per * ncoef(p + 2) * std::max(ep.nwbig, 1);
  return per * ncoef(p) * std::max(B->nleaf, 1);
}

hipError_t run_eval(const Launch& l, const EvalPlan& ep, int nrc, Exp e, double* u) {
  if (l.B->nleaf == 0) return hipSuccess;
  switch (nrc) {
    case 1: return launch_eval<1>(l, ep, e, u);
    case 2: return launch_eval<2>(l, ep, e, u);
    case 4: return launch_eval<4>(l, ep, e, u);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rpy
