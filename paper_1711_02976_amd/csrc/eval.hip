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

// Adds the 12 sets of ER right-hand sides (at D + q stride, m-major, nmax)
// evaluated at this lane's target, offset (vx, vy, vz) from the expansion
// centre, box side h, to vel[q].  The harmonics are formed once for the ER
// right-hand sides:
// S_n^m = (n-m)!(n+m)! R_n^m (local; the factor is folded into the sets) or
// I_n^m (multipole), both by
//   h_m^m = -(2m-1) (x' + i y') h_{m-1}^{m-1},  h_0^0 = s',
//   h_n   = (2n-1) z' h_{n-1} - ((n-1)^2 - m^2) r' h_{n-2},
// (x', y', z', r', s') = (x, y, z, r^2, 1) or (x/r^2, y/r^2, z/r^2, 1/r^2, 1/r)
// in box units.  Each right-hand side's sums run in the same order whatever
// ER is.
template <bool MULT, int ER>
__device__ inline void eval_sets(const double2* __restrict__ D, int64_t stride, int nmax, double vx, double vy,
                                 double vz, double h, double C1, double (*vel)[3]) {
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
  double s[ER][12];
#pragma unroll
  for (int q = 0; q < ER; ++q)
#pragma unroll
    for (int e = 0; e < 12; ++e) s[q][e] = 0.0;
  auto acc = [&](double2 hv, const double2* d) {
#pragma unroll
    for (int q = 0; q < ER; ++q)
#pragma unroll
      for (int e = 0; e < 12; ++e) s[q][e] = fma(d[q * stride + e].x, hv.x, fma(-d[q * stride + e].y, hv.y, s[q][e]));
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
  for (int q = 0; q < ER; ++q)
#pragma unroll
    for (int i = 0; i < 3; ++i)
      vel[q][i] += s[q][i] - C1 * (vx * s[q][3 + 3 * i] + vy * s[q][4 + 3 * i] + vz * s[q][5 + 3 * i]);
}

// One wave per tile (leaf box, first bead, count <= 64, leaf ordinal),
// EV_WAVES consecutive tiles per block.  The evaluation shares the harmonics
// of each expansion between EV_RHS right-hand sides (two: on cube-15M the
// evaluation took 102 ms against 111 ms with one and 135 ms with four, where
// the sums' registers cut the occupancy).
constexpr int EV_WAVES = 4;
constexpr int EV_RHS = 2;
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
  constexpr int ER = NRC < EV_RHS ? NRC : EV_RHS;
  static_assert(NRC % ER == 0, "right-hand sides in whole groups of ER");
  for (int r = 0; r < NRC; ++r) vel[r][0] = vel[r][1] = vel[r][2] = 0.0;
  for (int r = 0; r < NRC; r += ER) {
    eval_sets<false, ER>(DL + ((int64_t)tl.w * NRC + r) * T * 12, (int64_t)T * 12, p, px - cx, py - cy, pz - cz, h,
                         C1, vel + r);
    for (int e = w0; e < w1; ++e) {
      const int C = W.ent[e];
      const int wi = widx[C];
      if (wi < 0) continue;  // few beads: summed directly with the near field
      eval_sets<true, ER>(DW + ((int64_t)wi * NRC + r) * To * 12, (int64_t)To * 12, p + 2, px - t.cx[C],
                          py - t.cy[C], pz - t.cz[C], t.h[C], C1, vel + r);
    }
  }
  if (lane < tl.z)
#pragma unroll
    for (int r = 0; r < NRC; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) u[((int64_t)r * 3 + k) * n + tl.y + lane] = vel[r][k];
}

// ------------------------------------------- second evaluation approach ---
// Sec. 2 names a second way to evaluate eq. (2.8): simplify each velocity
// component into a single expansion, then evaluate it.  About a leaf centre c
// the local part of component k,
//   U_k(v) = C1 L_k - C1 sum_s v_s d_k L_s + C1 d_k L_4 - C2 d_k sum_s d_s L_s,
// v = x - c, is a polynomial of degree p in v (v_s d_k L_s is not harmonic),
// so each leaf's three components are pre-assembled as polynomials in the
// monomials u_x^a u_y^b u_z^c of u = v / h, and every target evaluates them
// with nested Horner-like products.  These are also the polynomial
// expansions the paper's conclusion proposes for low accuracy: per target
// and right-hand side 3 (p+1)(p+2)(p+3)/6 multiply-adds and no harmonic
// recurrence, against 12 complex sets of (p+1)(p+2)/2 coefficients.
//
// Three kernels: k_poly_conv turns each (leaf, density) local expansion into
// monomial coefficients (a dense product with a table KcT of the monomial
// coefficients of R_n^m, shared by all leaves), k_poly_assemble forms the
// three components by index arithmetic (derivatives and products with u_s
// shift monomial indices), and k_eval_poly_apply evaluates them and adds the
// W-list multipoles (first approach, harmonic sets).
//
// Monomials of degree <= p are numbered with a outermost, then b, then c:
//   mono_index(a, b, c) = t3(p+1) - t3(p+1-a) + b (p-a+1) - b (b-1)/2 + c,
// t3(n) = n(n+1)(n+2)/6 (the number of monomials of degree < n).
__host__ __device__ inline int t3(int n) { return n * (n + 1) * (n + 2) / 6; }
__host__ __device__ inline int mono_count(int p) { return t3(p + 1); }
__host__ __device__ inline int mono_index(int p, int a, int b, int c) {
  return t3(p + 1) - t3(p + 1 - a) + b * (p - a + 1) - b * (b - 1) / 2 + c;
}

constexpr int POLY_T = 256;

// C[(i * ND + d) * NM + j] = (1/h) Re sum_n,m f_m E_d[n][m] R_n^m |_j for the
// ND densities of leaf i (f_m = 2 for m > 0), from the stored coefficients
// (L h^{n+1}) and KcT[t'][j] (t' = 2 (n,m) + {0: real, 1: imaginary part}).
// One block per leaf; each thread takes monomials j and keeps ND sums.
template <int ND>
__global__ void __launch_bounds__(POLY_T) k_poly_conv(int p, const int* leaves, Tree t, const double2* E,
                                                      const double* __restrict__ kct, double* C) {
  const int i = blockIdx.x, b = leaves[i];
  const int T = ncoef(p), NM = mono_count(p);
  extern __shared__ double Lr[];  // [2T][ND]
  const double2* src = E + (int64_t)b * ND * T;
  for (int x = threadIdx.x; x < ND * T; x += POLY_T) {
    const int d = x / T, c = x - d * T;
    const double2 v = src[x];
    Lr[(2 * c) * ND + d] = v.x;
    Lr[(2 * c + 1) * ND + d] = v.y;
  }
  __syncthreads();
  const double ih = 1.0 / t.h[b];
  for (int j = threadIdx.x; j < NM; j += POLY_T) {
    double acc[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] = 0.0;
    for (int q = 0; q < 2 * T; ++q) {
      const double k = kct[(int64_t)q * NM + j];
      if (k == 0.0) continue;  // R_n^m has only degree-n monomials
#pragma unroll
      for (int d = 0; d < ND; ++d) acc[d] = fma(k, Lr[q * ND + d], acc[d]);
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) C[((int64_t)i * ND + d) * NM + j] = acc[d] * ih;
  }
}

// The three component polynomials of leaf i and right-hand side r from its
// four density polynomials c_s (in u = v/h, with d/dv = (1/h) d/du):
//   U_k = C1 c_k - C1 sum_s u_s d_k c_s + (C1/h) d_k c_4 - (C2/h^2) d_k sum_s d_s c_s,
// written to U[((i * NM + j) * NRC + r) * 3 + k] (the order the evaluation
// reads them).
template <int NRC>
__global__ void __launch_bounds__(POLY_T) k_poly_assemble(int p, const int* leaves, Tree t, const double* C,
                                                          double C1, double C2, double* U) {
  constexpr int ND = 4 * NRC;
  const int i = blockIdx.x, r = blockIdx.y, b = leaves[i];
  const int NM = mono_count(p);
  extern __shared__ double cs[];  // [4][NM]
  for (int x = threadIdx.x; x < 4 * NM; x += POLY_T) {
    const int s = x / NM, j = x - s * NM;
    cs[x] = C[((int64_t)i * ND + 4 * r + s) * NM + j];
  }
  __syncthreads();
  const double h = t.h[b], c1h = C1 / h, c2h = C2 / (h * h);
  // coefficient of density s at exponents e (0 past degree p or below 0)
  auto at = [&](int s, int e0, int e1, int e2) -> double {
    if (e0 < 0 || e1 < 0 || e2 < 0 || e0 + e1 + e2 > p) return 0.0;
    return cs[s * NM + mono_index(p, e0, e1, e2)];
  };
  for (int x = threadIdx.x; x < 3 * NM; x += POLY_T) {
    const int k = x / NM, j = x - k * NM;
    int al[3] = {0, 0, 0};
    {
      int a = 0;
      while (t3(p + 1) - t3(p - a) <= j) ++a;
      const int rem = j - (t3(p + 1) - t3(p + 1 - a));
      int bb = 0;
      while (bb * (p - a + 1) - bb * (bb - 1) / 2 + (p - a - bb + 1) <= rem) ++bb;
      al[0] = a;
      al[1] = bb;
      al[2] = rem - (bb * (p - a + 1) - bb * (bb - 1) / 2);
    }
    double v = C1 * cs[k * NM + j];
    // -C1 sum_s u_s d_k c_s: the monomial alpha comes from beta = alpha - e_s
    // of d_k c_s, whose coefficient is (beta_k + 1) c_s[beta + e_k]
    for (int s = 0; s < 3; ++s) {
      if (al[s] == 0) continue;
      int be[3] = {al[0], al[1], al[2]};
      be[s] -= 1;
      const int bk = be[k];
      be[k] += 1;
      v -= C1 * (bk + 1) * at(s, be[0], be[1], be[2]);
    }
    int ak[3] = {al[0], al[1], al[2]};
    ak[k] += 1;  // alpha + e_k
    v += c1h * (al[k] + 1) * at(3, ak[0], ak[1], ak[2]);
    // -(C2/h^2) d_k sum_s d_s c_s
    double lc = 0.0;
    for (int s = 0; s < 3; ++s) {
      int g[3] = {ak[0], ak[1], ak[2]};
      const int gs = g[s];
      g[s] += 1;
      lc += (gs + 1) * at(s, g[0], g[1], g[2]);
    }
    v -= c2h * (al[k] + 1) * lc;
    U[(((int64_t)i * NM + j) * NRC + r) * 3 + k] = v;
  }
}

// One wave per tile of up to 64 beads of one leaf (as k_eval_apply): the
// leaf's component polynomials at u = (x - c)/h, read through scalar loads,
// plus the W-list multipoles through their evaluation sets.
template <int NRC>
__global__ void __launch_bounds__(64 * EV_WAVES) k_eval_poly_apply(int p, const int4* tiles, int ntiles, Tree t,
                                                                   List W, const int* widx, const double* sx,
                                                                   const double* sy, const double* sz, int64_t n,
                                                                   const double* __restrict__ DP,
                                                                   const double2* __restrict__ DW, double C1,
                                                                   double* __restrict__ u) {
  const int ti = blockIdx.x * EV_WAVES + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (ti >= ntiles) return;
  const int4 tl = tiles[ti];
  const int b = tl.x, lane = threadIdx.x & 63;
  const int j = tl.y + min(lane, tl.z - 1);
  const double px = sx[j], py = sy[j], pz = sz[j];
  const int To = ncoef(p + 2), NM = mono_count(p);
  const double ih = 1.0 / t.h[b];
  const double ux = (px - t.cx[b]) * ih, uy = (py - t.cy[b]) * ih, uz = (pz - t.cz[b]) * ih;
  double vel[NRC][3];
#pragma unroll
  for (int r = 0; r < NRC; ++r) vel[r][0] = vel[r][1] = vel[r][2] = 0.0;
  const double* D = DP + (int64_t)tl.w * NM * NRC * 3;
  double xa = 1.0;
  for (int a = 0; a <= p; ++a) {
    double yb = xa;
    for (int bb = 0; a + bb <= p; ++bb) {
      double zc = yb;
      for (int c = 0; a + bb + c <= p; ++c) {
#pragma unroll
        for (int r = 0; r < NRC; ++r)
#pragma unroll
          for (int k = 0; k < 3; ++k) vel[r][k] = fma(D[3 * r + k], zc, vel[r][k]);
        D += 3 * NRC;
        zc *= uz;
      }
      yb *= uy;
    }
    xa *= ux;
  }
  const int w0 = W.off[b], w1 = W.off[b + 1];
  for (int r = 0; r < NRC; ++r)
    for (int e = w0; e < w1; ++e) {
      const int C = W.ent[e];
      const int wi = widx[C];
      if (wi < 0) continue;  // few beads: summed directly with the near field
      eval_sets<true, 1>(DW + ((int64_t)wi * NRC + r) * To * 12, 0, p + 2, px - t.cx[C], py - t.cy[C],
                         pz - t.cz[C], t.h[C], C1, vel + r);
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
  if (ep.nwbig > 0)
    ks<<<dim3(ep.nwbig, NRC), SETS_T, shm_m, l.s>>>(p, true, ep.wbig, B->tree, e.M, l.tb->rscale, C1, C2, e.DW);
  he = hipGetLastError();
  if (he != hipSuccess) return he;
  if (ep.mode == EVAL_POLY) {
    // second approach: component polynomials per leaf (DL's buffer holds them)
    constexpr int ND = 4 * NRC;
    const int NM = mono_count(p);
    double* DP = reinterpret_cast<double*>(e.DL);
    const size_t shm_c = sizeof(double) * 2 * ncoef(p) * ND, shm_a = sizeof(double) * 4 * NM;
    auto kc = k_poly_conv<ND>;
    auto ka = k_poly_assemble<NRC>;
    he = hipFuncSetAttribute(reinterpret_cast<const void*>(kc), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm_c);
    if (he == hipSuccess)
      he = hipFuncSetAttribute(reinterpret_cast<const void*>(ka), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm_a);
    if (he != hipSuccess) return he;
    kc<<<B->nleaf, POLY_T, shm_c, l.s>>>(p, B->leaf_ids, B->tree, e.L, ep.kct, e.PV);
    ka<<<dim3(B->nleaf, NRC), POLY_T, shm_a, l.s>>>(p, B->leaf_ids, B->tree, e.PV, C1, C2, DP);
    if (ep.tiles.n > 0)
      k_eval_poly_apply<NRC><<<(ep.tiles.n + EV_WAVES - 1) / EV_WAVES, 64 * EV_WAVES, 0, l.s>>>(
          p, ep.tiles.t, ep.tiles.n, B->tree, B->lists[LW], ep.widx, B->sx, B->sy, B->sz, B->n, DP, e.DW, C1, u);
    return hipGetLastError();
  }
  ks<<<dim3(B->nleaf, NRC), SETS_T, shm_l, l.s>>>(p, false, B->leaf_ids, B->tree, e.L, l.tb->rscale, C1, C2, e.DL);
  if (ep.tiles.n > 0)
    k_eval_apply<NRC><<<(ep.tiles.n + EV_WAVES - 1) / EV_WAVES, 64 * EV_WAVES, 0, l.s>>>(
        p, ep.tiles.t, ep.tiles.n, B->tree, B->lists[LW], ep.widx, B->sx, B->sy, B->sz,
                                                  B->n, e.DL, e.DW, C1, u);
  return hipGetLastError();
}

}  // namespace

// Monomial coefficients of the regular harmonics R_n^m(u) = r^n P_n^m e^{i m phi}
// / (n+m)! (0 <= m <= n <= p), generated as polynomials by the recurrence
//   R_0^0 = 1,  R_m^m = -(u_x + i u_y) R_{m-1}^{m-1} / (2m),  R_{m+1}^m = u_z R_m^m,
//   R_n^m = ((2n-1) u_z R_{n-1}^m - |u|^2 R_{n-2}^m) / ((n+m)(n-m)),
// and written, with the factor 2 for m > 0, as the real table
// KcT[2 (n,m) + 0][j] = f_m Re R_n^m|_j, KcT[2 (n,m) + 1][j] = -f_m Im R_n^m|_j,
// so that Re(f_m E R_n^m) = sum_q KcT[q][j] e_q for E = e_0 + i e_1.
static std::vector<double> poly_table(int p) {
  const int T = ncoef(p), NM = mono_count(p);
  std::vector<double> re((size_t)T * NM, 0.0), im((size_t)T * NM, 0.0);
  auto I = [&](int n, int m) { return (size_t)tri(n) + m; };
  auto J = [&](int a, int b, int c) { return mono_index(p, a, b, c); };
  // dst (degree n) += w * (u_z^k or |u|^2 or (u_x + i u_y)) * src (degree n-1 or n-2)
  re[I(0, 0) * NM + J(0, 0, 0)] = 1.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      const double w = -1.0 / (2.0 * m);
      const size_t s = I(m - 1, m - 1) * NM, d = I(m, m) * NM;
      for (int a = 0; a <= p; ++a)
        for (int b = 0; a + b <= p; ++b)
          for (int c = 0; a + b + c < p; ++c) {
            const double xr = re[s + J(a, b, c)], xi = im[s + J(a, b, c)];
            if (xr == 0.0 && xi == 0.0) continue;
            // (u_x + i u_y)(xr + i xi) = u_x xr - u_y xi + i (u_x xi + u_y xr)
            re[d + J(a + 1, b, c)] += w * xr;
            im[d + J(a + 1, b, c)] += w * xi;
            re[d + J(a, b + 1, c)] -= w * xi;
            im[d + J(a, b + 1, c)] += w * xr;
          }
    }
    for (int n = m + 1; n <= p; ++n) {
      const size_t d = I(n, m) * NM, s1 = I(n - 1, m) * NM;
      const double w1 = n == m + 1 ? 1.0 : (2.0 * n - 1.0) / ((double)(n + m) * (n - m));
      const double w2 = n == m + 1 ? 0.0 : -1.0 / ((double)(n + m) * (n - m));
      for (int a = 0; a <= p; ++a)
        for (int b = 0; a + b <= p; ++b)
          for (int c = 0; a + b + c < p; ++c) {
            const double xr = re[s1 + J(a, b, c)], xi = im[s1 + J(a, b, c)];
            re[d + J(a, b, c + 1)] += w1 * xr;
            im[d + J(a, b, c + 1)] += w1 * xi;
          }
      if (w2 != 0.0) {
        const size_t s2 = I(n - 2, m) * NM;
        for (int a = 0; a <= p; ++a)
          for (int b = 0; a + b <= p; ++b)
            for (int c = 0; a + b + c + 2 <= p; ++c) {
              const double xr = re[s2 + J(a, b, c)], xi = im[s2 + J(a, b, c)];
              const int e[3][3] = {{a + 2, b, c}, {a, b + 2, c}, {a, b, c + 2}};
              for (const auto& q : e) {
                re[d + J(q[0], q[1], q[2])] += w2 * xr;
                im[d + J(q[0], q[1], q[2])] += w2 * xi;
              }
            }
      }
    }
  }
  std::vector<double> kct((size_t)2 * T * NM);
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m <= n; ++m) {
      const double f = m ? 2.0 : 1.0;
      for (int j = 0; j < NM; ++j) {
        kct[(2 * I(n, m)) * NM + j] = f * re[I(n, m) * NM + j];
        kct[(2 * I(n, m) + 1) * NM + j] = -f * im[I(n, m) * NM + j];
      }
    }
  return kct;
}

int make_eval_plan(const Built* B, int p, int wd, int mode, EvalPlan* out, hipStream_t s, Error* err) {
  out->nwbig = 0;
  out->widx = out->wbig = nullptr;
  out->kct = nullptr;
  out->mode = mode;
  if (mode == EVAL_POLY) {
    const std::vector<double> k = poly_table(p);
    RPY_HIP(hipMalloc(&out->kct, sizeof(double) * k.size()));
    RPY_HIP(hipMemcpy(out->kct, k.data(), sizeof(double) * k.size(), hipMemcpyHostToDevice));
  }
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
  if (ep->kct) (void)hipFree(ep->kct);
  ep->tiles = Tiles{};
  ep->widx = ep->wbig = nullptr;
  ep->kct = nullptr;
  ep->nwbig = 0;
}

int64_t eval_sets_bytes(const Built* B, const EvalPlan& ep, int p, int nrc, int64_t* dw_bytes, int64_t* pv_bytes) {
  const int64_t per = (int64_t)sizeof(double2) * 12 * nrc;
  const int64_t nleaf = std::max(B->nleaf, 1);
  *dw_bytes = per * ncoef(p + 2) * std::max(ep.nwbig, 1);
  if (ep.mode == EVAL_POLY) {
    // component polynomials (in DL's buffer) and the density polynomials
    *pv_bytes = (int64_t)sizeof(double) * 4 * nrc * mono_count(p) * nleaf;
    return (int64_t)sizeof(double) * 3 * nrc * mono_count(p) * nleaf;
  }
  *pv_bytes = sizeof(double);
  return per * ncoef(p) * nleaf;
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
