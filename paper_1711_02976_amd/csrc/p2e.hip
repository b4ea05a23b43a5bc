// Particle -> expansion kernels of the four-Laplace FMM (arXiv:1711.02976,
// Sec. 2, the multipole and local expansion forms of a Laplace potential;
// Fig. 1's S->M and S->L operators): S->M for the leaves and S->L for the X
// lists of the adaptive tree.  Both are the contraction
//
//   E_n^m[d] = sum_j conj(Y_n^m(r_j - c)) q_j[d]
//
// of the bead charges q_j (F_x, F_y, F_z and the fourth charge F.(r - c) per
// right-hand side) with the regular (S->M) or irregular (S->L) solid
// harmonics about the expansion centre c, in the box-scaled normalisation of
// the other far-field kernels.
//
// Layout of the work.  A block (8 waves) sweeps the beads of its source
// leaves in chunks of 64.  Generation: lane = bead, and each wave walks a
// fixed set of orders m (a balanced bin of whole columns n = m..p), so the
// degree/order of every step is wave-uniform (a per-pass descriptor says
// where columns start) and no step reads memory; the harmonics go to LDS
// as [bead][slot].
// Accumulation: a dense product on the FP64 matrix cores.  Per chunk and
// pass it is D[2S rows][ND] += H^T[2S rows][64 beads] x Q[64 beads][ND], the
// rows being the real and imaginary parts of the pass's S coefficient slots,
// done as v_mfma_f64_16x16x4f64 tiles of 16 rows x 16 densities (densities
// past ND are zero) over 4 beads per instruction; wave w owns the row tiles
// w, w + 8, ... for the whole box, so no sums cross waves.  One right-hand
// side (ND = 4) would leave three quarters of each tile empty and
// accumulates on the vector units instead (see k_p2e).  A column may run
// over several passes of K steps per wave; the recurrence state stays in
// registers between passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "fmm.h"

namespace rpy {

namespace {

__device__ inline double2 zmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

typedef double v4d __attribute__((ext_vector_type(4)));  // a 16x16 FP64 matrix-core tile per wave

constexpr int P2E_WAVES = 8;
constexpr int P2E_THREADS = 64 * P2E_WAVES;
constexpr int P2E_CHUNK = 64;  // beads per chunk = lanes per wave

// Charges per bead for the S->M/S->L contraction, [n][4 nrc] (bead-major so a
// wave reads one bead's charges with a scalar load): F_x, F_y, F_z and
// F.(r - c_leaf) per right-hand side, c_leaf the centre of the bead's leaf.
template <int NRC>
__global__ void __launch_bounds__(256) k_leaf_q(const int* leaves, Tree t, const double* sx, const double* sy,
                                                const double* sz, const double* sF, int64_t n, double* Q) {
  constexpr int ND = 4 * NRC;
  const int b = leaves[blockIdx.x];
  const double cx = t.cx[b], cy = t.cy[b], cz = t.cz[b];
  for (int j = t.begin[b] + threadIdx.x; j < t.end[b]; j += blockDim.x) {
    const double dx = sx[j] - cx, dy = sy[j] - cy, dz = sz[j] - cz;
#pragma unroll
    for (int r = 0; r < NRC; ++r) {
      const double fx = sF[((int64_t)r * 3 + 0) * n + j], fy = sF[((int64_t)r * 3 + 1) * n + j],
                   fz = sF[((int64_t)r * 3 + 2) * n + j];
      double* q = Q + (int64_t)j * ND + 4 * r;
      q[0] = fx;
      q[1] = fy;
      q[2] = fz;
      q[3] = fx * dx + fy * dy + fz * dz;
    }
  }
}

// The regular harmonics are generated unnormalised, S_n^m = (n-m)!(n+m)! R_n^m,
// and the irregular ones as they are, so that both obey
//   h_n = (2n-1) z' h_{n-1} - ((n-1)^2 - m^2) r' h_{n-2},
//   h_m = (-1)^m (2m-1)!! (x' + i y')^m s'
// with (x', y', z', r', s') = (x, y, z, r^2, 1) for S_n^m and
// (x/r^2, y/r^2, z/r^2, 1/r^2, 1/r) for I_n^m (box units about the centre);
// the two integer coefficients are kept as running FP64 counters, and
// S_n^m is scaled back to R_n^m per coefficient when the sums are written.
//
// K generation steps per wave and pass, P passes: S = 8 K slots per pass,
// G = S / 64 slot groups, NB = 8 / G bead subsets (partial sums per slot).
template <int ND, bool LOCAL, int K, int P>
__global__ void __launch_bounds__(P2E_THREADS) k_p2e(int p, const int* ids, const int4* __restrict__ xwork,
                                                     const int2* __restrict__ xchunks, Tree t, List X, const double* sx,
                                                     const double* sy, const double* sz, const double* __restrict__ Q,
                                                     const P2EPass* __restrict__ desc,
                                                     const int* __restrict__ slot_coef,
                                                     const double* __restrict__ slot_scale,
                                                     const double* __restrict__ dk, double2* E,
                                                     double2* __restrict__ part) {
  constexpr int NRC = ND / 4;
  constexpr int S = P2E_WAVES * K;
  constexpr int LD = S + 1;  // odd row stride: conflict-free [bead][slot] writes
  constexpr int TPW = K / 8;  // 16-row tiles per wave: 2S rows / 16 / 8 waves
  // One right-hand side (4 densities) fills only a quarter of a 16-column
  // matrix-core tile: it accumulates on the vector units instead, lane =
  // slot of one of G = S / 64 slot groups, the waves split into NB = 8 / G
  // bead subsets of BPW beads whose partial sums are added at the end.
  constexpr bool VEC = ND == 4;
  constexpr int G = S / 64, NB = P2E_WAVES / G, BPW = P2E_CHUNK / NB;
  static_assert(!VEC || NB * ND * S <= P2E_CHUNK * LD, "partial sums fit in the harmonics' LDS");
  const int T = ncoef(p);
  // S->M: one leaf per block.  S->L: one work item per block, a run of the
  // box's X entries and a range of 64-bead chunks of each; a box whose X
  // work was split over several items writes each item's share to its own
  // slot of `part`, and k_p2l_reduce adds the slots in a fixed order
  int b, e0 = 0, e1 = 1, clo = 0, chi = 0x7fffffff;
  int pslot = -1;
  if (LOCAL) {
    const int4 wk = xwork[blockIdx.x];
    const int2 ch = xchunks[blockIdx.x];
    b = wk.x;
    e0 = wk.y;
    e1 = wk.z;
    pslot = wk.w - 1;
    clo = ch.x;
    chi = ch.y;
  } else {
    b = ids ? ids[blockIdx.x] : blockIdx.x;
  }
  extern __shared__ double2 Hs[];  // [64][LD]
  // S->L: the chunk's charges with the fourth one re-centred on this machine,
  // computed once per bead instead of once per (bead, slot)
  __shared__ double Qs[LOCAL ? P2E_CHUNK * ND : 1];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;  // matrix-core operand row / column and k index
  const int grp = wv % G, sub = wv / G, slot = grp * 64 + lane;  // vector accumulation
  const double cx = t.cx[b], cy = t.cy[b], cz = t.cz[b], ih = 1.0 / t.h[b];
  v4d acc[VEC ? 1 : P][VEC ? 1 : TPW];
  double2 vacc[VEC ? P : 1][VEC ? ND : 1];
#pragma unroll
  for (int ps = 0; ps < (VEC ? 0 : P); ++ps)
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[ps][q] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ps = 0; ps < (VEC ? P : 0); ++ps)
#pragma unroll
    for (int d = 0; d < ND; ++d) vacc[ps][d] = make_double2(0.0, 0.0);

  for (int e = e0; e < e1; ++e) {
    const int C = LOCAL ? X.ent[e] : b;
    int j0 = t.begin[C], j1 = t.end[C];
    if (LOCAL) {
      j1 = (int)min((int64_t)j1, (int64_t)j0 + (int64_t)chi * P2E_CHUNK);
      j0 += clo * P2E_CHUNK;
    }
    // Q holds the fourth charge about the source leaf's centre; about c:
    // F.(r - c) = F.(r - c_C) + F.(c_C - c)
    double wx = 0.0, wy = 0.0, wz = 0.0;
    if (LOCAL) {
      wx = t.cx[C] - cx;
      wy = t.cy[C] - cy;
      wz = t.cz[C] - cz;
    }
    for (int jc = j0; jc < j1; jc += P2E_CHUNK) {
      const int nb = min(P2E_CHUNK, j1 - jc);
      const int jl = jc + (lane < nb ? lane : 0);  // idle lanes: a valid bead, zero weight
      const double x = (sx[jl] - cx) * ih, y = (sy[jl] - cy) * ih, z = (sz[jl] - cz) * ih;
      const double r2 = x * x + y * y + z * z;
      double zz, rr, ux, uy, sc;
      if (LOCAL) {
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
      if (lane >= nb) sc = 0.0;  // every harmonic of an idle lane is zero
      double2 h0 = make_double2(0.0, 0.0), h1 = h0;
      double ca = 0.0, cb = 0.0;  // 2n - 1 and (n-1)^2 - m^2 for the next degree n
#pragma unroll
      for (int ps = 0; ps < P; ++ps) {
        const P2EPass d = desc[wv * P + ps];
        uint64_t ml = ((uint64_t)d.mhi << 32) | d.mlo;
        double2* hw = Hs + lane * LD + wv * K;  // this lane's row, this wave's slots
        __syncthreads();                        // the previous accumulation is done with Hs
        if (LOCAL && ps == 0 && (int)threadIdx.x < P2E_CHUNK * NRC) {
          const int bb = threadIdx.x % P2E_CHUNK, r = threadIdx.x / P2E_CHUNK;
          const double* q = Q + (int64_t)(jc + bb) * ND + 4 * r;
          const double q0 = q[0], q1 = q[1], q2 = q[2];
          double* o = Qs + bb * ND + 4 * r;
          o[0] = q0;
          o[1] = q1;
          o[2] = q2;
          o[3] = fma(q0, wx, fma(q1, wy, fma(q2, wz, q[3])));
        }
        // conj(h) obeys the same recurrence (real coefficients): generate it directly
        int k = 0;
        while (k < d.nvalid) {
          if ((d.start >> k) & 1u) {
            // a column starts: diagonal harmonic of order m by binary powering
            const int m = (int)(ml & 31u);
            ml >>= 5;
            double2 hv = make_double2(dk[m] * sc, 0.0);
            double2 bp = make_double2(ux, -uy);
            for (int ex = m; ex; ex >>= 1) {
              if (ex & 1) hv = zmul(hv, bp);
              bp = zmul(bp, bp);
            }
            h0 = make_double2(0.0, 0.0);
            h1 = hv;
            ca = 2.0 * m + 1.0;
            cb = 0.0;
            hw[k] = hv;
            ++k;
          }
          const uint32_t rest = k < 32 ? d.start >> k : 0u;
          const int ke = rest ? min(k + __builtin_ctz(rest), d.nvalid) : d.nvalid;
          // two steps per trip, each overwriting the older of (h0, h1)
          for (; k + 1 < ke; k += 2) {
            double A = ca * zz, Bc = cb * rr;
            h0 = make_double2(A * h1.x - Bc * h0.x, A * h1.y - Bc * h0.y);
            cb += ca;
            ca += 2.0;
            hw[k] = h0;
            A = ca * zz;
            Bc = cb * rr;
            h1 = make_double2(A * h0.x - Bc * h1.x, A * h0.y - Bc * h1.y);
            cb += ca;
            ca += 2.0;
            hw[k + 1] = h1;
          }
          if (k < ke) {
            const double A = ca * zz, Bc = cb * rr;
            const double2 hv = make_double2(A * h1.x - Bc * h0.x, A * h1.y - Bc * h0.y);
            cb += ca;
            ca += 2.0;
            h0 = h1;
            h1 = hv;
            hw[k] = hv;
            ++k;
          }
        }
        for (; k < K; ++k) hw[k] = make_double2(0.0, 0.0);
        __syncthreads();
        // D += H^T Q over the chunk's beads, 4 per instruction: A[row][k] in
        // lane row + 16 k (row = real or imaginary part of a slot), B[k][d]
        // in lane d + 16 k, D[row][d] in lane d + 16 (row % 4), item row / 4;
        // beads past nb have zero harmonics and finite (padded) charges
        if constexpr (VEC) {
          // beads past nb have zero harmonics; Q is padded past the last bead
          if (sub * BPW < nb) {
#pragma unroll
            for (int i = 0; i < BPW; ++i) {
              const int bb = sub * BPW + i;
              const double* q = LOCAL ? Qs + bb * ND : Q + (int64_t)(jc + bb) * ND;
              const double2 h = Hs[bb * LD + slot];
#pragma unroll
              for (int dd = 0; dd < ND; ++dd) {
                const double qd = q[dd];
                vacc[ps][dd].x = fma(qd, h.x, vacc[ps][dd].x);
                vacc[ps][dd].y = fma(qd, h.y, vacc[ps][dd].y);
              }
            }
          }
        } else {
          const double* hd = reinterpret_cast<const double*>(Hs);
          for (int kk = 0; kk < nb; kk += 4) {
            const int bb = kk + lk;
            double bq = 0.0;
            if (li < ND) bq = LOCAL ? Qs[bb * ND + li] : Q[(int64_t)(jc + bb) * ND + li];
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
              const int row = (wv + 8 * q) * 16 + li;
              const double a = hd[2 * (bb * LD + (row >> 1)) + (row & 1)];
              acc[ps][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bq, acc[ps][q], 0, 0, 0);
            }
          }
        }
      }
    }
  }
  if constexpr (VEC) {
    // add the NB partial sums per slot (through LDS) and write the expansion
    double2* Rs = Hs;
#pragma unroll
    for (int ps = 0; ps < P; ++ps) {
      __syncthreads();
#pragma unroll
      for (int d = 0; d < ND; ++d) Rs[(sub * ND + d) * S + slot] = vacc[ps][d];
      __syncthreads();
      for (int o = threadIdx.x; o < ND * S; o += P2E_THREADS) {
        const int d = o / S, sl = o - d * S;
        const int c = slot_coef[ps * S + sl];
        if (c < 0) continue;
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const double2 w = Rs[(k * ND + d) * S + sl];
          v.x += w.x;
          v.y += w.y;
        }
        if (LOCAL && pslot >= 0) {
          part[((int64_t)pslot * ND + d) * T + c] = v;
          continue;
        }
        double2* out = E + ((int64_t)b * ND + d) * T + c;
        if (LOCAL) {
          const double2 o0 = *out;
          v.x += o0.x;
          v.y += o0.y;
        } else {
          const double f = slot_scale[ps * S + sl];  // S_n^m -> R_n^m
          v.x *= f;
          v.y *= f;
        }
        *out = v;
      }
    }
    return;
  }
  // write the expansion: D[i][d] sits in lane d + 16 (i % 4), item i / 4, so
  // a lane holds rows of one parity only (real parts for even lk, imaginary
  // parts for odd lk) and writes each component on its own
#pragma unroll
  for (int ps = 0; ps < P; ++ps)
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
      const int d = li;
      if (d >= ND) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = (wv + 8 * q) * 16 + 4 * v + lk;
        const int sl = row >> 1;  // slot within the pass; row & 1: real or imaginary part
        const int c = slot_coef[ps * S + sl];
        if (c < 0) continue;
        double x = acc[ps][q][v];
        if (LOCAL && pslot >= 0) {
          reinterpret_cast<double*>(part + ((int64_t)pslot * ND + d) * T + c)[row & 1] = x;
          continue;
        }
        double* out = reinterpret_cast<double*>(E + ((int64_t)b * ND + d) * T + c) + (row & 1);
        if (LOCAL) x += *out;
        else x *= slot_scale[ps * S + sl];  // S_n^m -> R_n^m
        *out = x;
      }
    }
}

// Adds the split S->L shares of one box (xred: box, first slot, slot count)
// to its local expansion, slot by slot in item order.
template <int ND>
__global__ void __launch_bounds__(256) k_p2l_reduce(int p, const int4* __restrict__ xred, const double2* __restrict__ part,
                                                    double2* E) {
  const int T = ncoef(p);
  const int4 rd = xred[blockIdx.x];
  for (int i = threadIdx.x; i < ND * T; i += blockDim.x) {
    double2 v = E[(int64_t)rd.x * ND * T + i];
    for (int k = 0; k < rd.z; ++k) {
      const double2 w = part[(int64_t)(rd.y + k) * ND * T + i];
      v.x += w.x;
      v.y += w.y;
    }
    E[(int64_t)rd.x * ND * T + i] = v;
  }
}

template <int ND, bool LOCAL, int K, int P>
hipError_t launch_p2e(const Launch& l, const P2ESched& sc, int grid, const int* ids, const double* Q, double2* E,
                      double2* part) {
  const Built* B = l.B;
  if (grid == 0) return hipSuccess;
  const size_t shm = sizeof(double2) * P2E_CHUNK * (P2E_WAVES * K + 1);
  auto kern = k_p2e<ND, LOCAL, K, P>;
  hipError_t he = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (he != hipSuccess) return he;
  kern<<<grid, P2E_THREADS, shm, l.s>>>(l.p, ids, B->xwork, B->xchunks, B->tree, B->lists[LX], B->sx, B->sy, B->sz, Q,
                                        sc.desc, sc.slot, sc.scale, l.tb->p2e_dk, E, part);
  he = hipGetLastError();
  if (he != hipSuccess || !LOCAL || B->nxred == 0) return he;
  k_p2l_reduce<ND><<<B->nxred, 256, 0, l.s>>>(l.p, B->xred, part, E);
  return hipGetLastError();
}

// Schedule choice: 8 steps per wave and pass (66 KB of LDS, two blocks per
// CU) whenever its packing fits in at most 4 passes (7 for one right-hand
// side, the orders above 21); else 16 steps (132 KB, one block per CU).  The
// matrix-core accumulators take 8 registers per pass and row tile.
template <int ND, bool LOCAL>
hipError_t launch_p2e_kp(const Launch& l, int grid, const int* ids, const double* Q, double2* E, double2* part) {
  const P2ESched& s8 = l.tb->p2e[0];
  const P2ESched& s16 = l.tb->p2e[1];
  switch (s8.P) {
    case 1: return launch_p2e<ND, LOCAL, 8, 1>(l, s8, grid, ids, Q, E, part);
    case 2: return launch_p2e<ND, LOCAL, 8, 2>(l, s8, grid, ids, Q, E, part);
    case 3: return launch_p2e<ND, LOCAL, 8, 3>(l, s8, grid, ids, Q, E, part);
    case 4: return launch_p2e<ND, LOCAL, 8, 4>(l, s8, grid, ids, Q, E, part);
    default: break;
  }
  if constexpr (ND == 4) {
    switch (s8.P) {
      case 5: return launch_p2e<ND, LOCAL, 8, 5>(l, s8, grid, ids, Q, E, part);
      case 6: return launch_p2e<ND, LOCAL, 8, 6>(l, s8, grid, ids, Q, E, part);
      case 7: return launch_p2e<ND, LOCAL, 8, 7>(l, s8, grid, ids, Q, E, part);
      default: break;
    }
  }
  if (s16.P == 1) return launch_p2e<ND, LOCAL, 16, 1>(l, s16, grid, ids, Q, E, part);
  if (s16.P == 2) return launch_p2e<ND, LOCAL, 16, 2>(l, s16, grid, ids, Q, E, part);
  return hipErrorInvalidValue;
}

template <bool LOCAL>
hipError_t launch_p2e_nd(const Launch& l, int nrc, int grid, const int* ids, const double* Q, double2* E,
                         double2* part) {
  switch (nrc) {
    case 1: return launch_p2e_kp<4, LOCAL>(l, grid, ids, Q, E, part);
    case 2: return launch_p2e_kp<8, LOCAL>(l, grid, ids, Q, E, part);
    case 4: return launch_p2e_kp<16, LOCAL>(l, grid, ids, Q, E, part);
    default: return hipErrorInvalidValue;
  }
}

// First-fit decreasing of the columns m = 0..p (lengths p - m + 1) into 8
// bins of capacity cap.
bool pack_columns(int p, int cap, std::vector<std::vector<int>>& bins) {
  bins.assign(P2E_WAVES, {});
  std::vector<int> load(P2E_WAVES, 0);
  for (int m = 0; m <= p; ++m) {
    const int len = p - m + 1;
    int w = 0;
    while (w < P2E_WAVES && load[w] + len > cap) ++w;
    if (w == P2E_WAVES) return false;
    bins[w].push_back(m);
    load[w] += len;
  }
  return true;
}

}  // namespace

// Builds the schedule with K steps per wave and pass and the fewest passes
// (at most maxp) whose column packing fits; false if none does.
static int build_sched(int p, int K, int maxp, P2ESched* out, Error* err, int64_t* bytes) {
  out->K = K;
  out->P = 0;
  std::vector<std::vector<int>> bins;
  int P = 0;
  for (int q = 1; q <= maxp && P == 0; ++q)
    if (pack_columns(p, K * q, bins)) P = q;
  if (P == 0) return 0;
  const int S = P2E_WAVES * K;
  std::vector<P2EPass> desc((size_t)P2E_WAVES * P, P2EPass{0u, 0, 0u, 0u});
  std::vector<int> slot((size_t)P * S, -1);
  std::vector<double> scale((size_t)P * S, 0.0), fac(2 * p + 2, 1.0);
  for (int j = 1; j <= 2 * p + 1; ++j) fac[j] = fac[j - 1] * j;
  for (int w = 0; w < P2E_WAVES; ++w) {
    int k = 0;
    std::vector<int> nst(P, 0);
    for (int m : bins[w])
      for (int n = m; n <= p; ++n, ++k) {
        const int ps = k / K, kk = k % K;
        P2EPass& d = desc[(size_t)w * P + ps];
        if (n == m) {
          if (nst[ps] == 12) {
            err->code = -1;
            err->msg = "particle-to-expansion schedule: too many columns in one pass";
            return -1;
          }
          d.start |= 1u << kk;
          const uint64_t ml = ((uint64_t)d.mhi << 32 | d.mlo) | ((uint64_t)m << (5 * nst[ps]++));
          d.mlo = (uint32_t)ml;
          d.mhi = (uint32_t)(ml >> 32);
        }
        d.nvalid = kk + 1;
        slot[(size_t)ps * S + w * K + kk] = tri(n) + m;
        scale[(size_t)ps * S + w * K + kk] = 1.0 / (fac[n - m] * fac[n + m]);
      }
  }
  RPY_HIP(hipMalloc(&out->desc, sizeof(P2EPass) * desc.size()));
  RPY_HIP(hipMalloc(&out->slot, sizeof(int) * slot.size()));
  RPY_HIP(hipMalloc(&out->scale, sizeof(double) * scale.size()));
  RPY_HIP(hipMemcpy(out->desc, desc.data(), sizeof(P2EPass) * desc.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(out->slot, slot.data(), sizeof(int) * slot.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(out->scale, scale.data(), sizeof(double) * scale.size(), hipMemcpyHostToDevice));
  *bytes += sizeof(P2EPass) * desc.size() + (sizeof(int) + sizeof(double)) * slot.size();
  out->P = P;
  return 1;
}

// S->L work items.  A box's X entries are cut into runs of at most `cap`
// 64-bead chunks, and an entry longer than that into chunk ranges, so that
// no block carries much more than its share: on 64 systems at leaf 1640 one
// box held 344 chunks against 17 per CU on average, and its block set the
// kernel's length.  cap = max(16, total / 2048).
int make_p2l_work(Built* B, hipStream_t s, Error* err) {
  if (B->xwork) (void)hipFree(B->xwork);
  if (B->xchunks) (void)hipFree(B->xchunks);
  if (B->xred) (void)hipFree(B->xred);
  B->xwork = nullptr;
  B->xchunks = nullptr;
  B->xred = nullptr;
  B->nxwork = B->nxshared = B->nxred = 0;
  const List& X = B->lists[LX];
  const int nbox = B->tree.nbox;
  if (X.len == 0 || nbox == 0) return 0;
  std::vector<int> off(nbox + 1), ent(X.len), beg(nbox), end(nbox);
  RPY_HIP(hipMemcpyAsync(off.data(), X.off, sizeof(int) * (nbox + 1), hipMemcpyDeviceToHost, s));
  RPY_HIP(hipMemcpyAsync(ent.data(), X.ent, sizeof(int) * X.len, hipMemcpyDeviceToHost, s));
  RPY_HIP(hipMemcpyAsync(beg.data(), B->tree.begin, sizeof(int) * nbox, hipMemcpyDeviceToHost, s));
  RPY_HIP(hipMemcpyAsync(end.data(), B->tree.end, sizeof(int) * nbox, hipMemcpyDeviceToHost, s));
  RPY_HIP(hipStreamSynchronize(s));
  auto chunks = [&](int e) { return (end[ent[e]] - beg[ent[e]] + P2E_CHUNK - 1) / P2E_CHUNK; };
  int64_t total = 0;
  for (int64_t e = 0; e < X.len; ++e) total += chunks((int)e);
  const int cap = (int)std::max<int64_t>(16, total / 2048);
  std::vector<int4> work, red;
  std::vector<int2> rng;
  int nslot = 0;
  for (int b = 0; b < nbox; ++b) {
    const size_t first = work.size();
    int e = off[b];
    while (e < off[b + 1]) {
      const int c = chunks(e);
      if (c > cap) {  // one long entry: chunk ranges of it
        for (int lo = 0; lo < c; lo += cap) {
          work.push_back(make_int4(b, e, e + 1, 0));
          rng.push_back(make_int2(lo, std::min(c, lo + cap)));
        }
        ++e;
        continue;
      }
      int e1 = e, sum = 0;
      while (e1 < off[b + 1] && chunks(e1) <= cap && sum + chunks(e1) <= cap) sum += chunks(e1++);
      work.push_back(make_int4(b, e, e1, 0));
      rng.push_back(make_int2(0, 0x7fffffff));
      e = e1;
    }
    if (work.size() - first > 1) {
      // shares of one box: slots nslot.. in item order, reduced afterwards
      red.push_back(make_int4(b, nslot, (int)(work.size() - first), 0));
      for (size_t i = first; i < work.size(); ++i) work[i].w = 1 + nslot++;
    }
  }
  B->nxwork = (int)work.size();
  B->nxshared = nslot;
  B->nxred = (int)red.size();
  RPY_HIP(hipMalloc(&B->xwork, sizeof(int4) * work.size()));
  RPY_HIP(hipMalloc(&B->xchunks, sizeof(int2) * rng.size()));
  RPY_HIP(hipMemcpy(B->xwork, work.data(), sizeof(int4) * work.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(B->xchunks, rng.data(), sizeof(int2) * rng.size(), hipMemcpyHostToDevice));
  B->bytes += (int64_t)(sizeof(int4) + sizeof(int2)) * work.size();
  if (!red.empty()) {
    RPY_HIP(hipMalloc(&B->xred, sizeof(int4) * red.size()));
    RPY_HIP(hipMemcpy(B->xred, red.data(), sizeof(int4) * red.size(), hipMemcpyHostToDevice));
    B->bytes += (int64_t)sizeof(int4) * red.size();
  }
  return 0;
}

int make_p2e_tables(int p, Tables* tb, Error* err) {
  int64_t bytes = 0;
  const int r8 = build_sched(p, 8, 7, &tb->p2e[0], err, &bytes);
  if (r8 < 0) return -1;
  const int r16 = build_sched(p, 16, 2, &tb->p2e[1], err, &bytes);
  if (r16 < 0) return -1;
  if (r8 == 0 && r16 == 0) {
    err->code = -1;  // invalid argument
    err->msg = "expansion order too large for the particle-to-expansion schedule";
    return -1;
  }
  // diagonal constants (-1)^m (2m-1)!!
  std::vector<double> dk(p + 1);
  double dd = 1.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) dd *= -(2.0 * m - 1.0);
    dk[m] = dd;
  }
  RPY_HIP(hipMalloc(&tb->p2e_dk, sizeof(double) * dk.size()));
  RPY_HIP(hipMemcpy(tb->p2e_dk, dk.data(), sizeof(double) * dk.size(), hipMemcpyHostToDevice));
  tb->bytes += bytes + sizeof(double) * dk.size();
  return 0;
}

hipError_t run_p2m(const Launch& l, int nrc, const double* sF, Exp e) {
  const Built* B = l.B;
  if (B->nleaf == 0) return hipSuccess;
  switch (nrc) {
    case 1: k_leaf_q<1><<<B->nleaf, 256, 0, l.s>>>(B->leaf_ids, B->tree, B->sx, B->sy, B->sz, sF, B->n, e.Q); break;
    case 2: k_leaf_q<2><<<B->nleaf, 256, 0, l.s>>>(B->leaf_ids, B->tree, B->sx, B->sy, B->sz, sF, B->n, e.Q); break;
    case 4: k_leaf_q<4><<<B->nleaf, 256, 0, l.s>>>(B->leaf_ids, B->tree, B->sx, B->sy, B->sz, sF, B->n, e.Q); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t he = hipGetLastError();
  if (he != hipSuccess) return he;
  return launch_p2e_nd<false>(l, nrc, B->nleaf, B->leaf_ids, e.Q, e.M, nullptr);
}

hipError_t run_p2l(const Launch& l, int nrc, const double* sF, Exp e) {
  (void)sF;  // the charges come from the per-bead array written by run_p2m
  const Built* B = l.B;
  if (B->lists[LX].len == 0) return hipSuccess;
  if (!B->xwork && B->nxwork > 0) return hipErrorInvalidValue;
  if (B->nxred > 0 && !e.XP) return hipErrorInvalidValue;
  return launch_p2e_nd<true>(l, nrc, B->nxwork, nullptr, e.Q, e.L, e.XP);
}

}  // namespace rpy
