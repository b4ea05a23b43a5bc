// Plan-time kernels: bounding cubes, Morton keys, stable LSD radix sort,
// level-synchronous adaptive octree and the U/V/W/X/O interaction lists.
//
// The octree follows the refinement rule of arXiv:1711.02976, Sec. 4.2 (a box
// is split while it holds more than `threshold` beads); the list
// definitions are those of the adaptive FMM the paper builds on (Sec. 1 and
// 3.2): U = adjacent leaves, V = well-separated children of the parent's
// colleagues, W = finer non-adjacent boxes whose parent is adjacent,
// X = transpose of W; O = non-adjacent leaves closer than 2a (overlap
// correction).  Every integer result is canonical: keys quantise with two
// correctly rounded FP64 operations, the sort is stable, boxes are numbered
// by (level, system, key) and every list is sorted by box id.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"

namespace rpy {

// ------------------------------------------------------------------ scan --
constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;

__global__ void __launch_bounds__(SCAN_T) k_scan_tile(const int* in, int* out, int64_t n, int* sums) {
  __shared__ int warp_tot[SCAN_T / 64];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    int t = v[i];
    v[i] = tot;
    tot += t;
  }
  // inclusive scan of per-thread totals within the wave
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = tot;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) warp_tot[w] = x;
  __syncthreads();
  int woff = 0;
  for (int i = 0; i < w; ++i) woff += warp_tot[i];
  int excl = woff + x - tot;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) out[base + i] = v[i] + excl;
  if (threadIdx.x == SCAN_T - 1 && sums) sums[blockIdx.x] = woff + x;
}

__global__ void k_scan_add(int* out, int64_t n, const int* sums) {
  int64_t i = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x;
  int add = sums[blockIdx.x];
  for (int k = 0; k < SCAN_ITEMS; ++k, i += SCAN_T)
    if (i < n) out[i] += add;
}

size_t scan_tmp_ints(int64_t n) {
  size_t t = 0;
  while (n > SCAN_TILE) {
    n = (n + SCAN_TILE - 1) / SCAN_TILE;
    t += n + 1;
  }
  return t + 1;
}

hipError_t scan_exclusive(const int* in, int* out, int64_t n, int* tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 1) {
    k_scan_tile<<<1, SCAN_T, 0, s>>>(in, out, n, nullptr);
    return hipGetLastError();
  }
  int* sums = tmp;
  k_scan_tile<<<(unsigned)nb, SCAN_T, 0, s>>>(in, out, n, sums);
  hipError_t e = scan_exclusive(sums, sums, nb, tmp + nb + 1, s);
  if (e != hipSuccess) return e;
  k_scan_add<<<(unsigned)nb, SCAN_T, 0, s>>>(out, n, sums);
  return hipGetLastError();
}

// --------------------------------------------------------- bounding cube --
constexpr int BB_T = 256;

// grid (nblk, nsys): per-system partial min/max of x, y, z.
__global__ void __launch_bounds__(BB_T) k_bbox_partial(const double* pos, const int* sys_begin, int nblk,
                                                       double* part) {
  int s = blockIdx.y;
  int64_t b0 = sys_begin[s], b1 = sys_begin[s + 1];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = b0 + (int64_t)blockIdx.x * BB_T + threadIdx.x; i < b1; i += (int64_t)nblk * BB_T)
    for (int k = 0; k < 3; ++k) {
      double v = pos[3 * i + k];
      mn[k] = fmin(mn[k], v);
      mx[k] = fmax(mx[k], v);
    }
  __shared__ double red[6][BB_T];
  for (int k = 0; k < 3; ++k) { red[k][threadIdx.x] = mn[k]; red[3 + k][threadIdx.x] = mx[k]; }
  __syncthreads();
  for (int w = BB_T / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[((int64_t)s * nblk + blockIdx.x) * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// one block per system: reduce partials, flag non-finite coordinates.  An
// empty system gets the unit cube at the origin.
__global__ void k_bbox_final(const double* part, int nblk, const int* sys_begin, double* out /*[nsys][6]*/,
                             int* bad) {
  int s = blockIdx.x;
  if (sys_begin[s] == sys_begin[s + 1]) {
    if (threadIdx.x < 6) out[s * 6 + threadIdx.x] = 0.0;
    return;
  }
  __shared__ double red[6][64];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int i = threadIdx.x; i < nblk; i += 64)
    for (int k = 0; k < 6; ++k) {
      double x = part[((int64_t)s * nblk + i) * 6 + k];
      v[k] = k < 3 ? fmin(v[k], x) : fmax(v[k], x);
    }
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 64; ++i)
      for (int k = 0; k < 6; ++k) v[k] = k < 3 ? fmin(v[k], red[k][i]) : fmax(v[k], red[k][i]);
    for (int k = 0; k < 6; ++k) {
      out[s * 6 + k] = v[k];
      if (!isfinite(v[k])) *bad = 1;
    }
  }
}

// Scans all coordinates for NaN/Inf (fmin/fmax drop NaN).
__global__ void k_check_finite(const double* pos, int64_t n3, int* bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(pos[i])) *bad = 1;
}

// ------------------------------------------------------------ Morton keys --
__device__ inline uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ inline int sys_of(const int* sys_begin, int nsys, int64_t i) {
  int lo = 0, hi = nsys;  // largest s with sys_begin[s] <= i
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (sys_begin[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void k_morton(const double* pos, int64_t n, const int* sys_begin, int nsys, const double* lo,
                         const double* side, uint64_t* keys, int* idx) {
#pragma clang fp contract(off)
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int s = nsys > 1 ? sys_of(sys_begin, nsys, i) : 0;
  const double scale = 2097152.0 / side[s];
  uint64_t key = 0;
  for (int k = 0; k < 3; ++k) {
    double d = __dsub_rn(pos[3 * i + k], lo[3 * s + k]);
    double q = floor(__dmul_rn(d, scale));
    uint32_t qi = q >= 2097151.0 ? 2097151u : (q <= 0.0 ? 0u : (uint32_t)q);
    key |= spread3(qi) << k;
  }
  keys[i] = key;
  idx[i] = (int)i;
}

// ------------------------------------------------------------- radix sort --
constexpr int RS_T = 256;
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = RS_T * RS_ROUNDS;

__device__ inline int rs_digit(uint64_t key, int val, int shift, const int* sys_begin, int nsys, int mode) {
  if (mode == 0) return (int)((key >> shift) & 0xffu);
  return (sys_of(sys_begin, nsys, val) >> shift) & 0xff;
}

__global__ void __launch_bounds__(RS_T) k_rs_hist(const uint64_t* keys, const int* vals, int64_t n, int shift,
                                                  int mode, const int* sys_begin, int nsys, int* hist, int nblk) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t e = base + r * RS_T + threadIdx.x;
    if (e < n) atomicAdd(&cnt[rs_digit(keys[e], vals[e], shift, sys_begin, nsys, mode)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(RS_T) k_rs_scatter(const uint64_t* kin, const int* vin, uint64_t* kout, int* vout,
                                                     int64_t n, int shift, int mode, const int* sys_begin, int nsys,
                                                     const int* offs, int nblk) {
  __shared__ int base[256];
  __shared__ int wcnt[RS_T / 64][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  base[threadIdx.x] = offs[(int64_t)threadIdx.x * nblk + blockIdx.x];
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t t0 = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    for (int k = 0; k < RS_T / 64; ++k) wcnt[k][threadIdx.x] = 0;
    __syncthreads();
    int64_t e = t0 + r * RS_T + threadIdx.x;
    bool valid = e < n;
    uint64_t key = valid ? kin[e] : 0;
    int val = valid ? vin[e] : 0;
    int d = valid ? rs_digit(key, val, shift, sys_begin, nsys, mode) : 0;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t m = __ballot(valid && ((d >> b) & 1));
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    int rank = __popcll(peers & below);
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = base[d] + rank;
      for (int k = 0; k < w; ++k) pos += wcnt[k][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int add = 0;
    for (int k = 0; k < RS_T / 64; ++k) add += wcnt[k][threadIdx.x];
    base[threadIdx.x] += add;
    __syncthreads();
  }
}

__global__ void k_gather_pos(const double* pos, const int* idx, int64_t n, double* sx, double* sy, double* sz) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int j = idx[i];
  sx[i] = pos[3 * (int64_t)j];
  sy[i] = pos[3 * (int64_t)j + 1];
  sz[i] = pos[3 * (int64_t)j + 2];
}

// ---------------------------------------------------------------- octree --
__device__ inline int child_digit(uint64_t key, int child_level) {
  return (int)((key >> (3 * (KBITS - child_level))) & 7u);
}

// first index in [lo, hi) whose child digit is >= o (digits are sorted).
__device__ inline int lower_digit(const uint64_t* keys, int lo, int hi, int lev, int o) {
  while (lo < hi) {
    int mid = lo + ((hi - lo) >> 1);
    if (child_digit(keys[mid], lev) < o) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void k_tree_roots(Tree t, const int* sys_begin, int nsys) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  t.level[s] = 0; t.sys[s] = s; t.ax[s] = 0; t.ay[s] = 0; t.az[s] = 0;
  t.begin[s] = sys_begin[s]; t.end[s] = sys_begin[s + 1];
  t.parent[s] = -1; t.child[s] = -1; t.nchild[s] = 0;
}

__global__ void k_tree_count(Tree t, const uint64_t* keys, int ls, int le, int lev, int leaf_size, int max_depth,
                             int* cnt) {
  int b = ls + blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= le) return;
  int c = 0;
  int b0 = t.begin[b], b1 = t.end[b];
  if (b1 - b0 > leaf_size && lev < max_depth) {
    int prev = b0;
    for (int o = 1; o <= 8; ++o) {
      int nxt = o < 8 ? lower_digit(keys, prev, b1, lev + 1, o) : b1;
      if (nxt > prev) ++c;
      prev = nxt;
    }
  }
  cnt[b - ls] = c;
}

__global__ void k_tree_write(Tree t, const uint64_t* keys, int ls, int le, int lev, const int* cnt, const int* off) {
  int b = ls + blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= le) return;
  int nc = cnt[b - ls];
  t.nchild[b] = nc;
  if (nc == 0) { t.child[b] = -1; return; }
  int cid = le + off[b - ls];
  t.child[b] = cid;
  int b0 = t.begin[b], b1 = t.end[b];
  int prev = b0;
  for (int o = 0; o < 8; ++o) {
    int nxt = o < 7 ? lower_digit(keys, prev, b1, lev + 1, o + 1) : b1;
    if (nxt > prev) {
      t.level[cid] = lev + 1; t.sys[cid] = t.sys[b];
      t.ax[cid] = 2 * t.ax[b] + (o & 1);
      t.ay[cid] = 2 * t.ay[b] + ((o >> 1) & 1);
      t.az[cid] = 2 * t.az[b] + ((o >> 2) & 1);
      t.begin[cid] = prev; t.end[cid] = nxt; t.parent[cid] = b;
      t.child[cid] = -1; t.nchild[cid] = 0;
      ++cid;
    }
    prev = nxt;
  }
}

__global__ void k_box_geometry(Tree t, const double* lo, const double* side) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= t.nbox) return;
  int s = t.sys[b];
  double h = ldexp(side[s], -t.level[b]);
  t.h[b] = h;
  t.cx[b] = lo[3 * s] + (t.ax[b] + 0.5) * h;
  t.cy[b] = lo[3 * s + 1] + (t.ay[b] + 0.5) * h;
  t.cz[b] = lo[3 * s + 2] + (t.az[b] + 0.5) * h;
}

// ------------------------------------------------------------ colleagues --
__global__ void k_colleagues(Tree t, int ls, int le, int* col) {
  int b = ls + blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= le) return;
  int* cb = col + (int64_t)b * NSLOT;
  for (int s = 0; s < NSLOT; ++s) cb[s] = -1;
  int P = t.parent[b];
  if (P < 0) { cb[13] = b; return; }
  const int* cp = col + (int64_t)P * NSLOT;
  for (int s = 0; s < NSLOT; ++s) {
    int Q = cp[s];
    if (Q < 0 || t.nchild[Q] == 0) continue;
    for (int C = t.child[Q]; C < t.child[Q] + t.nchild[Q]; ++C) {
      int dx = t.ax[C] - t.ax[b], dy = t.ay[C] - t.ay[b], dz = t.az[C] - t.az[b];
      if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1)
        cb[(dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)] = C;
    }
  }
}

// --------------------------------------------------------------- lists ----
__device__ inline bool adjacent(const Tree& t, int A, int B) {
  int la = t.level[A], lb = t.level[B];
  int L = la > lb ? la : lb;
  int sa = L - la, sb = L - lb;
  int64_t a0, a1, b0, b1;
  a0 = (int64_t)t.ax[A] << sa; a1 = ((int64_t)t.ax[A] + 1) << sa;
  b0 = (int64_t)t.ax[B] << sb; b1 = ((int64_t)t.ax[B] + 1) << sb;
  if (a0 > b1 || b0 > a1) return false;
  a0 = (int64_t)t.ay[A] << sa; a1 = ((int64_t)t.ay[A] + 1) << sa;
  b0 = (int64_t)t.ay[B] << sb; b1 = ((int64_t)t.ay[B] + 1) << sb;
  if (a0 > b1 || b0 > a1) return false;
  a0 = (int64_t)t.az[A] << sa; a1 = ((int64_t)t.az[A] + 1) << sa;
  b0 = (int64_t)t.az[B] << sb; b1 = ((int64_t)t.az[B] + 1) << sb;
  if (a0 > b1 || b0 > a1) return false;
  return true;
}

// Closest distance between the two cubes is below 2a: integer gaps at the
// finer level, threshold (2a)/(side 2^-L) in FP64 (no contraction).
__device__ inline bool near_2a(const Tree& t, int A, int B, const double* side, double a) {
#pragma clang fp contract(off)
  int la = t.level[A], lb = t.level[B];
  int L = la > lb ? la : lb;
  int sa = L - la, sb = L - lb;
  const int* ca[3] = {t.ax, t.ay, t.az};
  int64_t g2 = 0;
  for (int k = 0; k < 3; ++k) {
    int64_t a0 = (int64_t)ca[k][A] << sa, a1 = ((int64_t)ca[k][A] + 1) << sa;
    int64_t b0 = (int64_t)ca[k][B] << sb, b1 = ((int64_t)ca[k][B] + 1) << sb;
    int64_t g = 0;
    if (b0 > a1) g = b0 - a1;
    if (a0 > b1) g = a0 - b1;
    g2 += g * g;
  }
  double unit = ldexp(side[t.sys[A]], -L);
  double thr = __ddiv_rn(2.0 * a, unit);
  return (double)g2 < __dmul_rn(thr, thr);
}

struct Emit {
  int* dst;
  int n;
  __device__ inline void put(int c) {
    if (dst) dst[n] = c;
    ++n;
  }
};

// Shell sort (gaps 3h+1): O(n^1.5) for the long O lists of dense clusters.
__device__ inline void sort_segment(int* v, int n) {
  int h = 1;
  while (h < n / 3) h = 3 * h + 1;
  for (; h >= 1; h /= 3)
    for (int i = h; i < n; ++i) {
      int x = v[i], j = i - h;
      while (j >= 0 && v[j] > x) { v[j + h] = v[j]; j -= h; }
      v[j + h] = x;
    }
}

// mode 0: count into cnt[5][nbox]; mode 1: fill at off[L][b].
__global__ void k_lists(Tree t, const int* col, int nbox, int mode, int* cnt, List l0, List l1, List l2, List l3,
                        List l4, int want_o, const double* side, double a) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  List ls[5] = {l0, l1, l2, l3, l4};
  Emit e[5];
  for (int L = 0; L < 5; ++L) {
    e[L].n = 0;
    e[L].dst = mode ? ls[L].ent + ls[L].off[b] : nullptr;
  }
  const bool leaf = t.nchild[b] == 0;
  const int* cb = col + (int64_t)b * NSLOT;
  int stack[STACK];
  // V: children of the parent's colleagues not adjacent to b.
  int P = t.parent[b];
  if (P >= 0) {
    const int* cp = col + (int64_t)P * NSLOT;
    for (int s = 0; s < NSLOT; ++s) {
      int Q = cp[s];
      if (Q < 0 || t.nchild[Q] == 0) continue;
      for (int C = t.child[Q]; C < t.child[Q] + t.nchild[Q]; ++C)
        if (!adjacent(t, C, b)) e[LV].put(C);
    }
    // X: coarser leaf colleagues of b's ancestors, adjacent to b's parent but not to b.
    for (int A = P; A >= 0; A = t.parent[A]) {
      const int* ca = col + (int64_t)A * NSLOT;
      for (int s = 0; s < NSLOT; ++s) {
        int Q = ca[s];
        if (Q < 0 || Q == A || t.nchild[Q] != 0) continue;
        if (adjacent(t, Q, P) && !adjacent(t, Q, b)) e[LX].put(Q);
      }
    }
  }
  if (leaf) {
    // U, same level (b itself included) and finer; W from the same descent.
    for (int s = 0; s < NSLOT; ++s) {
      int Q = cb[s];
      if (Q < 0) continue;
      if (t.nchild[Q] == 0) { e[LU].put(Q); continue; }
      int sp = 0;
      stack[sp++] = Q;
      while (sp > 0) {
        int D = stack[--sp];
        for (int C = t.child[D]; C < t.child[D] + t.nchild[D]; ++C) {
          if (adjacent(t, C, b)) {
            if (t.nchild[C] == 0) e[LU].put(C);
            else if (sp < STACK) stack[sp++] = C;
          } else {
            e[LW].put(C);
          }
        }
      }
    }
    // U, coarser: leaf colleagues of ancestors that touch b.
    for (int A = P; A >= 0; A = t.parent[A]) {
      const int* ca = col + (int64_t)A * NSLOT;
      for (int s = 0; s < NSLOT; ++s) {
        int Q = ca[s];
        if (Q < 0 || Q == A || t.nchild[Q] != 0) continue;
        if (adjacent(t, Q, b)) e[LU].put(Q);
      }
    }
    // O: leaves of the same system closer than 2a but not adjacent.
    if (want_o) {
      int root = t.sys[b];
      int sp = 0;
      stack[sp++] = root;
      while (sp > 0) {
        int D = stack[--sp];
        if (!near_2a(t, D, b, side, a)) continue;
        if (t.nchild[D] == 0) {
          if (!adjacent(t, D, b)) e[LO].put(D);
          continue;
        }
        for (int C = t.child[D] + t.nchild[D] - 1; C >= t.child[D]; --C)
          if (sp < STACK) stack[sp++] = C;
      }
    }
  }
  if (mode == 0) {
    for (int L = 0; L < 5; ++L) cnt[(int64_t)L * nbox + b] = e[L].n;
  } else {
    for (int L = 0; L < 5; ++L) sort_segment(e[L].dst, e[L].n);
  }
}

__global__ void k_leaf_flags(Tree t, int* flag) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < t.nbox) flag[b] = t.nchild[b] == 0 ? 1 : 0;
}

__global__ void k_leaf_compact(Tree t, const int* off, int* ids) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < t.nbox && t.nchild[b] == 0) ids[off[b]] = b;
}

hipError_t radix_sort(uint64_t** keys, int** vals, uint64_t* kalt, int* valt, int64_t n, int key_passes,
                      int sys_passes, const int* sys_begin, int nsys, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t rblk = (n + RS_TILE - 1) / RS_TILE;
  int64_t hn = 256 * rblk;
  int *hist = nullptr, *stmp = nullptr;
  hipError_t e = hipMalloc(&hist, sizeof(int) * hn);
  if (e == hipSuccess) e = hipMalloc(&stmp, sizeof(int) * scan_tmp_ints(hn));
  uint64_t *k0 = *keys, *k1 = kalt;
  int *v0 = *vals, *v1 = valt;
  for (int pass = 0; e == hipSuccess && pass < key_passes + sys_passes; ++pass) {
    int mode = pass < key_passes ? 0 : 1;
    int shift = pass < key_passes ? 8 * pass : 8 * (pass - key_passes);
    k_rs_hist<<<(unsigned)rblk, RS_T, 0, s>>>(k0, v0, n, shift, mode, sys_begin, nsys, hist, (int)rblk);
    e = hipGetLastError();
    if (e == hipSuccess) e = scan_exclusive(hist, hist, hn, stmp, s);
    if (e == hipSuccess) {
      k_rs_scatter<<<(unsigned)rblk, RS_T, 0, s>>>(k0, v0, k1, v1, n, shift, mode, sys_begin, nsys, hist,
                                                   (int)rblk);
      e = hipGetLastError();
    }
    std::swap(k0, k1);
    std::swap(v0, v1);
  }
  if (hipStreamSynchronize(s) != hipSuccess && e == hipSuccess) e = hipErrorUnknown;
  if (hist) (void)hipFree(hist);
  if (stmp) (void)hipFree(stmp);
  // result in k0/v0; hand the other buffers back through kalt/valt's owners
  if (k0 != *keys) {
    // the sorted data lives in the alternate buffers: copy back
    if (e == hipSuccess) e = hipMemcpyAsync(*keys, k0, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(*vals, v0, sizeof(int) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  return e;
}

// ---------------------------------------------------------------- driver --
namespace {

template <class T>
int dalloc(T** p, int64_t count, Built* out, Error* err) {
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
  if (e != hipSuccess) {
    err->code = -3;
    err->msg = "hipMalloc failed (" + std::to_string(sizeof(T) * count) + " bytes)";
    *p = nullptr;
    return -3;
  }
  out->bytes += sizeof(T) * count;
  return 0;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int grow_tree(Built* B, int need, hipStream_t s, Error* err) {
  if (need <= B->cap) return 0;
  int ncap = std::max(need, B->cap * 2);
  Tree& t = B->tree;
  int* fields_old[10] = {t.level, t.sys, t.ax, t.ay, t.az, t.begin, t.end, t.parent, t.child, t.nchild};
  int* fields_new[10];
  for (int f = 0; f < 10; ++f) {
    if (dalloc(&fields_new[f], ncap, B, err)) return -3;
    if (fields_old[f])
      RPY_HIP(hipMemcpyAsync(fields_new[f], fields_old[f], sizeof(int) * B->cap, hipMemcpyDeviceToDevice, s));
  }
  RPY_HIP(hipStreamSynchronize(s));
  for (int f = 0; f < 10; ++f) {
    if (fields_old[f]) {
      RPY_HIP(hipFree(fields_old[f]));
      B->bytes -= sizeof(int) * B->cap;
    }
  }
  t.level = fields_new[0]; t.sys = fields_new[1]; t.ax = fields_new[2]; t.ay = fields_new[3];
  t.az = fields_new[4]; t.begin = fields_new[5]; t.end = fields_new[6]; t.parent = fields_new[7];
  t.child = fields_new[8]; t.nchild = fields_new[9];
  B->cap = ncap;
  return 0;
}

}  // namespace

void retire_built(Built* b, Spare* spare) {
  if (!b) return;
  if (spare && spare->n < 0 && b->keys && b->perm && b->sx && b->sy && b->sz) {
    spare->n = b->n;
    spare->keys = b->keys;
    spare->perm = b->perm;
    spare->sx = b->sx;
    spare->sy = b->sy;
    spare->sz = b->sz;
    b->keys = nullptr;
    b->perm = nullptr;
    b->sx = b->sy = b->sz = nullptr;
  }
  free_built(b);
}

void free_spare(Spare* spare) {
  if (!spare) return;
  void* ps[] = {spare->keys, spare->perm, spare->sx, spare->sy, spare->sz};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  *spare = Spare{};
}

void free_built(Built* b) {
  if (!b) return;
  void* ps[] = {b->keys, b->perm, b->sx, b->sy, b->sz, b->d_lo, b->d_side, b->d_sys_begin,
                b->tree.level, b->tree.sys, b->tree.ax, b->tree.ay, b->tree.az, b->tree.begin,
                b->tree.end, b->tree.parent, b->tree.child, b->tree.nchild, b->tree.cx, b->tree.cy,
                b->tree.cz, b->tree.h, b->colleague, b->leaf_ids, b->m2l_map, b->xwork, b->xchunks, b->xred};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  for (auto& L : b->lists) {
    if (L.off) (void)hipFree(L.off);
    if (L.ent) (void)hipFree(L.ent);
  }
  *b = Built{};
}

int build_tree(const BuildArgs& A, Built* B, Error* err) {
  hipStream_t s = A.stream;
  const int64_t n = A.n;
  const int nsys = A.nsys;
  B->n = n;
  B->nsys = nsys;
  std::vector<int> sb(nsys + 1);
  for (int i = 0; i <= nsys; ++i) sb[i] = (int)A.sys_begin_h[i];
  if (dalloc(&B->d_sys_begin, nsys + 1, B, err)) return -3;
  RPY_HIP(hipMemcpy(B->d_sys_begin, sb.data(), sizeof(int) * (nsys + 1), hipMemcpyHostToDevice));

  if (A.presorted) {
    // Same beads and systems as an earlier tree: its cubes, keys and sorted
    // order do not depend on the leaf size, so they are copied, not rebuilt.
    const Built* S = A.presorted;
    if (S->n != n || S->nsys != nsys) {
      err->code = -1;
      err->msg = "internal: presorted tree of other beads";
      return -1;
    }
    B->lo = S->lo;
    B->side = S->side;
    Spare* sp = A.spare;
    if (sp && sp->n == n) {
      B->keys = sp->keys;
      B->perm = sp->perm;
      B->sx = sp->sx;
      B->sy = sp->sy;
      B->sz = sp->sz;
      B->bytes += (int64_t)std::max<int64_t>(n, 1) * (sizeof(uint64_t) + sizeof(int) + 3 * sizeof(double));
      *sp = Spare{};
    } else if (dalloc(&B->keys, n, B, err) || dalloc(&B->perm, n, B, err) || dalloc(&B->sx, n, B, err) ||
               dalloc(&B->sy, n, B, err) || dalloc(&B->sz, n, B, err)) {
      return -3;
    }
    if (dalloc(&B->d_lo, 3 * nsys, B, err) || dalloc(&B->d_side, nsys, B, err)) return -3;
    RPY_HIP(hipMemcpyAsync(B->d_lo, S->d_lo, sizeof(double) * 3 * nsys, hipMemcpyDeviceToDevice, s));
    RPY_HIP(hipMemcpyAsync(B->d_side, S->d_side, sizeof(double) * nsys, hipMemcpyDeviceToDevice, s));
    if (n > 0) {
      RPY_HIP(hipMemcpyAsync(B->keys, S->keys, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
      RPY_HIP(hipMemcpyAsync(B->perm, S->perm, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
      RPY_HIP(hipMemcpyAsync(B->sx, S->sx, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      RPY_HIP(hipMemcpyAsync(B->sy, S->sy, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      RPY_HIP(hipMemcpyAsync(B->sz, S->sz, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
  } else {
    // Bounding cubes and the non-finite check.
    int nblk = 64;
    double* part = nullptr;
    double* bb = nullptr;
    int* bad = nullptr;
    if (dalloc(&part, (int64_t)nsys * nblk * 6, B, err)) return -3;
    if (dalloc(&bb, nsys * 6, B, err)) return -3;
    if (dalloc(&bad, 1, B, err)) return -3;
    RPY_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    // the bead passes (bounding cubes, keys, sort, gather) are timed with
    // events for the plan statistics
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    for (hipEvent_t& e : ev)
      if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    auto rec = [&](int i) {
      if (ev[i]) (void)hipEventRecord(ev[i], s);
    };
    auto drop = [&]() {
      for (hipEvent_t& e : ev)
        if (e) (void)hipEventDestroy(e);
    };
    rec(0);
    k_bbox_partial<<<dim3(nblk, nsys), BB_T, 0, s>>>(A.pos, B->d_sys_begin, nblk, part);
    k_bbox_final<<<nsys, 64, 0, s>>>(part, nblk, B->d_sys_begin, bb, bad);
    k_check_finite<<<1024, 256, 0, s>>>(A.pos, 3 * n, bad);
    rec(1);
    RPY_HIP(hipGetLastError());
    std::vector<double> hbb(nsys * 6);
    int hbad = 0;
    RPY_HIP(hipMemcpyAsync(hbb.data(), bb, sizeof(double) * nsys * 6, hipMemcpyDeviceToHost, s));
    RPY_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    RPY_HIP(hipStreamSynchronize(s));
    (void)hipFree(part); (void)hipFree(bb); (void)hipFree(bad);
    B->bytes -= sizeof(double) * ((int64_t)nsys * nblk * 6 + nsys * 6) + sizeof(int);
    if (hbad) {
      drop();
      err->code = -2;
      err->msg = "a position is NaN or infinite";
      return -2;
    }
    B->lo.assign(3 * nsys, 0.0);
    B->side.assign(nsys, 1.0);
    for (int k = 0; k < nsys; ++k) {
      double sd = 0.0;
      for (int d = 0; d < 3; ++d) {
        B->lo[3 * k + d] = hbb[6 * k + d];
        double ext = hbb[6 * k + 3 + d] - hbb[6 * k + d];
        if (ext > sd) sd = ext;
      }
      B->side[k] = sd == 0.0 ? 1.0 : sd;
    }
    if (dalloc(&B->d_lo, 3 * nsys, B, err) || dalloc(&B->d_side, nsys, B, err)) return -3;
    RPY_HIP(hipMemcpyAsync(B->d_lo, B->lo.data(), sizeof(double) * 3 * nsys, hipMemcpyHostToDevice, s));
    RPY_HIP(hipMemcpyAsync(B->d_side, B->side.data(), sizeof(double) * nsys, hipMemcpyHostToDevice, s));

    // Morton keys and the stable sort by (key, caller index) [, system].
    uint64_t *k0 = nullptr, *k1 = nullptr;
    int *v0 = nullptr, *v1 = nullptr;
    if (dalloc(&k0, n, B, err) || dalloc(&k1, n, B, err) || dalloc(&v0, n, B, err) || dalloc(&v1, n, B, err)) {
      drop();
      return -3;
    }
    rec(2);
    if (n > 0) k_morton<<<nblocks(n, 256), 256, 0, s>>>(A.pos, n, B->d_sys_begin, nsys, B->d_lo, B->d_side, k0, v0);
    RPY_HIP(hipGetLastError());
    int npass_sys = nsys > 1 ? (nsys > 256 ? 2 : 1) : 0;
    B->sort_passes = 8 + npass_sys;
    RPY_HIP(radix_sort(&k0, &v0, k1, v1, n, 8, npass_sys, B->d_sys_begin, nsys, s));
    (void)hipFree(k1); (void)hipFree(v1);
    B->bytes -= (sizeof(uint64_t) + sizeof(int)) * std::max<int64_t>(n, 1);
    B->keys = k0;
    B->perm = v0;
    if (dalloc(&B->sx, n, B, err) || dalloc(&B->sy, n, B, err) || dalloc(&B->sz, n, B, err)) {
      drop();
      return -3;
    }
    if (n > 0) k_gather_pos<<<nblocks(n, 256), 256, 0, s>>>(A.pos, v0, n, B->sx, B->sy, B->sz);
    rec(3);
    RPY_HIP(hipGetLastError());
    if (ev[0] && ev[1] && ev[2] && ev[3] && hipEventSynchronize(ev[3]) == hipSuccess) {
      float t0 = 0.f, t1 = 0.f;
      if (hipEventElapsedTime(&t0, ev[0], ev[1]) == hipSuccess && hipEventElapsedTime(&t1, ev[2], ev[3]) == hipSuccess)
        B->bead_pass_ms = (double)t0 + (double)t1;
    }
    drop();
  }

  // Octree, level by level.
  int cap0 = (int)std::max<int64_t>(1024, 4 * (n / std::max(A.leaf_size, 1)) + 16 * nsys);
  if (grow_tree(B, cap0, s, err)) return err->code;
  Tree& t = B->tree;
  k_tree_roots<<<nblocks(nsys, 64), 64, 0, s>>>(t, B->d_sys_begin, nsys);
  RPY_HIP(hipGetLastError());
  B->level_start.assign(1, 0);
  B->level_start.push_back(nsys);
  int* cnt = nullptr;
  int* off = nullptr;
  int* tmp = nullptr;
  int64_t ccap = 0;
  int lev = 0;
  for (;;) {
    int ls = B->level_start[lev], le = B->level_start[lev + 1];
    int nb = le - ls;
    if (nb > ccap) {
      if (cnt) { (void)hipFree(cnt); (void)hipFree(off); (void)hipFree(tmp); }
      ccap = std::max<int64_t>(nb, 2 * ccap);
      if (dalloc(&cnt, ccap, B, err) || dalloc(&off, ccap, B, err) ||
          dalloc(&tmp, (int64_t)scan_tmp_ints(ccap), B, err))
        return -3;
    }
    k_tree_count<<<nblocks(nb, 128), 128, 0, s>>>(t, B->keys, ls, le, lev, A.leaf_size, A.max_depth, cnt);
    RPY_HIP(hipGetLastError());
    RPY_HIP(scan_exclusive(cnt, off, nb, tmp, s));
    int last[2] = {0, 0};
    RPY_HIP(hipMemcpyAsync(&last[0], off + nb - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    RPY_HIP(hipMemcpyAsync(&last[1], cnt + nb - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    RPY_HIP(hipStreamSynchronize(s));
    int nnext = last[0] + last[1];
    if (grow_tree(B, le + nnext, s, err)) return err->code;
    k_tree_write<<<nblocks(nb, 128), 128, 0, s>>>(t, B->keys, ls, le, lev, cnt, off);
    RPY_HIP(hipGetLastError());
    if (nnext == 0) break;
    B->level_start.push_back(le + nnext);
    ++lev;
  }
  (void)hipFree(cnt); (void)hipFree(off); (void)hipFree(tmp);
  B->bytes -= sizeof(int) * (2 * ccap + scan_tmp_ints(ccap));
  B->depth = (int)B->level_start.size() - 2;
  t.nbox = B->level_start.back();
  const int nbox = t.nbox;
  if (dalloc(&t.cx, nbox, B, err) || dalloc(&t.cy, nbox, B, err) || dalloc(&t.cz, nbox, B, err) ||
      dalloc(&t.h, nbox, B, err))
    return -3;
  k_box_geometry<<<nblocks(nbox, 128), 128, 0, s>>>(t, B->d_lo, B->d_side);
  RPY_HIP(hipGetLastError());

  // Colleagues, level by level.
  if (dalloc(&B->colleague, (int64_t)nbox * NSLOT, B, err)) return -3;
  for (int l = 0; l <= B->depth; ++l) {
    int ls = B->level_start[l], le = B->level_start[l + 1];
    k_colleagues<<<nblocks(le - ls, 128), 128, 0, s>>>(t, ls, le, B->colleague);
    RPY_HIP(hipGetLastError());
  }

  // Leaves.
  int* flag = nullptr;
  int* loff = nullptr;
  int* ltmp = nullptr;
  if (dalloc(&flag, nbox, B, err) || dalloc(&loff, nbox, B, err) ||
      dalloc(&ltmp, (int64_t)scan_tmp_ints(nbox), B, err))
    return -3;
  k_leaf_flags<<<nblocks(nbox, 256), 256, 0, s>>>(t, flag);
  RPY_HIP(scan_exclusive(flag, loff, nbox, ltmp, s));
  int lastf[2];
  RPY_HIP(hipMemcpyAsync(&lastf[0], loff + nbox - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  RPY_HIP(hipMemcpyAsync(&lastf[1], flag + nbox - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  RPY_HIP(hipStreamSynchronize(s));
  B->nleaf = lastf[0] + lastf[1];
  if (dalloc(&B->leaf_ids, B->nleaf, B, err)) return -3;
  k_leaf_compact<<<nblocks(nbox, 256), 256, 0, s>>>(t, loff, B->leaf_ids);
  RPY_HIP(hipGetLastError());
  (void)hipFree(flag); (void)hipFree(loff); (void)hipFree(ltmp);
  B->bytes -= sizeof(int) * (2 * (int64_t)nbox + scan_tmp_ints(nbox));

  // Interaction lists: count, scan, fill (sorted by box id).  The O list is
  // empty, and skipped, when every leaf side is at least 2a.
  int want_o = 0;
  for (int k = 0; k < nsys; ++k)
    if (!A.skip_o && ldexp(B->side[k], -B->depth) < 2.0 * A.a) want_o = 1;
  int* lcnt = nullptr;
  int* lt = nullptr;
  if (dalloc(&lcnt, 5 * (int64_t)nbox, B, err) || dalloc(&lt, (int64_t)scan_tmp_ints(nbox + 1), B, err)) return -3;
  List none[5] = {};
  k_lists<<<nblocks(nbox, 64), 64, 0, s>>>(t, B->colleague, nbox, 0, lcnt, none[0], none[1], none[2], none[3],
                                           none[4], want_o, B->d_side, A.a);
  RPY_HIP(hipGetLastError());
  // The five scans, then one read-back of their last offsets and counts.
  // Copies to or from the host arrays below are drained before any return.
  int lastc[5][2];
  int tot32[5];
  hipError_t le = hipSuccess;
  int lrc = 0;
  for (int L = 0; L < 5 && le == hipSuccess; ++L) {
    if ((lrc = dalloc(&B->lists[L].off, nbox + 1, B, err)) != 0) break;
    le = scan_exclusive(lcnt + (int64_t)L * nbox, B->lists[L].off, nbox, lt, s);
    if (le == hipSuccess)
      le = hipMemcpyAsync(&lastc[L][0], B->lists[L].off + nbox - 1, sizeof(int), hipMemcpyDeviceToHost, s);
    if (le == hipSuccess)
      le = hipMemcpyAsync(&lastc[L][1], lcnt + (int64_t)L * nbox + nbox - 1, sizeof(int), hipMemcpyDeviceToHost, s);
  }
  hipError_t se = hipStreamSynchronize(s);
  if (lrc) return lrc;
  RPY_HIP(le);
  RPY_HIP(se);
  for (int L = 0; L < 5; ++L) {
    const int64_t total = (int64_t)lastc[L][0] + lastc[L][1];
    B->lists[L].len = total;
    tot32[L] = (int)total;
    if (dalloc(&B->lists[L].ent, total, B, err)) return -3;
  }
  for (int L = 0; L < 5 && le == hipSuccess; ++L)
    le = hipMemcpyAsync(B->lists[L].off + nbox, &tot32[L], sizeof(int), hipMemcpyHostToDevice, s);
  se = hipStreamSynchronize(s);
  RPY_HIP(le);
  RPY_HIP(se);
  k_lists<<<nblocks(nbox, 64), 64, 0, s>>>(t, B->colleague, nbox, 1, lcnt, B->lists[0], B->lists[1], B->lists[2],
                                           B->lists[3], B->lists[4], want_o, B->d_side, A.a);
  RPY_HIP(hipGetLastError());
  RPY_HIP(hipStreamSynchronize(s));
  (void)hipFree(lcnt); (void)hipFree(lt);
  B->bytes -= sizeof(int) * (5 * (int64_t)nbox + scan_tmp_ints(nbox + 1));
  return 0;
}

}  // namespace rpy
