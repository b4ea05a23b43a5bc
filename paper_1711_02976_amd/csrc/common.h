// Internal declarations shared by the HIP sources of librpyfmm (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace rpy {

constexpr int KBITS = 21;            // quantisation bits per axis (63-bit Morton key)
constexpr int NSLOT = 27;            // colleague slots: offsets in {-1,0,1}^3
constexpr int MAX_ORDER = 27;        // (p+1)(p+2)/2 <= 406 coefficients per expansion
constexpr int MAX_ORDER_MULTI = 21;  // highest order at which a pass carries 2 or 4 right-hand sides
constexpr int STACK = 192;           // private DFS stack of the list kernels

__host__ __device__ constexpr int tri(int n) { return n * (n + 1) / 2; }
__host__ __device__ constexpr int ncoef(int p) { return (p + 1) * (p + 2) / 2; }

// Blocks are dealt to the 8 XCDs round-robin (block i to XCD i mod 8), each
// with its own L2.  Work items in leaf (Morton) order share most of their
// inputs with their neighbours, so items are dealt in chunks of XCD_CHUNK
// consecutive ones: XCD x takes chunks x, x + 8, x + 16, ... (its k-th block
// the item (8 (k / XCD_CHUNK) + x) XCD_CHUNK + k mod XCD_CHUNK), which keeps
// neighbouring items in one L2 and, chunk by chunk, the XCDs' work even when
// it varies along the item order (clustered beads).  Blocks past the last
// whole round of 8 chunks take their own index.  A permutation of 0 .. G - 1.
constexpr int XCD_CHUNK = 128;
__device__ inline int xcd_run(int i, int G) {
  const int full = G / (8 * XCD_CHUNK) * (8 * XCD_CHUNK);
  if (i >= full) return i;
  const int x = i & 7, k = i >> 3;
  return (8 * (k / XCD_CHUNK) + x) * XCD_CHUNK + k % XCD_CHUNK;
}

// Device view of the octree.  Boxes are numbered by (level, system, Morton
// key); begin/end index the sorted bead order.
struct Tree {
  int nbox;
  int* level;
  int* sys;
  int* ax;
  int* ay;
  int* az;
  int* begin;
  int* end;
  int* parent;
  int* child;    // first child, -1 for a leaf
  int* nchild;
  double* cx;    // centre
  double* cy;
  double* cz;
  double* h;     // side
};

// CSR list: entries of box b are ent[off[b] .. off[b+1]).
struct List {
  int* off;
  int* ent;
  int64_t len;
};

enum { LU = 0, LV = 1, LW = 2, LX = 3, LO = 4 };

struct Error {
  int code;
  std::string msg;
};

// ---- scan (exclusive prefix sum of int32) -------------------------------
// Scans n ints from `in` to `out` (may alias) on stream; returns 0 or a HIP
// error code.  Uses `tmp` scratch of scan_tmp_ints(n) ints.
size_t scan_tmp_ints(int64_t n);
hipError_t scan_exclusive(const int* in, int* out, int64_t n, int* tmp, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by 8-bit digits: key_passes
// digits of the key (least significant first), then sys_passes digits of
// the system index of each value (for concatenated systems).  The result is
// left in (*keys, *vals); kalt/valt are scratch of the same size.
hipError_t radix_sort(uint64_t** keys, int** vals, uint64_t* kalt, int* valt, int64_t n, int key_passes,
                      int sys_passes, const int* sys_begin, int nsys, hipStream_t s);

// ---- tree build (tree.hip) ---------------------------------------------
// The bead-sized arrays of a discarded trial tree (n entries each), kept for
// the next trial tree of the same beads instead of being freed.
struct Spare {
  int64_t n = -1;  // -1: empty
  uint64_t* keys = nullptr;
  int* perm = nullptr;
  double *sx = nullptr, *sy = nullptr, *sz = nullptr;
};

struct BuildArgs {
  int64_t n;
  int nsys;
  const int64_t* sys_begin_h;   // host [nsys+1]
  const double* pos;            // device [n][3], caller order
  int leaf_size;
  int max_depth;
  double a;
  hipStream_t stream;
  bool skip_o = false;          // leave the O list empty (trial trees of the leaf-size search)
  const struct Built* presorted = nullptr;  // a tree of the same beads: copy its cubes and sort
  Spare* spare = nullptr;                   // with presorted: bead arrays to reuse, if any
};

// Everything rpy_plan builds on the device.  Owned buffers are released by
// free_built().
struct Built {
  // beads in tree order
  int64_t n = 0;
  uint64_t* keys = nullptr;
  int* perm = nullptr;        // tree order -> caller index
  double* sx = nullptr;       // sorted positions, SoA
  double* sy = nullptr;
  double* sz = nullptr;
  // systems
  int nsys = 0;
  std::vector<double> lo;      // [nsys][3]
  std::vector<double> side;    // [nsys]
  double* d_lo = nullptr;      // device copies
  double* d_side = nullptr;
  int* d_sys_begin = nullptr;  // [nsys+1]
  // tree
  Tree tree{};
  int cap = 0;
  std::vector<int> level_start;  // boxes of level l are [level_start[l], level_start[l+1])
  int depth = 0;
  int* colleague = nullptr;     // [nbox][27]
  int nleaf = 0;
  int* leaf_ids = nullptr;      // [nleaf]
  List lists[5]{};
  // block -> target box of the rotation M->L (make_m2l_map), -1: no box;
  // blocks [m2l_part[0], m2l_part[1]) take the deepest level's boxes, whose
  // sources need only S->M, blocks [m2l_part[1], m2l_part[2]) the others
  int* m2l_map = nullptr;
  int m2l_part[3] = {0, 0, 0};
  // S->L work items (make_p2l_work): (box, first X entry, end X entry,
  // 1 + partial-sum slot or 0) and the range of 64-bead chunks taken from
  // each entry; a box split over several items has one reduction entry
  // (box, first slot, slot count) in xred
  int4* xwork = nullptr;
  int2* xchunks = nullptr;
  int4* xred = nullptr;
  int nxwork = 0;
  int nxshared = 0;   // partial-sum slots (items whose box is split)
  int nxred = 0;      // boxes split over several items
  // bead passes of the build (bounding cubes, keys, sort, gather): GPU time
  // and radix-sort passes; 0 for a tree that copied them from another
  double bead_pass_ms = 0.0;
  int sort_passes = 0;
  int64_t bytes = 0;
};

int build_tree(const BuildArgs& a, Built* out, Error* err);
void free_built(Built* b);
// Moves b's bead arrays into an empty spare (else leaves them in b); then
// frees what is left of b.
void retire_built(Built* b, Spare* spare);
void free_spare(Spare* spare);

}  // namespace rpy

#define RPY_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      if (err) {                                                                   \
        err->code = -4;                                                            \
        err->msg = std::string(#expr) + ": " + hipGetErrorString(e_);              \
      }                                                                            \
      return -4;                                                                   \
    }                                                                              \
  } while (0)
