// Vector kernels and the small host eigensolver behind rpy_sqrt_matvec: the
// Brownian displacement y = D^{1/2} z of the Ermak-McCammon model is drawn
// from the Krylov space {D^k z} (arXiv:1711.02976, Sec. 1), which needs only
// matvecs with D.  The Lanczos recurrence lives in api.hip; these are its
// building blocks.
//
// Vectors are FP64, one per right-hand side, each of length L = 3n in the
// caller's [n][3] layout; a set of nrhs vectors is stored [nrhs][L], and the
// Lanczos basis [k][nrhs][L].
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "fmm.h"

namespace rpy {

namespace {
constexpr int KT = 256;  // threads per block of the vector kernels
}

// part[(r * kcap + j) * nchunk + c] = sum over chunk c of V_j[r][i] w[r][i],
// j < k.  Grid (nchunk, k, nrhs); each block walks its chunk with stride KT.
__global__ void __launch_bounds__(KT) k_mdot(const double* __restrict__ V, int64_t vstride, const double* __restrict__ w,
                                             int64_t L, int kcap, int nchunk, double* __restrict__ part) {
  const int c = blockIdx.x, j = blockIdx.y, r = blockIdx.z;
  const int64_t per = (L + nchunk - 1) / nchunk;
  const int64_t i0 = (int64_t)c * per, i1 = min(L, i0 + per);
  const double* v = V + (int64_t)j * vstride + (int64_t)r * L;
  const double* x = w + (int64_t)r * L;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += KT) s = fma(v[i], x[i], s);
  __shared__ double red[KT];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = KT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[((int64_t)r * kcap + j) * nchunk + c] = red[0];
}

// out[r * kcap + j] = sum of the nchunk partials, in chunk order.
__global__ void k_mdot_sum(const double* __restrict__ part, int k, int kcap, int nrhs, int nchunk,
                           double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * nrhs) return;
  const int r = t / k, j = t - r * k;
  const double* p = part + ((int64_t)r * kcap + j) * nchunk;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += p[c];
  out[r * kcap + j] = s;
}

// out[r][i] = s[r] * (a * w[r][i] + sgn * sum_{j<k} coef[r * kcap + j] V_j[r][i]).
// out may alias w (each element is read before it is written by the same
// thread).  Grid (ceil(L / KT) capped, nrhs).
__global__ void __launch_bounds__(KT) k_comb(const double* __restrict__ V, int64_t vstride, int k, int kcap,
                                             const double* __restrict__ coef, double sgn, const double* w, double a,
                                             const double* __restrict__ s, int64_t L, double* out) {
  const int r = blockIdx.y;
  const double* cr = coef + (int64_t)r * kcap;
  const double sr = s ? s[r] : 1.0;
  for (int64_t i = (int64_t)blockIdx.x * KT + threadIdx.x; i < L; i += (int64_t)gridDim.x * KT) {
    double acc = w ? a * w[(int64_t)r * L + i] : 0.0;
    for (int j = 0; j < k; ++j) acc = fma(sgn * cr[j], V[(int64_t)j * vstride + (int64_t)r * L + i], acc);
    out[(int64_t)r * L + i] = sr * acc;
  }
}

static int mdot_chunks(int64_t L) {
  const int64_t c = (L + 8 * KT - 1) / (8 * KT);
  return (int)std::max<int64_t>(1, std::min<int64_t>(c, 256));
}

int64_t krylov_part_doubles(int64_t L, int kcap, int nrhs) { return (int64_t)mdot_chunks(L) * kcap * nrhs; }

hipError_t krylov_mdot(const double* V, int64_t vstride, int k, const double* w, int64_t L, int nrhs, int kcap,
                       double* part, double* out, hipStream_t st) {
  if (k <= 0 || nrhs <= 0 || k > kcap) return hipErrorInvalidValue;
  const int nchunk = mdot_chunks(L);
  k_mdot<<<dim3(nchunk, k, nrhs), KT, 0, st>>>(V, vstride, w, L, kcap, nchunk, part);
  hipError_t he = hipGetLastError();
  if (he != hipSuccess) return he;
  const int t = k * nrhs;
  k_mdot_sum<<<(t + 127) / 128, 128, 0, st>>>(part, k, kcap, nrhs, nchunk, out);
  return hipGetLastError();
}

hipError_t krylov_comb(const double* V, int64_t vstride, int k, int kcap, const double* coef, double sgn,
                       const double* w, double a, const double* s, int64_t L, int nrhs, double* out, hipStream_t st) {
  if (nrhs <= 0 || k < 0 || k > kcap || nrhs > 65535) return hipErrorInvalidValue;
  const int64_t nb = std::min<int64_t>((L + KT - 1) / KT, 4096);
  k_comb<<<dim3((unsigned)std::max<int64_t>(nb, 1), nrhs), KT, 0, st>>>(V, vstride, k, kcap, coef, sgn, w, a, s, L,
                                                                       out);
  return hipGetLastError();
}

// Eigenvalues lam[m] and orthonormal eigenvectors Q (column q in Q[i * m + q])
// of the symmetric tridiagonal matrix with diagonal d[0..m) and
// off-diagonal e[0..m-1) (e[i] couples i and i + 1), by the implicit QL
// method: each sweep applies a Wilkinson-shifted QL step to the unreduced
// block [l, k] as a chain of plane rotations from the bottom up, and the
// rotations are accumulated into Q.  O(m^2) per eigenvalue.  This is the
// published implicit QL algorithm with implicit shifts of Bowdler, Martin,
// Reinsch and Wilkinson (Numer. Math. 11 (1968) 293-306; the tql2 procedure
// of the Handbook for Automatic Computation, Vol. II, and of EISPACK),
// written here from that description: Wilkinson shift from the trailing
// 2x2 block, bottom-up plane rotations, and a split wherever an
// off-diagonal element is negligible against its neighbouring diagonal.
void tridiag_eig(int m, const std::vector<double>& d, const std::vector<double>& e, std::vector<double>& lam,
                 std::vector<double>& Q) {
  lam.assign(d.begin(), d.begin() + m);
  std::vector<double> off(m, 0.0);
  for (int i = 0; i + 1 < m; ++i) off[i] = e[i];
  Q.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
  for (int l = 0; l < m; ++l) {
    for (int it = 0; it < 64; ++it) {
      // first negligible coupling at or below l: the block [l, k] is unreduced
      int k = l;
      for (; k + 1 < m; ++k) {
        const double dd = std::fabs(lam[k]) + std::fabs(lam[k + 1]);
        if (std::fabs(off[k]) <= 1e-16 * dd) break;
      }
      if (k == l) break;
      // Wilkinson shift from the leading 2x2 of the block
      double g = (lam[l + 1] - lam[l]) / (2.0 * off[l]);
      double r = std::hypot(g, 1.0);
      g = lam[k] - lam[l] + off[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = k - 1;
      bool split = false;
      for (; i >= l; --i) {
        const double f = s * off[i], b = c * off[i];
        r = std::hypot(f, g);
        off[i + 1] = r;
        if (r == 0.0) {  // the rotation underflowed: the block splits here
          lam[i + 1] -= p;
          off[k] = 0.0;
          split = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = lam[i + 1] - p;
        r = (lam[i] - g) * s + 2.0 * c * b;
        p = s * r;
        lam[i + 1] = g + p;
        g = c * r - b;
        for (int q = 0; q < m; ++q) {
          double* row = &Q[(size_t)q * m];
          const double t = row[i + 1];
          row[i + 1] = s * row[i] + c * t;
          row[i] = c * row[i] - s * t;
        }
      }
      if (split) continue;
      lam[l] -= p;
      off[l] = g;
      off[k] = 0.0;
    }
  }
}

}  // namespace rpy
