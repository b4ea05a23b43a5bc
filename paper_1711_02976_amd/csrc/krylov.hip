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
// of a symmetric m x m matrix A (row-major; destroyed), by cyclic Jacobi
// rotations until the off-diagonal part is negligible.
void sym_eig(int m, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& Q) {
  Q.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        const double v = A[(size_t)i * m + j] * A[(size_t)i * m + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[(size_t)p * m + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
        // rotation angle that zeroes A[p][q]: tan(2 phi) = 2 apq / (aqq - app)
        const double th = (aqq - app) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; ++k) {
          const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
          A[(size_t)k * m + p] = c * akp - s * akq;
          A[(size_t)k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {
          const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
          A[(size_t)p * m + k] = c * apk - s * aqk;
          A[(size_t)q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double qkp = Q[(size_t)k * m + p], qkq = Q[(size_t)k * m + q];
          Q[(size_t)k * m + p] = c * qkp - s * qkq;
          Q[(size_t)k * m + q] = s * qkp + c * qkq;
        }
      }
  }
  lam.resize(m);
  for (int i = 0; i < m; ++i) lam[i] = A[(size_t)i * m + i];
}

}  // namespace rpy
