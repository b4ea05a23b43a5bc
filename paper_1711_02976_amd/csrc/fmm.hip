// Far-field kernels of the four-Laplace FMM (arXiv:1711.02976, Sec. 2):
// S->M, M->M, M->L, S->L, L->L and the target evaluation that assembles
// eq. (2.8) from the local expansion (L->T) and the W-list multipoles (M->T).
//
// Densities per right-hand side: F_x, F_y, F_z (the charges of L1..L3) and the
// fourth charge F.(r - c) centred on the box that owns the expansion
// (an exact rewriting of L4 = sum F.r_j/|r_i - r_j| that keeps every term
// O(box size)); whenever an expansion moves to a new centre its fourth
// density is re-centred by E4 += (c_old - c_new).(E1, E2, E3).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "fmm.h"

namespace rpy {

namespace {

constexpr double PI = 3.14159265358979323846;

__host__ __device__ inline int fidx(int n, int m) { return n * n + n + m; }  // full layout, |m| <= n

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cmulc(double2 a, double2 b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
__device__ inline void cfmac(double2& acc, double2 a, double2 b) {  // acc += a * conj(b)
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.y, b.x, fma(-a.x, b.y, acc.y));
}

// Coefficient C_n^m of a real-symmetric set stored for m >= 0 (C^{-m} =
// (-1)^m conj(C^m)); zero outside 0 <= n <= nmax, |m| <= n.
__device__ inline double2 getc(const double2* C, int n, int m, int nmax) {
  if (n < 0 || n > nmax || m > n || m < -n) return make_double2(0.0, 0.0);
  if (m >= 0) return C[tri(n) + m];
  double2 v = C[tri(n) - m];
  return (m & 1) ? make_double2(-v.x, v.y) : make_double2(v.x, -v.y);
}



inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ------------------------------------------------------------ host tables --
void host_regular(double x, double y, double z, int p, std::vector<double2>& out) {
  // full layout, all |mu| <= j
  out.assign((p + 1) * (p + 1), make_double2(0, 0));
  double r2 = x * x + y * y + z * z;
  std::vector<double2> col(ncoef(p));
  for (int m = 0; m <= p; ++m) {
    double2 rmm = make_double2(1, 0);
    for (int k = 1; k <= m; ++k) {
      double f = -0.5 / k;
      rmm = make_double2(f * (x * rmm.x - y * rmm.y), f * (x * rmm.y + y * rmm.x));
    }
    col[tri(m) + m] = rmm;
    if (m + 1 <= p) col[tri(m + 1) + m] = make_double2(z * rmm.x, z * rmm.y);
    for (int n = m + 2; n <= p; ++n) {
      double inv = 1.0 / ((double)(n + m) * (n - m));
      double2 a = col[tri(n - 1) + m], b = col[tri(n - 2) + m];
      col[tri(n) + m] = make_double2(((2 * n - 1) * z * a.x - r2 * b.x) * inv, ((2 * n - 1) * z * a.y - r2 * b.y) * inv);
    }
  }
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m <= n; ++m) {
      double2 v = col[tri(n) + m];
      out[fidx(n, m)] = v;
      out[fidx(n, -m)] = (m & 1) ? make_double2(-v.x, v.y) : make_double2(v.x, -v.y);
    }
}

void host_irregular(double x, double y, double z, int p, std::vector<double2>& out) {
  out.assign((p + 1) * (p + 1), make_double2(0, 0));
  double r2 = x * x + y * y + z * z, ir2 = 1.0 / r2;
  std::vector<double2> col(ncoef(p));
  for (int m = 0; m <= p; ++m) {
    double2 imm = make_double2(std::sqrt(ir2), 0);
    for (int k = 1; k <= m; ++k) {
      double f = -(2 * k - 1) * ir2;
      imm = make_double2(f * (x * imm.x - y * imm.y), f * (x * imm.y + y * imm.x));
    }
    col[tri(m) + m] = imm;
    if (m + 1 <= p) {
      double f1 = (2 * m + 1) * z * ir2;
      col[tri(m + 1) + m] = make_double2(f1 * imm.x, f1 * imm.y);
    }
    for (int n = m + 2; n <= p; ++n) {
      double a = (2 * n - 1) * z * ir2, b = (double)(n + m - 1) * (n - m - 1) * ir2;
      double2 u = col[tri(n - 1) + m], v = col[tri(n - 2) + m];
      col[tri(n) + m] = make_double2(a * u.x - b * v.x, a * u.y - b * v.y);
    }
  }
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m <= n; ++m) {
      double2 v = col[tri(n) + m];
      out[fidx(n, m)] = v;
      out[fidx(n, -m)] = (m & 1) ? make_double2(-v.x, v.y) : make_double2(v.x, -v.y);
    }
}

}  // namespace

// Paper-normalised Y_n^m(theta, phi) = sqrt((n-m)!/(n+m)!) P_n^m(cos theta)
// e^{i m phi}, Condon-Shortley phase in P_n^m, for 0 <= m <= n and
// nlo <= n <= p (lower degrees are left zero; their Legendre values are still
// needed by the recurrence, their normalisation and phases are not).
void host_ynm(int p, double ct, double phi, std::vector<double2>& y, int nlo) {
  y.assign(ncoef(p), make_double2(0, 0));
  double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
  std::vector<double> P(ncoef(p));
  double pmm = 1.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) pmm *= -(2.0 * m - 1.0) * st;
    P[tri(m) + m] = pmm;
    if (m + 1 <= p) P[tri(m + 1) + m] = ct * (2.0 * m + 1.0) * pmm;
    for (int n = m + 2; n <= p; ++n)
      P[tri(n) + m] = ((2.0 * n - 1.0) * ct * P[tri(n - 1) + m] - (n + m - 1.0) * P[tri(n - 2) + m]) / (n - m);
  }
  for (int n = nlo; n <= p; ++n) {
    double f = 1.0;  // (n-m)!/(n+m)! built up over m
    for (int m = 0; m <= n; ++m) {
      if (m > 0) f /= (double)(n + m) * (n - m + 1);
      double c = std::sqrt(f) * P[tri(n) + m];
      y[tri(n) + m] = make_double2(c * std::cos(m * phi), c * std::sin(m * phi));
    }
  }
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration).
void gauss_legendre(int N, std::vector<double>& x, std::vector<double>& w) {
  x.assign(N, 0.0);
  w.assign(N, 0.0);
  for (int i = 0; i < N; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (N + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= N; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = N == 1 ? z : p1, pm = N == 1 ? 1.0 : p0;
      dp = N * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// The rotation by +90 degrees about y acting on degree-n coefficient sets:
// D[m'][m] (m', m in -n..n) such that f(R^-1 x) = sum_{m'} (D c)_{m'} Y_n^{m'}
// for f = sum_m c_m Y_n^m, by quadrature exact for degree 2n
// (D = (2n+1)/(4 pi) * integral conj(Y^{m'}) Y^m(R^-1 x)).  Real orthogonal.
void host_rot90(int n, std::vector<double>& D) {
  const int W = 2 * n + 1;
  D.assign((size_t)W * W, 0.0);
  std::vector<double> gx, gw;
  gauss_legendre(n + 1, gx, gw);
  const int nphi = 2 * n + 1;
  std::vector<double2> y, yr;
  std::vector<double> ax(W), ay(W), bx(W), by(W);
  for (int i = 0; i <= n; ++i) {
    double ct = gx[i], st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
    for (int k = 0; k < nphi; ++k) {
      double ph = 2.0 * M_PI * k / nphi;
      double x = st * std::cos(ph), yv = st * std::sin(ph), z = ct;
      // R^-1 x for R = rotation by +pi/2 about y: (x, y, z) -> (-z, y, x)
      double xr = -z, yy = yv, zr = x;
      double ctr = std::max(-1.0, std::min(1.0, zr)), phr = std::atan2(yy, xr);
      host_ynm(n, ct, ph, y, n);
      host_ynm(n, ctr, phr, yr, n);
      double wt = gw[i] * (2.0 * M_PI / nphi) * (2 * n + 1) / (4.0 * M_PI);
      // degree-n values for orders -n..n (Y_n^{-m} = conj(Y_n^m) up to the
      // (-1)^m that cancels in the product below)
      for (int m = -n; m <= n; ++m) {
        const double2 u = y[tri(n) + std::abs(m)], v = yr[tri(n) + std::abs(m)];
        ax[m + n] = u.x;
        ay[m + n] = m < 0 ? -u.y : u.y;
        bx[m + n] = v.x;
        by[m + n] = m < 0 ? -v.y : v.y;
      }
      for (int r = 0; r < W; ++r) {
        const double arx = ax[r], ary = ay[r];
        double* row = &D[(size_t)r * W];
        // Re(conj(a) b)
        for (int c = 0; c < W; ++c) row[c] += wt * (arx * bx[c] + ary * by[c]);
      }
    }
  }
}

namespace {
// Host images of the translation tables of one order.  They depend on the
// order alone, so each order is computed once per process (12 ms of host
// work at p = 16, 32 ms at p = 21, 87 ms at p = 27) and every later plan
// only uploads it.  The cache holds at most one entry per order (0..27;
// 6 MB at p = 16 and 17 MB at p = 27, mostly the dense M2L kernels).
// Entries are never freed: the cache is a fixed array of plain pointers, so
// the library has no static object with a destructor and nothing of it runs
// during process teardown (the memory returns to the system at exit).
struct HostTables {
  std::vector<double2> oct, itab;
  std::vector<double> rot, zt, geo, sf, rsc;
  std::vector<float> rot32, zt32;
  int rlen = 0, zlen = 0;
};
std::mutex g_tables_mu;
const HostTables* g_tables[MAX_ORDER + 1];

int compute_tables(int p, HostTables* h, Error* err) {
  const int F1 = (p + 1) * (p + 1), F2 = (2 * p + 1) * (2 * p + 1);
  std::vector<double2> oct(8 * F1), itab((size_t)343 * F2, make_double2(0, 0)), tmp;
  for (int o = 0; o < 8; ++o) {
    double dx = (o & 1) ? 0.25 : -0.25, dy = ((o >> 1) & 1) ? 0.25 : -0.25, dz = ((o >> 2) & 1) ? 0.25 : -0.25;
    host_regular(dx, dy, dz, p, tmp);
    std::copy(tmp.begin(), tmp.end(), oct.begin() + (size_t)o * F1);
  }
  for (int tx = -3; tx <= 3; ++tx)
    for (int ty = -3; ty <= 3; ++ty)
      for (int tz = -3; tz <= 3; ++tz) {
        if (std::abs(tx) <= 1 && std::abs(ty) <= 1 && std::abs(tz) <= 1) continue;
        int o = (tx + 3) * 49 + (ty + 3) * 7 + (tz + 3);
        host_irregular(tx, ty, tz, 2 * p, tmp);
        std::copy(tmp.begin(), tmp.end(), itab.begin() + (size_t)o * F2);
      }
  // rotation-based M->L: the +90 degree rotation about y per degree n, split
  // for coefficient sets with x_{-m} = (-1)^m conj(x_m) into real matrices
  // acting on the real parts (A+) and on the imaginary parts (A-).  Both are
  // checkerboard-sparse: A+[m'][m] vanishes unless m' + m + n is even and
  // A-[m'][m] unless it is odd (and m >= 1).  Row m' of degree n stores the
  // nonzero A+ entries (m = q, q+2, ..., q = (n+m') mod 2), then the A-
  // entries (m = 1-q, 3-q, ..., m >= 1), in a row of n+1 slots.  The inverse
  // rotation S R S (S = diag((-1)^m)) is the same table with the signs
  // (-1)^n on A+ and -(-1)^n on A-.
  const int rlen = (p + 1) * (p + 2) * (2 * p + 3) / 6;
  std::vector<double> rot((size_t)rlen, 0.0);
  std::vector<double> D;
  for (int n = 0, off = 0; n <= p; off += (n + 1) * (n + 1), ++n) {
    host_rot90(n, D);
    const int W = 2 * n + 1, K = n + 1;
    for (int mp = 0; mp <= n; ++mp) {
      const int q = (n + mp) & 1;
      int j = 0;
      for (int m = 0; m <= n; ++m) {
        const double dp = D[(size_t)(mp + n) * W + (m + n)], dm = D[(size_t)(mp + n) * W + (n - m)];
        const double ap = m == 0 ? dp : dp + dm, am = m == 0 ? 0.0 : dp - dm;
        if (((m & 1) != q && std::fabs(ap) > 1e-12) || ((m & 1) == q && std::fabs(am) > 1e-12)) {
          err->code = -4;
          err->msg = "rotation table: unexpected nonzero entry";
          return -4;
        }
      }
      for (int m = q; m <= n; m += 2) {
        const double dp = D[(size_t)(mp + n) * W + (m + n)], dm = D[(size_t)(mp + n) * W + (n - m)];
        rot[off + mp * K + j++] = m == 0 ? dp : dp + dm;
      }
      for (int m = (q == 1 ? 2 : 1); m <= n; m += 2)
        rot[off + mp * K + j++] = D[(size_t)(mp + n) * W + (m + n)] - D[(size_t)(mp + n) * W + (n - m)];
    }
  }
  std::vector<double> sf(ncoef(p));
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m <= n; ++m) {
      double f = 1.0;
      for (int k = 2; k <= n - m; ++k) f *= k;
      double g = 1.0;
      for (int k = 2; k <= n + m; ++k) g *= k;
      sf[tri(n) + m] = std::sqrt(f * g);
    }
  // z translation by rho (box units) on rotated sets, per order l:
  //   L'_k^l = rho^-(k+1) sum_n H_l[k-l][n-l] rho^-n M'_n^l,
  //   H_l[k-l][n-l] = (-1)^(n+l) (n+k)! / (s_k^l s_n^l).
  const int zlen = (p + 1) * (p + 2) * (2 * p + 3) / 6;
  std::vector<double> zt(zlen, 0.0);
  {
    std::vector<double> fac(2 * p + 2, 1.0);
    for (int j = 1; j <= 2 * p + 1; ++j) fac[j] = fac[j - 1] * j;
    for (int l = 0, off = 0; l <= p; off += (p - l + 1) * (p - l + 1), ++l) {
      const int K = p - l + 1;
      for (int k = l; k <= p; ++k)
        for (int n = l; n <= p; ++n)
          zt[off + (k - l) * K + (n - l)] =
              (((n + l) & 1) ? -1.0 : 1.0) * fac[n + k] / (sf[tri(k) + l] * sf[tri(n) + l]);
    }
  }
  // per integer offset t (343 slots): e^{-i(pi/2 - phi_t)}, e^{i theta_t}, 1/|t|
  std::vector<double> geo((size_t)343 * 8, 0.0);
  for (int tx = -3; tx <= 3; ++tx)
    for (int ty = -3; ty <= 3; ++ty)
      for (int tz = -3; tz <= 3; ++tz) {
        if (std::abs(tx) <= 1 && std::abs(ty) <= 1 && std::abs(tz) <= 1) continue;
        double* q = geo.data() + (size_t)((tx + 3) * 49 + (ty + 3) * 7 + (tz + 3)) * 8;
        const double rho = std::sqrt((double)(tx * tx + ty * ty + tz * tz));
        const double th = std::acos(tz / rho), ph = std::atan2((double)ty, (double)tx);
        q[0] = std::cos(0.5 * M_PI - ph);
        q[1] = -std::sin(0.5 * M_PI - ph);
        q[2] = std::cos(th);
        q[3] = std::sin(th);
        q[4] = 1.0 / rho;
      }
  std::vector<double> rsc(ncoef(p));
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m <= n; ++m) rsc[tri(n) + m] = 1.0 / (sf[tri(n) + m] * sf[tri(n) + m]);
  h->rot32.assign(rot.begin(), rot.end());
  h->zt32.assign(zt.begin(), zt.end());
  h->oct = std::move(oct);
  h->itab = std::move(itab);
  h->rot = std::move(rot);
  h->zt = std::move(zt);
  h->geo = std::move(geo);
  h->sf = std::move(sf);
  h->rsc = std::move(rsc);
  h->rlen = rlen;
  h->zlen = zlen;
  return 0;
}
}  // namespace

int make_tables(int p, Tables* tb, hipStream_t s, Error* err) {
  tb->p = p;
  tb->bytes = 0;
  if (p < 0 || p > MAX_ORDER) {
    err->code = -1;
    err->msg = "expansion order out of range";
    return -1;
  }
  const HostTables* hp = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_tables_mu);
    hp = g_tables[p];
  }
  if (!hp) {
    HostTables* h = new HostTables();
    const int rc = compute_tables(p, h, err);
    if (rc != 0) {
      delete h;
      return rc;
    }
    std::lock_guard<std::mutex> lk(g_tables_mu);
    if (g_tables[p]) delete h;  // another thread filled it meanwhile
    else g_tables[p] = h;
    hp = g_tables[p];
  }
  const HostTables& H = *hp;
  const auto &oct = H.oct, &itab = H.itab;
  const auto &rot = H.rot, &zt = H.zt, &geo = H.geo, &sf = H.sf, &rsc = H.rsc;
  const auto &rot32 = H.rot32, &zt32 = H.zt32;
  tb->rot_len = H.rlen;
  tb->zt_len = H.zlen;
  RPY_HIP(hipMalloc(&tb->oct, sizeof(double2) * oct.size()));
  RPY_HIP(hipMalloc(&tb->itab, sizeof(double2) * itab.size()));
  RPY_HIP(hipMalloc(&tb->rot64, sizeof(double) * rot.size()));
  RPY_HIP(hipMalloc(&tb->rot32, sizeof(float) * rot32.size()));
  RPY_HIP(hipMalloc(&tb->zt64, sizeof(double) * zt.size()));
  RPY_HIP(hipMalloc(&tb->zt32, sizeof(float) * zt32.size()));
  RPY_HIP(hipMalloc(&tb->geo, sizeof(double) * geo.size()));
  RPY_HIP(hipMalloc(&tb->sfac, sizeof(double) * sf.size()));
  RPY_HIP(hipMalloc(&tb->rscale, sizeof(double) * rsc.size()));
  RPY_HIP(hipMemcpy(tb->rscale, rsc.data(), sizeof(double) * rsc.size(), hipMemcpyHostToDevice));
  tb->bytes = sizeof(double2) * (oct.size() + itab.size()) + (sizeof(double) + sizeof(float)) * (rot.size() + zt.size()) +
              sizeof(double) * (geo.size() + sf.size() + rsc.size());
  RPY_HIP(hipMemcpy(tb->oct, oct.data(), sizeof(double2) * oct.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(tb->itab, itab.data(), sizeof(double2) * itab.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(tb->rot64, rot.data(), sizeof(double) * rot.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(tb->rot32, rot32.data(), sizeof(float) * rot32.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(tb->zt64, zt.data(), sizeof(double) * zt.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(tb->zt32, zt32.data(), sizeof(float) * zt32.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(tb->geo, geo.data(), sizeof(double) * geo.size(), hipMemcpyHostToDevice));
  RPY_HIP(hipMemcpy(tb->sfac, sf.data(), sizeof(double) * sf.size(), hipMemcpyHostToDevice));
  (void)s;
  return make_p2e_tables(p, tb, err);
}

void free_tables(Tables* tb) {
  void* ps[] = {tb->oct, tb->itab, tb->rot64, tb->rot32, tb->zt64, tb->zt32, tb->geo, tb->sfac, tb->rscale,
                tb->p2e[0].desc, tb->p2e[0].slot, tb->p2e[0].scale, tb->p2e[1].desc, tb->p2e[1].slot,
                tb->p2e[1].scale, tb->p2e_dk};
  for (void* q : ps)
    if (q) (void)hipFree(q);
  tb->oct = tb->itab = nullptr;
  tb->rot64 = tb->zt64 = tb->geo = tb->sfac = tb->rscale = nullptr;
  tb->rot32 = tb->zt32 = nullptr;
  for (P2ESched& s : tb->p2e) {
    s.desc = nullptr;
    s.slot = nullptr;
    s.scale = nullptr;
    s.P = 0;
  }
  tb->p2e_dk = nullptr;
}

// ------------------------------------------------------------- permutes ----
__global__ void k_permute_forces(const double* F, const int* perm, int64_t n, int r0, int nrc, double* sF) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t j = perm[i];
  for (int r = 0; r < nrc; ++r) {
    const double* f = F + ((int64_t)(r0 + r) * n + j) * 3;
    for (int k = 0; k < 3; ++k) sF[((int64_t)r * 3 + k) * n + i] = f[k];
  }
}

__global__ void k_unpermute(const double* u, const double* uf, const int* perm, int64_t n, int r0, int nrc,
                            double* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t j = perm[i];
  for (int r = 0; r < nrc; ++r) {
    double* o = out + ((int64_t)(r0 + r) * n + j) * 3;
    for (int k = 0; k < 3; ++k) o[k] = u[((int64_t)r * 3 + k) * n + i] + uf[((int64_t)r * 3 + k) * n + i];
  }
}

hipError_t permute_forces(const Launch& l, const double* F, int nrhs_total, int r0, int nrc, double* sF) {
  (void)nrhs_total;
  int64_t n = l.B->n;
  if (n == 0) return hipSuccess;
  k_permute_forces<<<nblk(n, 256), 256, 0, l.s>>>(F, l.B->perm, n, r0, nrc, sF);
  return hipGetLastError();
}

hipError_t unpermute_velocities(const Launch& l, const double* u, const double* uf, int r0, int nrc, double* out) {
  int64_t n = l.B->n;
  if (n == 0) return hipSuccess;
  k_unpermute<<<nblk(n, 256), 256, 0, l.s>>>(u, uf, l.B->perm, n, r0, nrc, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ M->M --
// One block per parent box of one level; thread t = output coefficient (n,m):
// M_n^m(P) = sum_{k<=n,l} 2^-k M_k^l(C) conj(R_{n-k}^{m-l}(d/h_P)).
constexpr int TR_T = 256;

// One block per (parent box, right-hand side): thread t = output (n,m) of
// the four densities of that right-hand side, summing the children's
// translated multipoles in turn (Rt and the child's four densities staged in
// LDS, the fourth re-centred on the child first); each Rt entry read serves
// the four densities.
template <int ND>
__global__ void __launch_bounds__(TR_T) k_m2m(int p, int ls, Tree t, const double2* oct, double2* M) {
  const int b = ls + blockIdx.x, d0 = 4 * blockIdx.y;
  const int nc = t.nchild[b];
  if (nc == 0) return;
  const int T = ncoef(p), F1 = (p + 1) * (p + 1);
  extern __shared__ double2 sm[];
  double2* Rt = sm;       // F1
  double2* Mc = sm + F1;  // [4][F1]
  // outputs threadIdx.x and threadIdx.x + TR_T (T exceeds TR_T above order 21)
  double2 acc[2][4];
  int nq[2] = {0, 0}, mq[2] = {0, 0};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[q][g] = make_double2(0, 0);
    const int c = threadIdx.x + q * TR_T;
    if (c < T) {
      while (tri(nq[q] + 1) <= c) ++nq[q];
      mq[q] = c - tri(nq[q]);
    }
  }
  for (int C = t.child[b]; C < t.child[b] + nc; ++C) {
    const int o = (t.ax[C] & 1) | ((t.ay[C] & 1) << 1) | ((t.az[C] & 1) << 2);
    const double w[3] = {t.cx[C] - t.cx[b], t.cy[C] - t.cy[b], t.cz[C] - t.cz[b]};
    __syncthreads();
    for (int i = threadIdx.x; i < F1; i += TR_T) Rt[i] = oct[(int64_t)o * F1 + i];
    const double2* src = M + ((int64_t)C * ND + d0) * T;
    for (int f = threadIdx.x; f < F1; f += TR_T) {
      int k = (int)sqrt((double)f);
      while (k * k > f) --k;
      while ((k + 1) * (k + 1) <= f) ++k;
      const int l = f - k * k - k;
      const double sc = ldexp(1.0, -k);
      double2 v[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) v[g] = getc(src + g * T, k, l, p);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[3].x += w[c] * v[c].x;
        v[3].y += w[c] * v[c].y;
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) Mc[g * F1 + f] = make_double2(v[g].x * sc, v[g].y * sc);
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
      if (threadIdx.x + q * TR_T >= T) break;
      const int n = nq[q], m = mq[q];
      for (int k = 0; k <= n; ++k) {
        const int j = n - k;
        const int lmin = max(-k, m - j), lmax = min(k, m + j);
        const int mk = fidx(k, 0), rj = fidx(j, m);  // rj - l >= j*j for l <= lmax
        for (int l = lmin; l <= lmax; ++l) {
          const double2 r = Rt[rj - l];
#pragma unroll
          for (int g = 0; g < 4; ++g) cfmac(acc[q][g], Mc[g * F1 + mk + l], r);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q)
    if (threadIdx.x + q * TR_T < T)
#pragma unroll
      for (int g = 0; g < 4; ++g) M[((int64_t)b * ND + d0 + g) * T + threadIdx.x + q * TR_T] = acc[q][g];
}

// ------------------------------------------------------------------ L->L --
// One block per (child box of one level, right-hand side); thread t =
// output (k,l) of the four densities:
// L_k^l(C) += 2^-(k+1) sum_{n>=k,m} L_n^m(P) R_{n-k}^{m-l}(d/h_P),
// each Rt entry read serving the four densities.
template <int ND>
__global__ void __launch_bounds__(TR_T) k_l2l(int p, int ls, Tree t, const double2* oct, double2* L) {
  const int b = ls + blockIdx.x, d0 = 4 * blockIdx.y;
  const int P = t.parent[b];
  if (P < 0) return;
  const int T = ncoef(p), F1 = (p + 1) * (p + 1);
  extern __shared__ double2 sm[];
  double2* Rt = sm;       // F1
  double2* Lp = sm + F1;  // [4][F1]
  const int o = (t.ax[b] & 1) | ((t.ay[b] & 1) << 1) | ((t.az[b] & 1) << 2);
  const double w[3] = {t.cx[P] - t.cx[b], t.cy[P] - t.cy[b], t.cz[P] - t.cz[b]};
  for (int i = threadIdx.x; i < F1; i += TR_T) Rt[i] = oct[(int64_t)o * F1 + i];
  const double2* src = L + ((int64_t)P * ND + d0) * T;
  for (int f = threadIdx.x; f < F1; f += TR_T) {
    int k = (int)sqrt((double)f);
    while (k * k > f) --k;
    while ((k + 1) * (k + 1) <= f) ++k;
    const int l = f - k * k - k;
    double2 v[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) v[g] = getc(src + g * T, k, l, p);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[3].x += w[c] * v[c].x;
      v[3].y += w[c] * v[c].y;
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) Lp[g * F1 + f] = v[g];
  }
  __syncthreads();
  // outputs threadIdx.x and threadIdx.x + TR_T (T exceeds TR_T above order 21)
  for (int c = threadIdx.x; c < T; c += TR_T) {
    int k = 0;
    while (tri(k + 1) <= c) ++k;
    const int l = c - tri(k);
    double2 acc[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[g] = make_double2(0, 0);
    for (int n = k; n <= p; ++n) {
      const int j = n - k;
      const int mmin = max(-n, l - j), mmax = min(n, l + j);
      const int ln = fidx(n, 0), rj = fidx(j, -l);  // rj + m >= j*j for m >= mmin
      for (int m = mmin; m <= mmax; ++m) {
        const double2 r = Rt[rj + m];
#pragma unroll
        for (int g = 0; g < 4; ++g) cfma(acc[g], Lp[g * F1 + ln + m], r);
      }
    }
    const double sc = ldexp(1.0, -(k + 1));
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      double2* out = L + ((int64_t)b * ND + d0 + g) * T + c;
      const double2 v = *out;
      *out = make_double2(v.x + sc * acc[g].x, v.y + sc * acc[g].y);
    }
  }
}

// ----------------------------------------------------------- M->L (V) -----
// One block per target box; for every V-list source the offset table
// I_j^mu(t) and the (re-centred) source multipole are staged in LDS and
// thread (k,l) accumulates (-1)^l sum_{n,m} (-1)^n M_n^m I_{n+k}^{m-l}(t).
constexpr int M2L_T = 256;

template <int ND>
__global__ void __launch_bounds__(M2L_T) k_m2l_dense(int p, int c0, Tree t, List V, const double2* itab,
                                                     const double2* M, double2* L) {
  // outputs c0 .. c0 + M2L_T - 1 (a second launch covers T > M2L_T)
  const int b = blockIdx.x, c = c0 + threadIdx.x;
  const int T = ncoef(p), F1 = (p + 1) * (p + 1), F2 = (2 * p + 1) * (2 * p + 1);
  extern __shared__ double2 sm[];
  double2* It = sm;            // F2
  double2* Ms = sm + F2;       // ND * F1
  int k = 0, l = 0;
  if (c < T) {
    while (tri(k + 1) <= c) ++k;
    l = c - tri(k);
  }
  double2 acc[ND];
  for (int d = 0; d < ND; ++d) acc[d] = make_double2(0, 0);
  const int e0 = V.off[b], e1 = V.off[b + 1];
  for (int e = e0; e < e1; ++e) {
    const int S = V.ent[e];
    const int tx = t.ax[S] - t.ax[b], ty = t.ay[S] - t.ay[b], tz = t.az[S] - t.az[b];
    const int o = (tx + 3) * 49 + (ty + 3) * 7 + (tz + 3);
    const double w[3] = {t.cx[S] - t.cx[b], t.cy[S] - t.cy[b], t.cz[S] - t.cz[b]};
    __syncthreads();
    for (int i = threadIdx.x; i < F2; i += M2L_T) It[i] = itab[(int64_t)o * F2 + i];
    const double2* src = M + (int64_t)S * ND * T;
    for (int i = threadIdx.x; i < ND * F1; i += M2L_T) {
      int d = i / F1, f = i % F1;
      int n = (int)sqrt((double)f);
      while (n * n > f) --n;
      while ((n + 1) * (n + 1) <= f) ++n;
      int m = f - n * n - n;
      int dd = d & 3, base = d - dd;
      double2 v = getc(src + d * T, n, m, p);
      if (dd == 3)
        for (int c = 0; c < 3; ++c) {
          double2 u = getc(src + (base + c) * T, n, m, p);
          v.x += w[c] * u.x;
          v.y += w[c] * u.y;
        }
      if (n & 1) { v.x = -v.x; v.y = -v.y; }
      Ms[d * F1 + f] = v;
    }
    __syncthreads();
    if (c < T) {
      for (int n = 0; n <= p; ++n) {
        const int base_i = (n + k) * (n + k) + (n + k) - l;
        const int base_m = n * n + n;
        for (int m = -n; m <= n; ++m) {
          double2 iv = It[base_i + m];
#pragma unroll
          for (int d = 0; d < ND; ++d) cfma(acc[d], Ms[d * F1 + base_m + m], iv);
        }
      }
    }
  }
  if (c < T) {
    const double sg = (l & 1) ? -1.0 : 1.0;
    double2* out = L + (int64_t)b * ND * T + c;
    for (int d = 0; d < ND; ++d) out[d * T] = make_double2(sg * acc[d].x, sg * acc[d].y);
  }
}

#define DISPATCH_ND(nrc, KERNEL_CALL)                      \
  switch (nrc) {                                           \
    case 1: { constexpr int ND = 4; KERNEL_CALL; break; }  \
    case 2: { constexpr int ND = 8; KERNEL_CALL; break; }  \
    case 4: { constexpr int ND = 16; KERNEL_CALL; break; } \
    default: return hipErrorInvalidValue;                  \
  }

hipError_t run_m2m(const Launch& l, int nrc, Exp e) {
  const Built* B = l.B;
  const size_t shm = sizeof(double2) * 5 * (l.p + 1) * (l.p + 1);
  // parents down to level 2 only: multipoles at levels 0 and 1 are never
  // read (V lists start at level 2, and W-list boxes are descendants of a
  // leaf's colleagues, so they sit at level 2 or deeper)
  for (int lev = B->depth - 1; lev >= 2; --lev) {
    const int ls = B->level_start[lev], le = B->level_start[lev + 1];
    DISPATCH_ND(nrc, (k_m2m<ND><<<dim3(le - ls, ND / 4), TR_T, shm, l.s>>>(l.p, ls, B->tree, l.tb->oct, e.M)));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

hipError_t run_m2l(const Launch& l, int nrc, Exp e) {
  const Built* B = l.B;
  const int p = l.p;
  size_t shm = sizeof(double2) * ((2 * p + 1) * (2 * p + 1) + 4 * nrc * (p + 1) * (p + 1));
  if (shm > 160 * 1024) return hipErrorInvalidValue;
  auto go = [&](auto kern) {
    hipError_t he = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (he != hipSuccess) return he;
    for (int c0 = 0; c0 < ncoef(p); c0 += M2L_T)
      kern<<<B->tree.nbox, M2L_T, shm, l.s>>>(p, c0, B->tree, B->lists[LV], l.tb->itab, e.M, e.L);
    return hipSuccess;
  };
  hipError_t he = hipErrorInvalidValue;
  if (nrc == 1) he = go(k_m2l_dense<4>);
  else if (nrc == 2) he = go(k_m2l_dense<8>);
  else if (nrc == 4) he = go(k_m2l_dense<16>);
  if (he != hipSuccess) return he;
  return hipGetLastError();
}

hipError_t run_l2l(const Launch& l, int nrc, Exp e) {
  const Built* B = l.B;
  const size_t shm = sizeof(double2) * 5 * (l.p + 1) * (l.p + 1);
  // children from level 3: local expansions at levels 0 and 1 are zero (no
  // V or X entries there), so level 2 keeps what M->L and S->L wrote
  for (int lev = 3; lev <= B->depth; ++lev) {
    const int ls = B->level_start[lev], le = B->level_start[lev + 1];
    DISPATCH_ND(nrc, (k_l2l<ND><<<dim3(le - ls, ND / 4), TR_T, shm, l.s>>>(l.p, ls, B->tree, l.tb->oct, e.L)));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}


}  // namespace rpy
