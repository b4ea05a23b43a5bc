// Multipole-to-local translation (M->L over V lists) by rotation:
// every V-list source multipole is rotated so that the translation vector
// lies on the z axis, translated along z (an O(p^3) operator that keeps the
// order m), and rotated back.  The paper's FMM diagonalises this step with
// exponential expansions (arXiv:1711.02976, Sec. 1 and 3.2); this kernel
// uses the rotation factorisation instead and computes the same truncated
// operator as the dense M->L.
//
// Coefficients are handled in the paper's normalisation (Sec. 2: Y_n^m =
// sqrt((n-|m|)!/(n+|m|)!) P_n^|m| e^{i m phi}), where rotations are real
// orthogonal per degree.  A rotation taking the offset t = (rho, theta, phi)
// to +z is Phi(-pi/2) R90^T Phi(-theta) R90 Phi(pi/2 - phi), with
// Phi(a) = diag(e^{-i m a}) and R90 the fixed rotation by +90 degrees about
// y, whose inverse is S R90 S, S = diag((-1)^m).  The whole M->L is
//   Phi(phi - pi/2) R90^-1 Phi(theta) R90 Z(rho) R90^-1 Phi(-theta) R90 Phi(pi/2 - phi)
// with Z(rho) the translation along +z:
//   L'_k^l = sum_{n>=l} M'_n^l (-1)^{n+l} (n+k)! / (s_k^l s_n^l rho^{n+k+1}),
//   s_n^m = sqrt((n-m)!(n+m)!).
//
// One block per target box; its V-list sources times densities form the
// columns, processed RC at a time through two LDS buffers; each thread owns
// up to four outputs of one degree (or order) of one column.
#include <hip/hip_runtime.h>

#include "fmm.h"

namespace rpy {

namespace {

constexpr int ROT_T = 256;

template <class R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

template <class R>
struct RotSmem {
  using C = typename V2<R>::T;
  C* rot;         // rot_len
  double* sf;     // T
  C* X;           // RC * T
  C* Y;           // RC * T
  R* G;           // RC * (2p+1)
  C* E1;          // RC * (p+1)
  C* E2;          // RC * (p+1)
  int* colS;      // RC
  int* colD;      // RC
  int* roff;      // p+2
};

template <class C>
__device__ inline C cmul2(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// Y[c] = (inv ? S R90 S : R90) X[c] for every column, then times the phase
// (mode 0: none, 1: E, 2: conj(E)).
template <class R>
__device__ void dense_step(const RotSmem<R>& sm, int p, int RC, const typename V2<R>::T* X, typename V2<R>::T* Y,
                           bool inv, int mode, const typename V2<R>::T* E) {
  using C = typename V2<R>::T;
  const int T = ncoef(p);
  // items: (n, g) pairs enumerated degree by degree, times columns
  int ng = 0;
  for (int n = 0; n <= p; ++n) ng += (n + 4) / 4;
  const int nitem = ng * RC;
  for (int item = threadIdx.x; item < nitem; item += ROT_T) {
    const int c = item % RC;
    int it = item / RC, n = 0;
    while (it >= (n + 4) / 4) {
      it -= (n + 4) / 4;
      ++n;
    }
    const int g = it, pad = 4 * ((n + 4) / 4);
    const C* A = sm.rot + sm.roff[n] + 4 * g;
    const C* x = X + c * T + tri(n);
    R ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
    for (int m = 0; m <= n; ++m) {
      C v = x[m];
      if (inv && (m & 1)) { v.x = -v.x; v.y = -v.y; }
      const C* a = A + m * pad;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        C q = a[r];
        ar[r] = fma(q.x, v.x, ar[r]);
        ai[r] = fma(q.y, v.y, ai[r]);
      }
    }
    C* y = Y + c * T + tri(n);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int mp = 4 * g + r;
      if (mp > n) break;
      C v;
      v.x = ar[r];
      v.y = ai[r];
      if (inv && (mp & 1)) { v.x = -v.x; v.y = -v.y; }
      if (mode) {
        C e = E[c * (p + 1) + mp];
        if (mode == 2) e.y = -e.y;
        v = cmul2(v, e);
      }
      y[mp] = v;
    }
  }
}

// Translation along +z by rho (per column, through G[c][j] = j!/rho^{j+1}).
template <class R>
__device__ void ztrans_step(const RotSmem<R>& sm, int p, int RC, const typename V2<R>::T* X, typename V2<R>::T* Y) {
  using C = typename V2<R>::T;
  const int T = ncoef(p);
  int nz = 0;
  for (int l = 0; l <= p; ++l) nz += (p - l + 4) / 4;
  const int nitem = nz * RC;
  for (int item = threadIdx.x; item < nitem; item += ROT_T) {
    const int c = item % RC;
    int it = item / RC, l = 0;
    while (it >= (p - l + 4) / 4) {
      it -= (p - l + 4) / 4;
      ++l;
    }
    const int k0 = l + 4 * it;
    const R* G = sm.G + c * (2 * p + 1);
    const C* x = X + c * T;
    R accr[4] = {0, 0, 0, 0}, acci[4] = {0, 0, 0, 0};
    for (int n = l; n <= p; ++n) {
      R w = (R)(((n & 1) ? -1.0 : 1.0) / sm.sf[tri(n) + l]);
      C v = x[tri(n) + l];
      R vx = v.x * w, vy = v.y * w;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int k = k0 + r;
        R gk = k <= p ? G[n + k] : (R)0;
        accr[r] = fma(gk, vx, accr[r]);
        acci[r] = fma(gk, vy, acci[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int k = k0 + r;
      if (k > p) break;
      R w = (R)(((l & 1) ? -1.0 : 1.0) / sm.sf[tri(k) + l]);
      C o;
      o.x = accr[r] * w;
      o.y = acci[r] * w;
      Y[c * T + tri(k) + l] = o;
    }
  }
}

}  // namespace

template <int ND, class R>
__global__ void __launch_bounds__(ROT_T) k_m2l_rot(int p, int RC, Tree t, List V, const double2* rot,
                                                   const int* roff, int rot_len, const double* sfac,
                                                   const double* offtab, const double2* M, double2* L) {
  using C = typename V2<R>::T;
  extern __shared__ double2 smem[];
  const int b = blockIdx.x;
  const int T = ncoef(p), OT = 4 * (p + 1) + 2 * p + 1;
  RotSmem<R> sm;
  {
    double* d = reinterpret_cast<double*>(smem);
    sm.sf = d; d += T;
    C* cq = reinterpret_cast<C*>(d);
    sm.rot = cq; cq += rot_len;
    sm.X = cq; cq += RC * T;
    sm.Y = cq; cq += RC * T;
    sm.E1 = cq; cq += RC * (p + 1);
    sm.E2 = cq; cq += RC * (p + 1);
    R* rq = reinterpret_cast<R*>(cq);
    sm.G = rq; rq += RC * (2 * p + 1);
    int* iq = reinterpret_cast<int*>(rq);
    sm.colS = iq; iq += RC;
    sm.colD = iq; iq += RC;
    sm.roff = iq;
  }
  for (int i = threadIdx.x; i < rot_len; i += ROT_T) {
    C v;
    v.x = (R)rot[i].x;
    v.y = (R)rot[i].y;
    sm.rot[i] = v;
  }
  for (int i = threadIdx.x; i < T; i += ROT_T) sm.sf[i] = sfac[i];
  for (int i = threadIdx.x; i < p + 2; i += ROT_T) sm.roff[i] = roff[i];
  double2* Lb = L + (int64_t)b * ND * T;
  for (int i = threadIdx.x; i < ND * T; i += ROT_T) Lb[i] = make_double2(0, 0);
  const int e0 = V.off[b], e1 = V.off[b + 1];
  const int ncols = (e1 - e0) * ND;
  for (int c0 = 0; c0 < ncols; c0 += RC) {
    __syncthreads();
    if ((int)threadIdx.x < RC) {
      const int c = threadIdx.x, gc = c0 + c;
      sm.colS[c] = gc < ncols ? V.ent[e0 + gc / ND] : -1;
      sm.colD[c] = gc % ND;
    }
    __syncthreads();
    // per-column phases and translation factors from the offset tables
    const int per = 2 * (p + 1) + 2 * (p + 1) + 2 * p + 1;
    for (int i = threadIdx.x; i < RC * per; i += ROT_T) {
      const int c = i / per, k = i % per;
      const int S = sm.colS[c] >= 0 ? sm.colS[c] : V.ent[e0];
      const int o = (t.ax[S] - t.ax[b] + 3) * 49 + (t.ay[S] - t.ay[b] + 3) * 7 + (t.az[S] - t.az[b] + 3);
      const double* q = offtab + (int64_t)o * OT;
      if (k < 2 * (p + 1)) {
        R* e = reinterpret_cast<R*>(sm.E1 + c * (p + 1));
        e[k] = (R)q[k];
      } else if (k < 4 * (p + 1)) {
        R* e = reinterpret_cast<R*>(sm.E2 + c * (p + 1));
        e[k - 2 * (p + 1)] = (R)q[k];
      } else {
        sm.G[c * (2 * p + 1) + (k - 4 * (p + 1))] = (R)q[k];
      }
    }
    __syncthreads();
    // load: multipole (stored R-normalised, box-scaled) -> paper
    // normalisation, fourth density re-centred on this machine, times E1.
    for (int i = threadIdx.x; i < RC * T; i += ROT_T) {
      const int c = i / T, f = i % T;
      const int S = sm.colS[c];
      C out;
      out.x = 0;
      out.y = 0;
      if (S >= 0) {
        const int d = sm.colD[c];
        const double2* src = M + (int64_t)S * ND * T;
        double2 v = src[d * T + f];
        if ((d & 3) == 3) {
          const int base = d - 3;
          const double w[3] = {t.cx[S] - t.cx[b], t.cy[S] - t.cy[b], t.cz[S] - t.cz[b]};
          for (int k = 0; k < 3; ++k) {
            double2 u = src[(base + k) * T + f];
            v.x += w[k] * u.x;
            v.y += w[k] * u.y;
          }
        }
        int n = 0;
        while (tri(n + 1) <= f) ++n;
        const int m = f - tri(n);
        const double s = sm.sf[f];
        const C e = sm.E1[c * (p + 1) + m];
        double2 ed = make_double2((double)e.x, (double)e.y);
        v = cmul2(make_double2(v.x * s, v.y * s), ed);
        out.x = (R)v.x;
        out.y = (R)v.y;
      }
      sm.X[i] = out;
    }
    __syncthreads();
    dense_step(sm, p, RC, sm.X, sm.Y, false, 1, sm.E2);
    __syncthreads();
    dense_step(sm, p, RC, sm.Y, sm.X, true, 0, nullptr);
    __syncthreads();
    ztrans_step(sm, p, RC, sm.X, sm.Y);
    __syncthreads();
    dense_step(sm, p, RC, sm.Y, sm.X, false, 2, sm.E2);
    __syncthreads();
    dense_step(sm, p, RC, sm.X, sm.Y, true, 2, sm.E1);
    __syncthreads();
    // sum the columns of each density into this box's local expansion
    // (paper normalisation -> R-normalised storage, times s_k^l)
    for (int i = threadIdx.x; i < ND * T; i += ROT_T) {
      const int d = i / T, f = i % T;
      double ax = 0.0, ay = 0.0;
      bool any = false;
      for (int c = 0; c < RC; ++c)
        if (sm.colS[c] >= 0 && sm.colD[c] == d) {
          ax += (double)sm.Y[c * T + f].x;
          ay += (double)sm.Y[c * T + f].y;
          any = true;
        }
      if (any) {
        const double s = sm.sf[f];
        double2 v = Lb[i];
        Lb[i] = make_double2(v.x + ax * s, v.y + ay * s);
      }
    }
  }
}

static size_t rot_smem_bytes(int p, int RC, int rot_len, size_t real) {
  const int T = ncoef(p);
  return sizeof(double) * T + 2 * real * (rot_len + 2 * RC * T + 2 * RC * (p + 1)) + real * RC * (2 * p + 1) +
         sizeof(int) * (2 * RC + p + 2) + 16;
}

template <class R>
static hipError_t launch_rot(const Launch& l, int nrc, Exp e) {
  const Built* B = l.B;
  const int p = l.p;
  // 16 columns per chunk in FP32, 8 in FP64, fewer only if LDS runs out
  int RC = sizeof(R) == 4 ? 16 : 8;
  while (RC > 1 && rot_smem_bytes(p, RC, l.tb->rot_len, sizeof(R)) > 80 * 1024) RC /= 2;
  size_t shm = rot_smem_bytes(p, RC, l.tb->rot_len, sizeof(R));
  if (shm > 160 * 1024) return hipErrorInvalidValue;
  switch (nrc) {
    case 1: k_m2l_rot<4, R><<<B->tree.nbox, ROT_T, shm, l.s>>>(p, RC, B->tree, B->lists[LV], l.tb->rot, l.tb->rot_off, l.tb->rot_len, l.tb->sfac, l.tb->offtab, e.M, e.L); break;
    case 2: k_m2l_rot<8, R><<<B->tree.nbox, ROT_T, shm, l.s>>>(p, RC, B->tree, B->lists[LV], l.tb->rot, l.tb->rot_off, l.tb->rot_len, l.tb->sfac, l.tb->offtab, e.M, e.L); break;
    case 4: k_m2l_rot<16, R><<<B->tree.nbox, ROT_T, shm, l.s>>>(p, RC, B->tree, B->lists[LV], l.tb->rot, l.tb->rot_off, l.tb->rot_len, l.tb->sfac, l.tb->offtab, e.M, e.L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_m2l_rot(const Launch& l, int nrc, Exp e, int fp32) {
  return fp32 ? launch_rot<float>(l, nrc, e) : launch_rot<double>(l, nrc, e);
}

}  // namespace rpy
