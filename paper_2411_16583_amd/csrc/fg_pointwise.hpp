// Pointwise and vector kernels of the mechanics path.
//
// Field layout: component-major, a 3x3 tensor field is 9 planes of N voxels,
// plane 3i+j holds the ij component (row-major tensor index).
#pragma once
#include "fg_fft.hpp"
#include "fg_tangent.hpp"

namespace fg {

constexpr int FG_FLAG_DOMAIN = 1;  // det F <= 0 or 1 + Omega c <= 0

// Compressible Neo-Hookean point (Sec. 2, eqs. (1), (2), (9), (11), (27);
// energy per reference volume):
//   s^-2 = (1 + Omega c)^{-2/3}, ln J_e = ln det F - ln(1 + Omega c),
//   P = g [ G s^-2 F + (lambda ln J_e - G) F^-T ],  g = (1 - d)^2,
// and the 12-word tangent state {A = F^-T, alpha = g G s^-2, beta = g lambda,
// gamma = g (G - lambda ln J_e)} with which
//   K : X = alpha X + beta (A : X) A + gamma A X^T A.
// ok = false when det F <= 0 or 1 + Omega c <= 0 (then J = 1 is used).
struct NHPoint {
  double A[9];
  double c1, c2;             // P = c1 F + c2 A
  double alpha, beta, gamma;  // tangent scalars
  bool ok;
};

__device__ __forceinline__ NHPoint neo_hooke_point(const double (&f)[9], double cc, double dd, double EE, double nn,
                                                   double oo) {
  NHPoint q;
  // cofactor matrix: F^-T = cof(F) / det F
  double cof[9];
  cof[0] = f[4] * f[8] - f[5] * f[7];
  cof[1] = f[5] * f[6] - f[3] * f[8];
  cof[2] = f[3] * f[7] - f[4] * f[6];
  cof[3] = f[2] * f[7] - f[1] * f[8];
  cof[4] = f[0] * f[8] - f[2] * f[6];
  cof[5] = f[1] * f[6] - f[0] * f[7];
  cof[6] = f[1] * f[5] - f[2] * f[4];
  cof[7] = f[2] * f[3] - f[0] * f[5];
  cof[8] = f[0] * f[4] - f[1] * f[3];
  double J = f[0] * cof[0] + f[1] * cof[1] + f[2] * cof[2];
  const double a = 1.0 + oo * cc;
  q.ok = (J > 0.0) && (a > 0.0);
  if (!q.ok) J = 1.0;
  const double G = EE / (2.0 * (1.0 + nn));
  const double lam = EE * nn / ((1.0 + nn) * (1.0 - 2.0 * nn));
  const double g = (1.0 - dd) * (1.0 - dd);
  const double la = log(a > 0.0 ? a : 1.0);
  const double s2inv = exp(-2.0 / 3.0 * la);
  const double lnJe = log(J) - la;
  const double iJ = 1.0 / J;
#pragma unroll
  for (int k = 0; k < 9; ++k) q.A[k] = cof[k] * iJ;
  q.c1 = g * G * s2inv;
  q.c2 = g * (lam * lnJe - G);
  q.alpha = q.c1;
  q.beta = g * lam;
  q.gamma = g * (G - lam * lnJe);
  return q;
}

// Saint-Venant-Kirchhoff point (Sec. 2.1 eqs. (3), (4), (11), (12) with the
// swelling of eq. (2); energy per reference volume, F_e = F / s):
//   E_e = (s^-2 F^T F - I) / 2,  S = lambda tr E_e I + 2 G E_e,
//   P = g s^-2 F S   (eq. (12) when Omega c = 0),
// the tangent state {St = g s^-2 S, lp = g s^-4 lambda, mp = g s^-4 G} of
// svk_apply, and dP/dOmega = g s^-2 F [ -(2c/3a) S + lambda tr(dE) I + 2 G dE ]
// with dE = -(c/3a)(2 E_e + I), a = 1 + Omega c.
// ok = false when 1 + Omega c <= 0 (then a = 1 is used).
struct SVKPoint {
  double P[9];
  double St[6];  // 00 11 22 12 02 01
  double lp, mp;
  double t, q;   // tr E_e, E_e : E_e
  double e[6];   // E_e
  double S[6];   // undegraded S
  double s2inv, g, a, lam, G;
  bool ok;
};

__device__ __forceinline__ SVKPoint svk_point(const double (&f)[9], double cc, double dd, double EE, double nn,
                                              double oo) {
  SVKPoint q;
  double a = 1.0 + oo * cc;
  q.ok = a > 0.0;
  if (!q.ok) a = 1.0;
  q.a = a;
  q.G = EE / (2.0 * (1.0 + nn));
  q.lam = EE * nn / ((1.0 + nn) * (1.0 - 2.0 * nn));
  q.g = (1.0 - dd) * (1.0 - dd);
  q.s2inv = exp(-2.0 / 3.0 * log(a));
  // C = F^T F (symmetric): C_mn = sum_k F_km F_kn
  auto Cmn = [&](int m, int n) { return f[m] * f[n] + f[3 + m] * f[3 + n] + f[6 + m] * f[6 + n]; };
  const double e00 = 0.5 * (q.s2inv * Cmn(0, 0) - 1.0), e11 = 0.5 * (q.s2inv * Cmn(1, 1) - 1.0),
               e22 = 0.5 * (q.s2inv * Cmn(2, 2) - 1.0);
  const double e12 = 0.5 * q.s2inv * Cmn(1, 2), e02 = 0.5 * q.s2inv * Cmn(0, 2), e01 = 0.5 * q.s2inv * Cmn(0, 1);
  q.e[0] = e00;
  q.e[1] = e11;
  q.e[2] = e22;
  q.e[3] = e12;
  q.e[4] = e02;
  q.e[5] = e01;
  q.t = e00 + e11 + e22;
  q.q = e00 * e00 + e11 * e11 + e22 * e22 + 2.0 * (e12 * e12 + e02 * e02 + e01 * e01);
  const double lt = q.lam * q.t, G2 = 2.0 * q.G;
  q.S[0] = lt + G2 * e00;
  q.S[1] = lt + G2 * e11;
  q.S[2] = lt + G2 * e22;
  q.S[3] = G2 * e12;
  q.S[4] = G2 * e02;
  q.S[5] = G2 * e01;
  const double gs = q.g * q.s2inv;
#pragma unroll
  for (int k = 0; k < 6; ++k) q.St[k] = gs * q.S[k];
  q.lp = gs * q.s2inv * q.lam;
  q.mp = gs * q.s2inv * q.G;
  const double Sm[9] = {q.St[0], q.St[5], q.St[4], q.St[5], q.St[1], q.St[3], q.St[4], q.St[3], q.St[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      q.P[3 * i + j] = f[3 * i] * Sm[j] + f[3 * i + 1] * Sm[3 + j] + f[3 * i + 2] * Sm[6 + j];
  return q;
}

// dP/dOmega of the SVK law at fixed F (q from svk_point at the same point).
__device__ __forceinline__ void svk_dP_dOmega(const SVKPoint& q, const double (&f)[9], double cc, double (&o)[9]) {
  const double k = cc / (3.0 * q.a);
  const double(&e)[6] = q.e;
  // dE = -k (2 E_e + I)
  const double de[6] = {-k * (2.0 * e[0] + 1.0), -k * (2.0 * e[1] + 1.0), -k * (2.0 * e[2] + 1.0),
                        -k * 2.0 * e[3],         -k * 2.0 * e[4],         -k * 2.0 * e[5]};
  const double ltd = q.lam * (de[0] + de[1] + de[2]);
  const double m = -2.0 * k;  // -(2c / 3a)
  const double in6[6] = {m * q.S[0] + ltd + 2.0 * q.G * de[0], m * q.S[1] + ltd + 2.0 * q.G * de[1],
                         m * q.S[2] + ltd + 2.0 * q.G * de[2], m * q.S[3] + 2.0 * q.G * de[3],
                         m * q.S[4] + 2.0 * q.G * de[4],       m * q.S[5] + 2.0 * q.G * de[5]};
  const double In[9] = {in6[0], in6[5], in6[4], in6[5], in6[1], in6[3], in6[4], in6[3], in6[2]};
  const double gs = q.g * q.s2inv;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      o[3 * i + j] = gs * (f[3 * i] * In[j] + f[3 * i + 1] * In[3 + j] + f[3 * i + 2] * In[6 + j]);
}

// Constitutive update over the field: P (FP64) and the tangent state (type
// S).  F is either the field F (9 planes) or, when Fu != nullptr, the uniform
// tensor Fu.  P may be nullptr; state may be nullptr.  pnorm_partials
// (optional) receives per-block sums of P : P.
template <typename S>
__global__ void __launch_bounds__(256)
k_constitutive(const double* __restrict__ F, const double* __restrict__ Fu, const double* __restrict__ c,
               const double* __restrict__ d, const double* __restrict__ E, const double* __restrict__ nu,
               const double* __restrict__ Om, double* __restrict__ P, S* __restrict__ state,
               double* __restrict__ pnorm_partials, int* __restrict__ flags, long N,
               const int* __restrict__ idle, int law) {
  // voxel i of batch item b = blockIdx.y (item-major fields: material, c and
  // d at b N + i, tensor fields at (9 b + k) N + i, Fu per item); items with
  // idle[b] != 0 are left alone (idle may be nullptr); partial sums at
  // b gridDim.x + blockIdx.x
  __shared__ double red[16];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long b = blockIdx.y;
  if (idle && idle[b]) return;
  double pp = 0.0;
  if (i < N) {
    F += b * 9 * N;
    if (Fu) Fu += 9 * b;
    if (P) P += b * 9 * N;
    if (state) state += b * state_words(law) * N;
    c += b * N;
    d += b * N;
    E += b * N;
    nu += b * N;
    Om += b * N;
    double f[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = Fu ? Fu[k] : F[k * N + i];
    if (law == kLawSVK) {
      const SVKPoint q = svk_point(f, c[i], d[i], E[i], nu[i], Om[i]);
      if (!q.ok) flags[0] = FG_FLAG_DOMAIN;
      if (P) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          P[k * N + i] = q.P[k];
          pp += q.P[k] * q.P[k];
        }
      }
      if (state) {
#pragma unroll
        for (int k = 0; k < 9; ++k) state[k * N + i] = (S)f[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) state[(9 + k) * N + i] = (S)q.St[k];
        state[15 * N + i] = (S)q.lp;
        state[16 * N + i] = (S)q.mp;
        state[17 * N + i] = (S)0;
      }
    } else {
      const NHPoint q = neo_hooke_point(f, c[i], d[i], E[i], nu[i], Om[i]);
      if (!q.ok) flags[0] = FG_FLAG_DOMAIN;
      if (P) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const double pk = q.c1 * f[k] + q.c2 * q.A[k];
          P[k * N + i] = pk;
          pp += pk * pk;
        }
      }
      if (state) {
#pragma unroll
        for (int k = 0; k < 9; ++k) state[k * N + i] = (S)q.A[k];
        state[9 * N + i] = (S)q.alpha;
        state[10 * N + i] = (S)q.beta;
        state[11 * N + i] = (S)q.gamma;
      }
    }
  }
  if (pnorm_partials) {
    const double s = block_sum(pp, red);
    if (threadIdx.x == 0) pnorm_partials[b * gridDim.x + blockIdx.x] = s;
  }
}

// Y = K(F) : (W + X) in double precision with the tangent evaluated from F
// on the fly (no stored state): W uniform (9, device), X a 9-plane field.
__global__ void __launch_bounds__(256)
k_tangent_apply_f64(const double* __restrict__ F, const double* __restrict__ c, const double* __restrict__ d,
                    const double* __restrict__ E, const double* __restrict__ nu, const double* __restrict__ Om,
                    const double* __restrict__ W, const double* __restrict__ X, double* __restrict__ Y,
                    int* __restrict__ flags, long N, int law) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double f[9], x[9], y[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    f[k] = F[k * N + i];
    x[k] = W[k] + X[k * N + i];
  }
  if (law == kLawSVK) {
    const SVKPoint q = svk_point(f, c[i], d[i], E[i], nu[i], Om[i]);
    if (!q.ok) flags[0] = FG_FLAG_DOMAIN;
    svk_apply<double>(f, q.St, q.lp, q.mp, x, y);
  } else {
    const NHPoint q = neo_hooke_point(f, c[i], d[i], E[i], nu[i], Om[i]);
    if (!q.ok) flags[0] = FG_FLAG_DOMAIN;
    tangent_apply<double>(q.A, q.alpha, q.beta, q.gamma, x, y);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) Y[k * N + i] = y[k];
}

// Tangent contraction Y = K : X from the tangent state (12 words for the
// Neo-Hookean law, 18 for SVK; one application of K outside the CG, e.g.
// the operator diagnostic and the adjoint's right-hand side).  Two voxels per
// thread (one 2-vector load per plane); N is even.
template <typename T, int LAW>
__global__ void __launch_bounds__(256)
k_contract(T* __restrict__ Y, const T* __restrict__ X, const T* __restrict__ st, long N) {
  using V = cplx<T>;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long N2v = N / 2;
  if (i >= N2v) return;
  const V* xv = reinterpret_cast<const V*>(X);
  const V* sv = reinterpret_cast<const V*>(st);
  V* yv = reinterpret_cast<V*>(Y);
  T X0[9], X1[9], A0[9], A1[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const V x = xv[k * N2v + i];
    const V a = sv[k * N2v + i];
    X0[k] = x.x;
    X1[k] = x.y;
    A0[k] = a.x;
    A1[k] = a.y;
  }
  T Y0[9], Y1[9];
  if constexpr (LAW == kLawSVK) {
    T S0[6], S1[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const V a = sv[(9 + k) * N2v + i];
      S0[k] = a.x;
      S1[k] = a.y;
    }
    const V lp = sv[15 * N2v + i], mp = sv[16 * N2v + i];
    svk_apply<T>(A0, S0, lp.x, mp.x, X0, Y0);
    svk_apply<T>(A1, S1, lp.y, mp.y, X1, Y1);
  } else {
    const V al = sv[9 * N2v + i], be = sv[10 * N2v + i], ga = sv[11 * N2v + i];
    tangent_apply<T>(A0, al.x, be.x, ga.x, X0, Y0);
    tangent_apply<T>(A1, al.y, be.y, ga.y, X1, Y1);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) yv[k * N2v + i] = mk<V>(Y0[k], Y1[k]);
}

// 16-byte vector of the working precision (2 doubles or 4 floats).
template <typename T> struct vec16;
template <> struct vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};
template <> struct vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};

template <typename T, typename V> __device__ __forceinline__ T vget(const V& v, int k) {
  if constexpr (sizeof(V) == 16 && sizeof(T) == 8) {
    return k == 0 ? v.x : v.y;
  } else {
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
  }
}
template <typename T, typename V> __device__ __forceinline__ void vset(V& v, int k, T a) {
  if constexpr (sizeof(V) == 16 && sizeof(T) == 8) {
    if (k == 0) v.x = a; else v.y = a;
  } else {
    if (k == 0) v.x = a; else if (k == 1) v.y = a; else if (k == 2) v.z = a; else v.w = a;
  }
}

// x += alpha p, r -= alpha q, per-block partial sums of r.r.  16-byte
// accesses; n must be a multiple of the vector width (the scalar fields of
// the preconditioned solvers: N is even).
template <typename T>
__global__ void __launch_bounds__(256)
k_cg_update(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
            const KrylovScalars* __restrict__ ks, double* __restrict__ partials, long n) {
  using V = typename vec16<T>::type;
  constexpr int W = vec16<T>::n;
  __shared__ double red[16];
  if (ks->done) return;
  const T alpha = (T)ks->alpha;
  double acc = 0.0;
  const long nv = n / W;
  V* xv = reinterpret_cast<V*>(x);
  V* rv = reinterpret_cast<V*>(r);
  const V* pv = reinterpret_cast<const V*>(p);
  const V* qv = reinterpret_cast<const V*>(q);
  const long stride = (long)gridDim.x * blockDim.x;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + stride < nv; i += 2 * stride) {
    V xa = xv[i], ra = rv[i], pa = pv[i], qa = qv[i];
    V xb = xv[i + stride], rb = rv[i + stride], pb = pv[i + stride], qb = qv[i + stride];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      vset(xa, k, (T)(vget<T>(xa, k) + alpha * vget<T>(pa, k)));
      const T ta = vget<T>(ra, k) - alpha * vget<T>(qa, k);
      vset(ra, k, ta);
      acc += (double)ta * (double)ta;
      vset(xb, k, (T)(vget<T>(xb, k) + alpha * vget<T>(pb, k)));
      const T tb = vget<T>(rb, k) - alpha * vget<T>(qb, k);
      vset(rb, k, tb);
      acc += (double)tb * (double)tb;
    }
    xv[i] = xa;
    rv[i] = ra;
    xv[i + stride] = xb;
    rv[i + stride] = rb;
  }
  for (; i < nv; i += stride) {
    V xa = xv[i], ra = rv[i], pa = pv[i], qa = qv[i];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      vset(xa, k, (T)(vget<T>(xa, k) + alpha * vget<T>(pa, k)));
      const T ta = vget<T>(ra, k) - alpha * vget<T>(qa, k);
      vset(ra, k, ta);
      acc += (double)ta * (double)ta;
    }
    xv[i] = xa;
    rv[i] = ra;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// mode 0: alpha = rz / pAp (rz = rr for plain CG), breakdown check.
// mode 1: plain CG: rr_new, iteration count, convergence, beta.
// mode 2: store the sum into out[0] (norms).
// mode 3: PCG: r.r (convergence) -- z not yet formed.
// mode 4: PCG: r.z -> beta = rz_new / rz.
// mode 5: initialise a Krylov solve from rr0 = sum (b.b): rr = rr0, iter = 0.
__global__ void __launch_bounds__(1024)
k_finalize(const double* __restrict__ partials, int nparts, KrylovScalars* ks, double* out, int mode, int pcg) {
  // one workgroup per batch item: nparts partials, scalars and output each
  __shared__ double red[16];
  partials += (long)blockIdx.x * nparts;
  if (ks) ks += blockIdx.x;
  if (out) out += blockIdx.x;
  if (ks && ks->done && mode != 5 && mode != 2) return;
  const double s = sum_partials(partials, nparts, red);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    krylov_alpha(ks, s, pcg);
  } else if (mode == 1) {
    const double rr = s;
    ks->iter += 1;
    // beta is kept even when the solve stops here, so that a solve stopped
    // at a fixed iteration count can be continued
    ks->beta = rr / ks->rr;
    if (ks->tol2 > 0.0 && rr <= ks->tol2 * ks->rr0) {
      ks->done = 1;
    } else if (ks->iter >= ks->maxit) {
      ks->done = 1;
      ks->flag = (ks->tol2 > 0.0) ? 2 : 0;
    }
    ks->rr = rr;
  } else if (mode == 2) {
    out[0] = s;
  } else if (mode == 3) {
    ks->iter += 1;
    ks->rr = s;
    if (ks->tol2 > 0.0 && s <= ks->tol2 * ks->rr0) {
      ks->done = 1;
    } else if (ks->iter >= ks->maxit) {
      ks->done = 1;
      ks->flag = (ks->tol2 > 0.0) ? 2 : 0;
    }
  } else if (mode == 4) {
    if (ks->iter == 0) {
      ks->beta = 0.0;
    } else {
      ks->beta = s / ks->rz;
    }
    ks->rz = s;
  } else if (mode == 5) {
    ks->rr0 = s;
    ks->rr = s;
    ks->iter = 0;
    ks->flag = 0;
    ks->beta = 0.0;
    ks->done = (s == 0.0) ? 1 : 0;
  }
}

// F += x (F FP64, x in the CG precision), n = 9N.
template <typename T>
__global__ void __launch_bounds__(256) k_axpy_into_f64(double* __restrict__ F, const T* __restrict__ x, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) F[i] += (double)x[i];
}

// a -= b (double precision), n values.
__global__ void __launch_bounds__(256) k_sub_f64(double* __restrict__ a, const double* __restrict__ b, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] -= b[i];
}

// F_k += dF_k for a uniform 3x3 increment per batch item (dF: 9 per item).
__global__ void __launch_bounds__(256) k_add_uniform9(double* __restrict__ F, const double* __restrict__ dF, long N,
                                                      long Ntot) {
  const long gi = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= Ntot) return;
  const long b = gi / N, i = gi - b * N;
#pragma unroll
  for (int k = 0; k < 9; ++k) F[(9 * b + k) * N + i] += dF[9 * b + k];
}

template <typename A, typename B>
__global__ void __launch_bounds__(256) k_convert(B* __restrict__ dst, const A* __restrict__ src, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = (B)src[i];
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ dst, T v, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = v;
}

// Uniform 3x3 tensor field: dst plane k = w[k] (w: 9 doubles, device).
template <typename T>
__global__ void __launch_bounds__(256) k_fill_uniform9(T* __restrict__ dst, const double* __restrict__ w, long N) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[k * N + i] = (T)w[k];
}

// Adjoint gradient (derived from eq. (30); L = sum_ij W_ij <P_ij>):
//   dL/dlogE(x) = (W + lam(x)) : P(x) / N,
//   dL/dOmega(x) = (W + lam(x)) : dP/dOmega(x) / N,
// dP/dlogE = P (both Lame constants scale with E) and
//   dP/dOmega = g [ -(2/3) G c (1 + Omega c)^{-5/3} F - lambda c / (1 + Omega c) F^-T ]
// for the Neo-Hookean law (svk_dP_dOmega for SVK).
template <typename T>
__global__ void __launch_bounds__(256)
k_adjoint_grad(const double* __restrict__ F, const double* __restrict__ c, const double* __restrict__ d,
               const double* __restrict__ E, const double* __restrict__ nu, const double* __restrict__ Om,
               const T* __restrict__ lam, const double* __restrict__ W, double* __restrict__ gE,
               double* __restrict__ gO, int* __restrict__ flags, long N, int law) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double f[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) f[k] = F[k * N + i];
  if (law == kLawSVK) {
    const SVKPoint q = svk_point(f, c[i], d[i], E[i], nu[i], Om[i]);
    if (!q.ok) flags[0] = FG_FLAG_DOMAIN;
    double o[9];
    svk_dP_dOmega(q, f, c[i], o);
    double sE = 0.0, sO = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double w = W[k] + (double)lam[k * N + i];
      sE += w * q.P[k];
      sO += w * o[k];
    }
    const double invN = 1.0 / (double)N;
    if (gE) gE[i] = sE * invN;
    if (gO) gO[i] = sO * invN;
    return;
  }
  double cof[9];
  cof[0] = f[4] * f[8] - f[5] * f[7];
  cof[1] = f[5] * f[6] - f[3] * f[8];
  cof[2] = f[3] * f[7] - f[4] * f[6];
  cof[3] = f[2] * f[7] - f[1] * f[8];
  cof[4] = f[0] * f[8] - f[2] * f[6];
  cof[5] = f[1] * f[6] - f[0] * f[7];
  cof[6] = f[1] * f[5] - f[2] * f[4];
  cof[7] = f[2] * f[3] - f[0] * f[5];
  cof[8] = f[0] * f[4] - f[1] * f[3];
  double J = f[0] * cof[0] + f[1] * cof[1] + f[2] * cof[2];
  const double cc = c[i], dd = d[i], EE = E[i], nn = nu[i], oo = Om[i];
  const double a = 1.0 + oo * cc;
  if (!(J > 0.0) || !(a > 0.0)) {
    flags[0] = FG_FLAG_DOMAIN;
    J = 1.0;
  }
  const double G = EE / (2.0 * (1.0 + nn));
  const double lm = EE * nn / ((1.0 + nn) * (1.0 - 2.0 * nn));
  const double g = (1.0 - dd) * (1.0 - dd);
  const double la = log(a > 0.0 ? a : 1.0);
  const double s2inv = exp(-2.0 / 3.0 * la);
  const double lnJe = log(J) - la;
  const double iJ = 1.0 / J;
  const double c1 = g * G * s2inv, c2 = g * (lm * lnJe - G);
  const double o1 = -g * (2.0 / 3.0) * G * cc * s2inv / (a > 0.0 ? a : 1.0);  // (1+Oc)^{-5/3}
  const double o2 = -g * lm * cc / (a > 0.0 ? a : 1.0);
  double sE = 0.0, sO = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double A = cof[k] * iJ;
    const double w = W[k] + (double)lam[k * N + i];
    sE += w * (c1 * f[k] + c2 * A);
    sO += w * (o1 * f[k] + o2 * A);
  }
  const double invN = 1.0 / (double)N;
  if (gE) gE[i] = sE * invN;
  if (gO) gO[i] = sO * invN;
}

// Per-block partial sums of the 9 components of a tensor field (for <P>),
// batch item b = blockIdx.y: partials[(k gridDim.y + b) gridDim.x + block].
__global__ void __launch_bounds__(256) k_mean9_partials(const double* __restrict__ P, double* __restrict__ partials,
                                                        long N) {
  __shared__ double red[16];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long b = blockIdx.y;
  for (int k = 0; k < 9; ++k) {
    const double v = (i < N) ? P[(9 * b + k) * N + i] : 0.0;
    const double s = block_sum(v, red);
    if (threadIdx.x == 0) partials[((long)k * gridDim.y + b) * gridDim.x + blockIdx.x] = s;
  }
}

}  // namespace fg
