// Scalar-field kernels: phase-field fracture (Sec. 2.1 eqs. (5)-(8),
// Sec. 3.2 eqs. (32)-(36), Alg. 2) and the backward-Euler Fick step (Sec. 2.2,
// Sec. 3.2 eqs. (42)-(50), Alg. 3).  All double precision.
//
// The phase-field and Fick operators are applied in real space with the
// 7-point / forward-backward difference stencils whose symbols are exactly
// the finite-difference frequencies of the paper (lambda(q) =
// sum_j (2/h_j)^2 sin^2(q_j/2); xi_j = (e^{i q_j} - 1)/h_j), i.e. the same
// linear maps; the constant-coefficient preconditioners go through the FFT.
#pragma once
#include "fg_pointwise.hpp"

namespace fg {

struct Grid3 {
  int n0, n1, n2;
  double ih0, ih1, ih2;  // 1 / h_j
};

__device__ __forceinline__ long vox(const Grid3& g, int i0, int i1, int i2) {
  return ((long)i0 * g.n1 + i1) * g.n2 + i2;
}

// Eigenvalues of a symmetric 3x3 matrix (closed form, trigonometric).
__device__ __forceinline__ void sym_eig3(double a00, double a11, double a22, double a01, double a02, double a12,
                                         double& e0, double& e1, double& e2) {
  const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
  const double q = (a00 + a11 + a22) / 3.0;
  const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
  const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1;
  if (!(p2 > 0.0)) {
    e0 = e1 = e2 = q;
    return;
  }
  const double p = sqrt(p2 / 6.0);
  const double ip = 1.0 / p;
  const double c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip;
  const double c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
  const double detc = c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02);
  double r = 0.5 * detc;
  r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
  const double phi = acos(r) / 3.0;
  e0 = q + 2.0 * p * cos(phi);
  e2 = q + 2.0 * p * cos(phi + 2.0943951023931957);  // + 2 pi / 3
  e1 = 3.0 * q - e0 - e2;
}

// History update (eqs. (7), (8)): effective Cauchy stress
//   sigma = J^-1 [ G s^-2 F F^T + (lambda ln J_e - G) I ]   (Neo-Hookean),
//   sigma = J^-1 s^-2 F S F^T                               (SVK),
// D_f = < sum <sigma_i>^2 / sigma_max^2 - 1 >, H <- max(H, gc/(2 lc) D_f).
// Writes the PFF coefficient a = gc/lc + 2H, the right-hand side b = 2H (into
// r), zeroes the solution x, and per-block partials of H (part_h) and b.b
// (part_b).
__global__ void __launch_bounds__(256)
k_pff_history(const double* __restrict__ F, const double* __restrict__ c, const double* __restrict__ E,
              const double* __restrict__ nu, const double* __restrict__ Om, const double* __restrict__ smax,
              double* __restrict__ H, double* __restrict__ acoef, double* __restrict__ r, double* __restrict__ x,
              double gc, double lc, double* __restrict__ part_h, double* __restrict__ part_b, int* flags, long N,
              int law) {
  __shared__ double red[16];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double hv = 0.0, bb = 0.0;
  if (i < N) {
    double f[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = F[k * N + i];
    double J = f[0] * (f[4] * f[8] - f[5] * f[7]) - f[1] * (f[3] * f[8] - f[5] * f[6]) +
               f[2] * (f[3] * f[7] - f[4] * f[6]);
    const double cc = c ? c[i] : 0.0;
    const double a = 1.0 + Om[i] * cc;
    if (!(J > 0.0) || !(a > 0.0)) {
      flags[0] = FG_FLAG_DOMAIN;
      J = 1.0;
    }
    const double EE = E[i], nn = nu[i];
    const double G = EE / (2.0 * (1.0 + nn));
    const double lam = EE * nn / ((1.0 + nn) * (1.0 - 2.0 * nn));
    const double la = log(a > 0.0 ? a : 1.0);
    const double s2inv = exp(-2.0 / 3.0 * la);
    const double lnJe = log(J) - la;
    const double iJ = 1.0 / J;
    // b = F F^T
    double b[9];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
        b[3 * ii + jj] = f[3 * ii] * f[3 * jj] + f[3 * ii + 1] * f[3 * jj + 1] + f[3 * ii + 2] * f[3 * jj + 2];
    const double sh = lam * lnJe - G;
    double s00 = (G * s2inv * b[0] + sh) * iJ, s11 = (G * s2inv * b[4] + sh) * iJ, s22 = (G * s2inv * b[8] + sh) * iJ;
    double s01 = G * s2inv * b[1] * iJ, s02 = G * s2inv * b[2] * iJ, s12 = G * s2inv * b[5] * iJ;
    if (law == kLawSVK) {
      // undegraded P_0 = s^-2 F S (d = 0), sigma = J^-1 P_0 F^T
      const SVKPoint q = svk_point(f, cc, 0.0, EE, nn, Om[i]);
      auto sg = [&](int ii, int jj) {
        return (q.P[3 * ii] * f[3 * jj] + q.P[3 * ii + 1] * f[3 * jj + 1] + q.P[3 * ii + 2] * f[3 * jj + 2]) * iJ;
      };
      s00 = sg(0, 0);
      s11 = sg(1, 1);
      s22 = sg(2, 2);
      s01 = sg(0, 1);
      s02 = sg(0, 2);
      s12 = sg(1, 2);
    }
    double e0, e1, e2;
    sym_eig3(s00, s11, s22, s01, s02, s12, e0, e1, e2);
    const double sm = smax[i];
    const double p0 = e0 > 0.0 ? e0 / sm : 0.0, p1 = e1 > 0.0 ? e1 / sm : 0.0, p2 = e2 > 0.0 ? e2 / sm : 0.0;
    double Df = p0 * p0 + p1 * p1 + p2 * p2 - 1.0;
    Df = Df > 0.0 ? Df : 0.0;
    double h = H[i];
    const double cand = gc / (2.0 * lc) * Df;
    h = cand > h ? cand : h;
    H[i] = h;
    acoef[i] = gc / lc + 2.0 * h;
    r[i] = 2.0 * h;
    x[i] = 0.0;
    hv = h;
    bb = 4.0 * h * h;
  }
  double s = block_sum(hv, red);
  if (threadIdx.x == 0) part_h[blockIdx.x] = s;
  s = block_sum(bb, red);
  if (threadIdx.x == 0) part_b[blockIdx.x] = s;
}

// q = A(p) = a p - k Lap_h p (7-point), partial sums of p.q.
__global__ void __launch_bounds__(256)
k_pff_apply(const double* __restrict__ p, const double* __restrict__ acoef, double kdiff, Grid3 g,
            double* __restrict__ q, double* __restrict__ partials, const KrylovScalars* __restrict__ ks, long N) {
  __shared__ double red[16];
  if (ks->done) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < N) {
    const int i2 = (int)(i % g.n2);
    const int i1 = (int)((i / g.n2) % g.n1);
    const int i0 = (int)(i / ((long)g.n2 * g.n1));
    const double pc = p[i];
    const double l0 = (2.0 * pc - p[vox(g, (i0 + 1) % g.n0, i1, i2)] - p[vox(g, (i0 + g.n0 - 1) % g.n0, i1, i2)]) *
                      g.ih0 * g.ih0;
    const double l1 = (2.0 * pc - p[vox(g, i0, (i1 + 1) % g.n1, i2)] - p[vox(g, i0, (i1 + g.n1 - 1) % g.n1, i2)]) *
                      g.ih1 * g.ih1;
    const double l2 = (2.0 * pc - p[vox(g, i0, i1, (i2 + 1) % g.n2)] - p[vox(g, i0, i1, (i2 + g.n2 - 1) % g.n2)]) *
                      g.ih2 * g.ih2;
    const double qv = acoef[i] * pc + kdiff * (l0 + l1 + l2);
    q[i] = qv;
    acc = pc * qv;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// PCG search direction p = z (first iteration) or z + beta p.
__global__ void __launch_bounds__(256)
k_pcg_dir(double* __restrict__ p, const double* __restrict__ z, const KrylovScalars* __restrict__ ks, long N) {
  if (ks->done) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  p[i] = (ks->iter == 0) ? z[i] : z[i] + ks->beta * p[i];
}

// ---------------------------------------------------------------- Fick ----
// Flux coefficient Aplus = -M(d) c_t (1 - c_t) C^-1 (6 components xx, yy, zz,
// yz, xz, xy; symmetric positive definite), with M(d) = -D/RT (0.9 (1-d)^2 +
// 0.1 d^2) (eq. (20)) and C = F^T F; partials of tr(Aplus) and of c_t.c_t.
__global__ void __launch_bounds__(256)
k_fick_coef(const double* __restrict__ F, const double* __restrict__ d, const double* __restrict__ ct,
            const double* __restrict__ D, double RT, double* __restrict__ A6, double* __restrict__ part_tr,
            double* __restrict__ part_c, long N) {
  __shared__ double red[16];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double tr = 0.0, cc = 0.0;
  if (i < N) {
    double f[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = F[k * N + i];
    // C = F^T F
    double C[9];
#pragma unroll
    for (int ii = 0; ii < 3; ++ii)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) C[3 * ii + jj] = f[ii] * f[jj] + f[3 + ii] * f[3 + jj] + f[6 + ii] * f[6 + jj];
    const double k00 = C[4] * C[8] - C[5] * C[7], k01 = C[2] * C[7] - C[1] * C[8], k02 = C[1] * C[5] - C[2] * C[4];
    const double k11 = C[0] * C[8] - C[2] * C[6], k12 = C[2] * C[3] - C[0] * C[5], k22 = C[0] * C[4] - C[1] * C[3];
    const double det = C[0] * k00 + C[1] * (C[5] * C[6] - C[3] * C[8]) + C[2] * (C[3] * C[7] - C[4] * C[6]);
    const double dd = d ? d[i] : 0.0;
    const double c = ct[i];
    const double mob = D[i] / RT * (0.9 * (1.0 - dd) * (1.0 - dd) + 0.1 * dd * dd);
    const double s = mob * c * (1.0 - c) / det;
    A6[0 * N + i] = s * k00;
    A6[1 * N + i] = s * k11;
    A6[2 * N + i] = s * k22;
    A6[3 * N + i] = s * k12;
    A6[4 * N + i] = s * k02;
    A6[5 * N + i] = s * k01;
    tr = s * (k00 + k11 + k22);
    cc = c * c;
  }
  double sm = block_sum(tr, red);
  if (threadIdx.x == 0) part_tr[blockIdx.x] = sm;
  sm = block_sum(cc, red);
  if (threadIdx.x == 0) part_c[blockIdx.x] = sm;
}

// Chemical potential mu = RT log(c/(1-c)) + mu_e / c_max with
//   mu_e = -g Omega / (3 (1 + Omega c)) [ G (s^-2 tr C - 3) + 3 lambda ln J_e ]
// (Neo-Hookean) or, for SVK with t = tr E_e, q = E_e : E_e,
//   mu_e = -g Omega / (3 (1 + Omega c)) [ 2 lambda t^2 + 4 G q + (3 lambda + 2 G) t ],
// the slope w = RT (1/c + 1/(1-c)) and partials of 1/w.  Flags c outside (0,1).
__global__ void __launch_bounds__(256)
k_fick_mu(const double* __restrict__ c, const double* __restrict__ F, const double* __restrict__ d,
          const double* __restrict__ E, const double* __restrict__ nu, const double* __restrict__ Om, double RT,
          double cmax, double* __restrict__ mu, double* __restrict__ w, double* __restrict__ part_winv, int* flags,
          long N, int full_jacobian, int law) {
  __shared__ double red[16];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double wi = 0.0;
  if (i < N) {
    double cc = c[i];
    if (!(cc > 0.0 && cc < 1.0)) {
      flags[0] = FG_FLAG_DOMAIN;
      cc = 0.5;
    }
    double f[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = F[k * N + i];
    double J = f[0] * (f[4] * f[8] - f[5] * f[7]) - f[1] * (f[3] * f[8] - f[5] * f[6]) +
               f[2] * (f[3] * f[7] - f[4] * f[6]);
    const double oo = Om[i];
    const double a = 1.0 + oo * cc;
    if (!(J > 0.0) || !(a > 0.0)) {
      flags[0] = FG_FLAG_DOMAIN;
      J = 1.0;
    }
    double trC = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) trC += f[k] * f[k];
    const double EE = E[i], nn = nu[i];
    const double G = EE / (2.0 * (1.0 + nn));
    const double lam = EE * nn / ((1.0 + nn) * (1.0 - 2.0 * nn));
    const double dd = d ? d[i] : 0.0;
    const double g = (1.0 - dd) * (1.0 - dd);
    const double la = log(a > 0.0 ? a : 1.0);
    const double s2inv = exp(-2.0 / 3.0 * la);
    const double lnJe = log(J) - la;
    double mue = -g * oo / (3.0 * a) * (G * (trC * s2inv - 3.0) + 3.0 * lam * lnJe);
    // d(mu_e / cmax)/dc at fixed F and d:
    // g Omega^2 / (3 a^2) [ (5/3) G a^(-2/3) tr C - 3 G + 3 lambda (ln J_e + 1) ] / cmax
    double dmue = g * oo * oo / (3.0 * a * a) * ((5.0 / 3.0) * G * s2inv * trC - 3.0 * G + 3.0 * lam * (lnJe + 1.0));
    if (law == kLawSVK) {
      const SVKPoint q = svk_point(f, cc, dd, EE, nn, oo);
      const double T = 2.0 * lam * q.t * q.t + 4.0 * G * q.q + (3.0 * lam + 2.0 * G) * q.t;
      mue = -g * oo / (3.0 * a) * T;
      // g Omega^2 / (3 a^2) [ T + ((4 lambda t + 3 lambda + 2 G)(2 t + 3) + 8 G (2 q + t)) / 3 ]
      dmue = g * oo * oo / (3.0 * a * a) *
             (T + ((4.0 * lam * q.t + 3.0 * lam + 2.0 * G) * (2.0 * q.t + 3.0) + 8.0 * G * (2.0 * q.q + q.t)) / 3.0);
    }
    mu[i] = RT * log(cc / (1.0 - cc)) + mue / cmax;
    double ww = RT * (1.0 / cc + 1.0 / (1.0 - cc));
    if (full_jacobian) {
      ww += dmue / cmax;
      if (!(ww > 0.0)) {
        flags[0] = FG_FLAG_DOMAIN;  // the linear step would not be SPD
        ww = RT * (1.0 / cc + 1.0 / (1.0 - cc));
      }
    }
    w[i] = ww;
    wi = 1.0 / ww;
  }
  const double s = block_sum(wi, red);
  if (threadIdx.x == 0) part_winv[blockIdx.x] = s;
}

// L(v) = grad+^T ( Aplus grad+ v ) at voxel i (forward differences, their
// adjoint for the divergence).  With div = -grad+^T and Aplus = -M c(1-c) C^-1
// this is div[ M c(1-c) C^-1 grad v ], the operator of eq. (43).
__device__ __forceinline__ double fick_L(const double* __restrict__ v, const double* __restrict__ A6, const Grid3& g,
                                         long N, int i0, int i1, int i2) {
  const int im[3] = {(i0 + g.n0 - 1) % g.n0, (i1 + g.n1 - 1) % g.n1, (i2 + g.n2 - 1) % g.n2};
  const double ih[3] = {g.ih0, g.ih1, g.ih2};
  const int ic[3] = {i0, i1, i2};
  // Aplus component index for (j, k)
  const int aidx[9] = {0, 5, 4, 5, 1, 3, 4, 3, 2};
  auto gradp = [&](int a0, int a1, int a2, double (&gr)[3]) {
    const double vc = v[vox(g, a0, a1, a2)];
    gr[0] = (v[vox(g, (a0 + 1) % g.n0, a1, a2)] - vc) * g.ih0;
    gr[1] = (v[vox(g, a0, (a1 + 1) % g.n1, a2)] - vc) * g.ih1;
    gr[2] = (v[vox(g, a0, a1, (a2 + 1) % g.n2)] - vc) * g.ih2;
  };
  double gr[3];
  gradp(i0, i1, i2, gr);
  const long ic_lin = vox(g, i0, i1, i2);
  double out = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    // flux_j(x) = sum_k A_jk(x) gr_k(x)
    double fx = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) fx += A6[aidx[3 * j + k] * N + ic_lin] * gr[k];
    // flux_j(x - e_j)
    int b[3] = {ic[0], ic[1], ic[2]};
    b[j] = im[j];
    double gm[3];
    gradp(b[0], b[1], b[2], gm);
    const long bl = vox(g, b[0], b[1], b[2]);
    double fm = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) fm += A6[aidx[3 * j + k] * N + bl] * gm[k];
    // grad+^T w = sum_j (w_j(x - e_j) - w_j(x)) / h_j
    out += (fm - fx) * ih[j];
  }
  return out;
}

// Fick residual: b = -f(c) = -(c - c_t + dt L(mu) - dt cdot_B), partials of b.b;
// also zeroes the solution x.
__global__ void __launch_bounds__(256)
k_fick_residual(const double* __restrict__ c, const double* __restrict__ ct, const double* __restrict__ mu,
                const double* __restrict__ A6, const double* __restrict__ cdot, double dt, Grid3 g,
                double* __restrict__ b, double* __restrict__ x, double* __restrict__ partials, long N) {
  __shared__ double red[16];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < N) {
    const int i2 = (int)(i % g.n2);
    const int i1 = (int)((i / g.n2) % g.n1);
    const int i0 = (int)(i / ((long)g.n2 * g.n1));
    const double f = c[i] - ct[i] + dt * fick_L(mu, A6, g, N, i0, i1, i2) - dt * (cdot ? cdot[i] : 0.0);
    b[i] = -f;
    x[i] = 0.0;
    acc = f * f;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// q = B(p) = p / w + dt L(p), partials of p.q.
__global__ void __launch_bounds__(256)
k_fick_apply(const double* __restrict__ p, const double* __restrict__ w, const double* __restrict__ A6, double dt,
             Grid3 g, double* __restrict__ q, double* __restrict__ partials, const KrylovScalars* __restrict__ ks,
             long N) {
  __shared__ double red[16];
  if (ks->done) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < N) {
    const int i2 = (int)(i % g.n2);
    const int i1 = (int)((i / g.n2) % g.n1);
    const int i0 = (int)(i / ((long)g.n2 * g.n1));
    const double pc = p[i];
    const double qv = pc / w[i] + dt * fick_L(p, A6, g, N, i0, i1, i2);
    q[i] = qv;
    acc = pc * qv;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// c += dmu / w, partials of dc.dc.
__global__ void __launch_bounds__(256)
k_fick_update(double* __restrict__ c, const double* __restrict__ dmu, const double* __restrict__ w,
              double* __restrict__ partials, long N) {
  __shared__ double red[16];
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < N) {
    const double dc = dmu[i] / w[i];
    c[i] += dc;
    acc = dc * dc;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

}  // namespace fg
