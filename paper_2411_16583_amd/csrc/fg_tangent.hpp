// Tangent contractions K : X of the two material laws.
//
// The tangent contraction K : X of the compressible Neo-Hookean law with
// swelling and degradation (Sec. 2; eq. (30), K = dP/dF), evaluated from the
// 12-word state {A = F^-T, alpha, beta, gamma}:
//   K : X = alpha X + beta (A : X) A + gamma A X^T A.
#pragma once
#include <hip/hip_runtime.h>

namespace fg {

constexpr int kLawNH = 0;   // compressible Neo-Hookean (12-word tangent state)
constexpr int kLawSVK = 1;  // Saint-Venant-Kirchhoff (18-word tangent state)
__host__ __device__ constexpr int state_words(int law) { return law == kLawSVK ? 18 : 12; }

// K : X from the tangent state (in registers).
template <typename T>
__device__ __forceinline__ void tangent_apply(const T (&A)[9], T al, T be, T ga, const T (&X)[9], T (&Y)[9]) {
  T tr = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) tr += A[k] * X[k];
  // W = A X^T : W_ik = sum_l A_il X_kl
  T W[9];
#pragma unroll
  for (int ii = 0; ii < 3; ++ii)
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
      W[3 * ii + kk] = A[3 * ii] * X[3 * kk] + A[3 * ii + 1] * X[3 * kk + 1] + A[3 * ii + 2] * X[3 * kk + 2];
#pragma unroll
  for (int ii = 0; ii < 3; ++ii)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      const T awa = W[3 * ii] * A[jj] + W[3 * ii + 1] * A[3 + jj] + W[3 * ii + 2] * A[6 + jj];
      Y[3 * ii + jj] = al * X[3 * ii + jj] + be * tr * A[3 * ii + jj] + ga * awa;
    }
}

// Saint-Venant-Kirchhoff tangent contraction (eq. (12) differentiated, with
// the swelling split of eq. (2) and the degradation g), evaluated from the
// 18-word state {F (9), St = g s^-2 S (6: 00 11 22 12 02 01), lp = g s^-4
// lambda, mp = g s^-4 G, one unused word}:
//   K : X = X St + F (lp tr(W) I + mp (W + W^T)),   W = F^T X.
template <typename T>
__device__ __forceinline__ void svk_apply(const T (&F)[9], const T (&St)[6], T lp, T mp, const T (&X)[9],
                                          T (&Y)[9]) {
  // W = F^T X : W_mn = sum_k F_km X_kn
  T W[9];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int n = 0; n < 3; ++n) W[3 * m + n] = F[m] * X[n] + F[3 + m] * X[3 + n] + F[6 + m] * X[6 + n];
  const T tw = lp * (W[0] + W[4] + W[8]);
  // Sigma = lp tr(W) I + mp (W + W^T), symmetric
  const T s00 = tw + T(2) * mp * W[0], s11 = tw + T(2) * mp * W[4], s22 = tw + T(2) * mp * W[8];
  const T s12 = mp * (W[5] + W[7]), s02 = mp * (W[2] + W[6]), s01 = mp * (W[1] + W[3]);
  const T Sg[9] = {s00, s01, s02, s01, s11, s12, s02, s12, s22};
  const T Sm[9] = {St[0], St[5], St[4], St[5], St[1], St[3], St[4], St[3], St[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Y[3 * i + j] = X[3 * i] * Sm[j] + X[3 * i + 1] * Sm[3 + j] + X[3 * i + 2] * Sm[6 + j] + F[3 * i] * Sg[j] +
                     F[3 * i + 1] * Sg[3 + j] + F[3 * i + 2] * Sg[6 + j];
}

}  // namespace fg
