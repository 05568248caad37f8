// The tangent contraction K : X of the compressible Neo-Hookean law with
// swelling and degradation (Sec. 2; eq. (30), K = dP/dF), evaluated from the
// 12-word state {A = F^-T, alpha, beta, gamma}:
//   K : X = alpha X + beta (A : X) A + gamma A X^T A.
#pragma once
#include <hip/hip_runtime.h>

namespace fg {

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

}  // namespace fg
