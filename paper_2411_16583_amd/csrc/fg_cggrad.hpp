// Back end of one CG iteration in the potential form of the projection
// (k_fft_z_grad3): the projected field G(K p) = D U is formed from the real
// 3-component potential U by the corner stencil of the rotated scheme and
// used at once, so the 9-component field is never transformed back:
//   (D_j U_i)[n] = 1/(4 h_j) * sum over the four voxel edges parallel to
//                  axis j of (U_i at the upper corner - U_i at the lower one),
// with the corner n - 1/2 (in every axis) stored at index n - 1 (periodic).
//   mode 0 (CG):  r <- r - alpha D U (alpha of the item), per-block partial
//                 sums of the new r . r;
//   mode 1:       r <- D U (the projection itself; r is the output).
// U: component slots 0, 3, 6 of the item's 9-component buffer (real after
// the inverse passes).  Grid (ceil(N / (256 W)), items), one thread per W
// consecutive voxels along N2.
#pragma once
#include "fg_fft.hpp"

namespace fg {

// W consecutive voxels of a line per thread (W = 4 in single precision when
// N2 % 4 == 0, else 2): one W-vector access per plane and line.
template <typename T, int W> struct GradPack;
template <> struct GradPack<double, 2> { using type = double2; };
template <> struct GradPack<float, 2> { using type = float2; };
template <> struct GradPack<float, 4> { using type = float4; };

template <typename T, int W>
__global__ void __launch_bounds__(256)
k_cg_grad(const T* __restrict__ U, T* __restrict__ r, const KrylovScalars* __restrict__ ks,
          double* __restrict__ partials, int n0, int n1, int n2, T ih0, T ih1, T ih2, int mode) {
  using V = typename GradPack<T, W>::type;
  __shared__ double red[16];
  const int item = blockIdx.y;
  if (mode == 0 && ks[item].done) return;
  const long N = (long)n0 * n1 * n2;
  U += (long)item * 9 * N;
  r += (long)item * 9 * N;
  const int G = n2 / W;  // voxel groups per line
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (g < N / W) {
    const long line = g / G;
    const int x = W * (int)(g - line * G);
    const int i0 = (int)(line / n1), i1 = (int)(line - (long)i0 * n1);
    const int i0m = (i0 == 0) ? n0 - 1 : i0 - 1;
    const int i1m = (i1 == 0) ? n1 - 1 : i1 - 1;
    const int xm = (x == 0) ? n2 - 1 : x - 1;
    // the four lines (i0 - a, i1 - b), a, b in {0, 1}
    const long row[2][2] = {{((long)i0 * n1 + i1) * n2, ((long)i0 * n1 + i1m) * n2},
                            {((long)i0m * n1 + i1) * n2, ((long)i0m * n1 + i1m) * n2}};
    const T alpha = (mode == 0) ? (T)ks[item].alpha : T(0);
    const T q0 = T(0.25) * ih0, q1 = T(0.25) * ih1, q2 = T(0.25) * ih2;
    V* rv = reinterpret_cast<V*>(r);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T* Uc = U + 3 * c * N;
      // u[a][b][p]: corner values at x - 1 + p, p = 0..W
      T u[2][2][W + 1];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const V w = *reinterpret_cast<const V*>(Uc + row[a][b] + x);
          u[a][b][0] = Uc[row[a][b] + xm];
#pragma unroll
          for (int q = 0; q < W; ++q) u[a][b][q + 1] = reinterpret_cast<const T*>(&w)[q];
        }
      T Z[3][W];
#pragma unroll
      for (int v = 0; v < W; ++v) {
        const int lo = v, hi = v + 1;  // corners below / above voxel x + v along N2
        Z[0][v] = q0 * ((u[0][0][hi] + u[0][1][hi] + u[0][0][lo] + u[0][1][lo]) -
                        (u[1][0][hi] + u[1][1][hi] + u[1][0][lo] + u[1][1][lo]));
        Z[1][v] = q1 * ((u[0][0][hi] + u[1][0][hi] + u[0][0][lo] + u[1][0][lo]) -
                        (u[0][1][hi] + u[1][1][hi] + u[0][1][lo] + u[1][1][lo]));
        Z[2][v] = q2 * ((u[0][0][hi] + u[0][1][hi] + u[1][0][hi] + u[1][1][hi]) -
                        (u[0][0][lo] + u[0][1][lo] + u[1][0][lo] + u[1][1][lo]));
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        V* dst = rv + (3 * c + j) * (N / W) + g;
        V ro;
        if (mode == 0) {
          ro = *dst;
#pragma unroll
          for (int v = 0; v < W; ++v) {
            T& e = reinterpret_cast<T*>(&ro)[v];
            e -= alpha * Z[j][v];
            acc += (double)e * (double)e;
          }
        } else {
#pragma unroll
          for (int v = 0; v < W; ++v) reinterpret_cast<T*>(&ro)[v] = Z[j][v];
        }
        *dst = ro;
      }
    }
  }
  if (mode == 0) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) partials[(long)item * gridDim.x + blockIdx.x] = s;
  }
}

// Launch over all items; returns the number of partials per item.
template <typename T>
int launch_cg_grad(const T* U, T* r, const KrylovScalars* ks, double* partials, int n0, int n1, int n2, int nitems,
                   const double h[3], int mode, hipStream_t s) {
  const long N = (long)n0 * n1 * n2;
  const T ih0 = (T)(1.0 / h[0]), ih1 = (T)(1.0 / h[1]), ih2 = (T)(1.0 / h[2]);
  if (sizeof(T) == 4 && n2 % 4 == 0) {
    const dim3 grid((unsigned)((N / 4 + 255) / 256), (unsigned)nitems);
    hipLaunchKernelGGL((k_cg_grad<T, (sizeof(T) == 4 ? 4 : 2)>), grid, dim3(256), 0, s, U, r, ks, partials, n0, n1,
                       n2, ih0, ih1, ih2, mode);
    return (int)grid.x;
  }
  const dim3 grid((unsigned)((N / 2 + 255) / 256), (unsigned)nitems);
  hipLaunchKernelGGL((k_cg_grad<T, 2>), grid, dim3(256), 0, s, U, r, ks, partials, n0, n1, n2, ih0, ih1, ih2, mode);
  return (int)grid.x;
}

}  // namespace fg
