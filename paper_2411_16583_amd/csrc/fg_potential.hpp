// Corner-stencil gradient of a 3-component potential on the voxel grid, the
// real-space half of the potential form of the projection (eq. (28) with the
// rotated scheme): for the potential u_i,
//   (D_j u_i)[n] = 1/(4 h_j) * sum over the four voxel edges parallel to
//                  axis j of (u_i at the upper corner - u_i at the lower one),
// with the corner n - 1/2 (in every axis) stored at index n - 1 (periodic).
// Its symbol is i e^{-i Phi} r_j, Phi = (q0 + q1 + q2) / 2, so D maps onto the
// range of the projection: every compatible field of the CG (residual,
// direction, solution) is D of a 3-component field, and the CG kernels keep
// only those potentials in memory.
//
// A thread owns W consecutive voxels x .. x + W - 1 of one grid line (i0, i1)
// along N2; the stencil reads the corners x - 1 .. x + W - 1 of the four
// lines (i0 - a, i1 - b), a, b in {0, 1}.
#pragma once
#include <hip/hip_runtime.h>

namespace fg {

// W consecutive values of one plane in one 8- or 16-byte access.
template <typename T, int W> struct VecW;
template <> struct VecW<double, 2> { using type = double2; };
template <> struct VecW<float, 2> { using type = float2; };
template <> struct VecW<float, 4> { using type = float4; };

struct StencilLines {
  long row[2][2];  // element offset of line (i0 - a, i1 - b) within a component
  int x, xm;       // first voxel of the thread and its lower neighbour (periodic)
};

__device__ __forceinline__ StencilLines stencil_lines(long line, int x, int n0, int n1, int n2) {
  StencilLines s;
  const int i0 = (int)(line / n1), i1 = (int)(line - (long)i0 * n1);
  const int i0m = (i0 == 0) ? n0 - 1 : i0 - 1;
  const int i1m = (i1 == 0) ? n1 - 1 : i1 - 1;
  s.row[0][0] = ((long)i0 * n1 + i1) * n2;
  s.row[0][1] = ((long)i0 * n1 + i1m) * n2;
  s.row[1][0] = ((long)i0m * n1 + i1) * n2;
  s.row[1][1] = ((long)i0m * n1 + i1m) * n2;
  s.x = x;
  s.xm = (x == 0) ? n2 - 1 : x - 1;
  return s;
}

// u[a][b][p]: the component f at corner x - 1 + p of line (i0 - a, i1 - b).
template <typename T, int W>
__device__ __forceinline__ void load_corners(const T* __restrict__ f, const StencilLines& s, T (&u)[2][2][W + 1]) {
  using V = typename VecW<T, W>::type;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const V w = *reinterpret_cast<const V*>(f + s.row[a][b] + s.x);
      u[a][b][0] = f[s.row[a][b] + s.xm];
#pragma unroll
      for (int q = 0; q < W; ++q) u[a][b][q + 1] = reinterpret_cast<const T*>(&w)[q];
    }
}

// The value v held by the lane one below (lane 0 takes lane 63's): a
// wave-wide DPP rotation by one lane, no memory access.
__device__ __forceinline__ float lane_below(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x13C, 0xF, 0xF, false));
}
__device__ __forceinline__ double lane_below(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x13C, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x13C, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// As load_corners, with the corner x - 1 taken from the lane below rather
// than from memory.  Lane k of the wave must hold voxel group k of 64
// consecutive groups of one line (so the lane below holds x - W .. x - 1,
// and lane 0 of a wave that covers a whole line holds the periodic
// neighbour in lane 63); `edge` lanes (lane 0 when a line spans several
// waves) load their corner.  Every lane of the wave must be active.
template <typename T, int W>
__device__ __forceinline__ void load_corners_lanes(const T* __restrict__ f, const StencilLines& s,
                                                   T (&u)[2][2][W + 1], bool edge) {
  using V = typename VecW<T, W>::type;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const V w = *reinterpret_cast<const V*>(f + s.row[a][b] + s.x);
#pragma unroll
      for (int q = 0; q < W; ++q) u[a][b][q + 1] = reinterpret_cast<const T*>(&w)[q];
      u[a][b][0] = lane_below(u[a][b][W]);
    }
  if (edge) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) u[a][b][0] = f[s.row[a][b] + s.xm];
  }
}

// Z[j][v] = (D_j u)[x + v] with q_j = 1 / (4 h_j).
template <typename T, int W>
__device__ __forceinline__ void corner_grad(const T (&u)[2][2][W + 1], T q0, T q1, T q2, T (&Z)[3][W]) {
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
}

// Logical workgroup index that gives each XCD a contiguous range: the
// hardware deals workgroups out to the 8 XCDs round-robin in launch order,
// so workgroup `flat` is the k-th one of XCD flat % 8.  Neighbouring logical
// workgroups then share an L2.
__device__ __forceinline__ unsigned xcd_contiguous(unsigned flat, unsigned total) {
  const unsigned q = total / 8, r = total % 8;
  const unsigned x = flat % 8, k = flat / 8;
  return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Storage of the CG potentials of one item: rho (residual), pi (direction)
// and xi (solution), 3 components of N values each, at the start of the
// item's 9 N-value regions of the r, p and x buffers.  rho and pi alternate
// between the halves [0, 3N) and [3N, 6N) by iteration parity: a kernel
// reads its neighbours' corners of the old values while it writes new ones,
// so old and new never share memory.  At iteration k (KrylovScalars::iter):
//   rho_k in half k % 2, pi_k in half k % 2 (pi_{k-1} in the other half).
__host__ __device__ constexpr long pot_half(int iter, long N) { return (long)(iter & 1) * 3 * N; }

}  // namespace fg
