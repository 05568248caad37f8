// Back end of one CG iteration in the potential form of the projection
// (k_fft_z_grad3 and the inverse passes leave the real 3-component potential
// U with D U = G(K p), D the corner stencil of fg_potential.hpp), and the
// stencil kernels around the CG:
//   k_cg_rupd_march  mode 0 (CG):    rho <- rho - alpha U (so r = D rho is
//                                     updated by -alpha G(K p)), per-block
//                                     partial sums of the new r . r = |D rho|^2;
//                    mode 2 (start): partial sums of |D rho|^2 of the initial
//                                     rho.
//   k_grad_store                      Z = D U as a 9-component field (the
//                                     projection itself, or the CG solution
//                                     x = D xi in double precision).
//   k_grad_norm                       partial sums of |D U|^2 (the Newton
//                                     residual norm |G*P| from U(P)).
#pragma once
#include "fg_fft.hpp"
#include "fg_launch.hpp"
#include "fg_potential.hpp"

namespace fg {

// Marching residual update: a thread owns W voxels of one line (i1, x) of
// one component c, for a run of up to K consecutive planes i0, and carries
// the new rho of the previous plane in registers, so the stencil's lower
// plane is never read again; only the line i1 - 1 is read beside the own
// line (by the neighbouring workgroup too, which runs on the same XCD at the
// same time: xcd_contiguous).  |D rho|^2 is a sum over components, so the
// components run in separate workgroups (fewer registers per thread, more
// waves in flight).  All loads of a plane are issued before its store.
// Grid (3 * ceil(n0 / K) * ceil(n1 G / 256) * items) in one dimension,
// G = n2 / W; partials per item = blocks per item.  Accesses are a per-item
// base plus a 32-bit byte offset (the host checks that an item's 9 N values
// fit in 4 GiB).
template <typename T, int W, bool LANES>
__global__ void __launch_bounds__(256)
k_cg_rupd_march(const T* __restrict__ U, long ucs, T* __restrict__ rbuf, const KrylovScalars* __restrict__ ks,
                const int* __restrict__ idle, double* __restrict__ partials, int n0, int n1, int n2, int K, T q0,
                T q1, T q2, int mode) {
  using V = typename VecW<T, W>::type;
  __shared__ double red[16];
  const int G = n2 / W;
  const unsigned bx = (unsigned)((n1 * (long)G + 255) / 256);  // blocks per plane run
  const unsigned nseg = (unsigned)((n0 + K - 1) / K);
  const unsigned per_item = 3 * bx * nseg;
  const unsigned lb = xcd_contiguous(blockIdx.x, gridDim.x);
  const int item = (int)(lb / per_item);
  const unsigned rem = lb - (unsigned)item * per_item;
  const int c = (int)(rem / (bx * nseg));
  const unsigned rc = rem - (unsigned)c * bx * nseg;
  const int seg = (int)(rc / bx);
  const unsigned blk = rc - (unsigned)seg * bx;
  if (mode == 0 && ks[item].done) return;
  if (idle && idle[item]) return;
  const long N = (long)n0 * n1 * n2;
  const int iter = (mode == 0) ? ks[item].iter : 0;
  U += (long)item * 9 * N + c * ucs;
  const T* ro = rbuf + (long)item * 9 * N + pot_half(iter, N) + c * N;
  T* rn = rbuf + (long)item * 9 * N + pot_half(iter + 1, N) + c * N;
  const T alpha = (mode == 0) ? (T)ks[item].alpha : T(0);
  const long gl = (long)blk * 256 + threadIdx.x;  // (i1, x group) in the plane
  double acc = 0.0;
  if (gl < (long)n1 * G) {
    const int i1 = (int)(gl / G);
    const int x = W * (int)(gl - (long)i1 * G);
    const int i1m = (i1 == 0) ? n1 - 1 : i1 - 1;
    const int xm = (x == 0) ? n2 - 1 : x - 1;
    constexpr unsigned E = sizeof(T);
    const unsigned plane_b = (unsigned)n1 * (unsigned)n2 * E;
    const unsigned lo[2] = {((unsigned)i1 * (unsigned)n2 + (unsigned)x) * E,
                            ((unsigned)i1m * (unsigned)n2 + (unsigned)x) * E};
    const unsigned dxm = (unsigned)(xm - x) * E;  // x - 1 (or n2 - 1) relative to x, mod 2^32
    const int i0s = seg * K, i0e = min(n0, i0s + K);
    // LANES (a line is one wave: G = 64, lane k = group k): the corner x - 1
    // is the last value of the lane below instead of a load.
    // new rho at the corners x - 1 .. x + W - 1 of lines i1 - b of plane i0
    constexpr int q0c = LANES ? 1 : 0;  // first corner loaded from memory
    auto corners = [&](int i0, T (&u)[2][W + 1]) {
      const unsigned pb = (unsigned)i0 * plane_b;
      T d[2][W + 1];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const unsigned o = pb + lo[b];
        const V w = at_bytes(reinterpret_cast<const V*>(ro), o);
        if constexpr (!LANES) u[b][0] = at_bytes(ro, o + dxm);
#pragma unroll
        for (int q = 0; q < W; ++q) u[b][q + 1] = reinterpret_cast<const T*>(&w)[q];
        if (mode == 0) {
          const V wu = at_bytes(reinterpret_cast<const V*>(U), o);
          if constexpr (!LANES) d[b][0] = at_bytes(U, o + dxm);
#pragma unroll
          for (int q = 0; q < W; ++q) d[b][q + 1] = reinterpret_cast<const T*>(&wu)[q];
        }
      }
      if (mode == 0) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int q = q0c; q <= W; ++q) u[b][q] -= alpha * d[b][q];
      }
      if constexpr (LANES) {
#pragma unroll
        for (int b = 0; b < 2; ++b) u[b][0] = lane_below(u[b][W]);
      }
    };
    T prev[2][W + 1];
    corners(i0s == 0 ? n0 - 1 : i0s - 1, prev);
    // one plane: store the own voxels, add |D rho|^2 against the lower plane
    auto plane_step = [&](int i0, const T (&cur)[2][W + 1]) {
      if (mode == 0) {
        // streaming store: the new rho is read again only by the next
        // iteration's front (measured at 256^3: 283 -> 244 us FP64)
        typedef T nvw __attribute__((ext_vector_type(W)));
        nvw a;
#pragma unroll
        for (int q = 0; q < W; ++q) a[q] = cur[0][q + 1];
        __builtin_nontemporal_store(a, reinterpret_cast<nvw*>(&at_bytes(reinterpret_cast<V*>(rn),
                                                                        (unsigned)i0 * plane_b + lo[0])));
      }
      T u[2][2][W + 1];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q <= W; ++q) {
          u[0][b][q] = cur[b][q];
          u[1][b][q] = prev[b][q];
          prev[b][q] = cur[b][q];
        }
      T Z[3][W];
      corner_grad<T, W>(u, q0, q1, q2, Z);
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int v = 0; v < W; ++v) acc += (double)Z[j][v] * (double)Z[j][v];
    };
    // two planes per step, their loads issued together (the second one
    // repeats the last plane when the run has an odd length)
    for (int i0 = i0s; i0 < i0e; i0 += 2) {
      T ca[2][W + 1], cb[2][W + 1];
      corners(i0, ca);
      corners(min(i0 + 1, i0e - 1), cb);
      plane_step(i0, ca);
      if (i0 + 1 < i0e) plane_step(i0 + 1, cb);
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[(long)item * per_item + rem] = s;
}

// Z = D U: component 3 c + j of Z (N values apart, zis per item) is D_j of
// component c of U (ucs apart, uis per item), evaluated in TO precision.
template <typename TI, typename TO, int W>
__global__ void __launch_bounds__(256)
k_grad_store(const TI* __restrict__ U, long ucs, long uis, TO* __restrict__ Z, long zis, const int* __restrict__ idle,
             int n0, int n1, int n2, TO q0, TO q1, TO q2) {
  using VO = typename VecW<TO, W>::type;
  const int item = blockIdx.y;
  if (idle && idle[item]) return;
  const long N = (long)n0 * n1 * n2;
  U += (long)item * uis;
  Z += (long)item * zis;
  const int G = n2 / W;
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N / W) return;
  const long line = g / G;
  const StencilLines sl = stencil_lines(line, W * (int)(g - line * G), n0, n1, n2);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    TI ui[2][2][W + 1];
    load_corners<TI, W>(U + c * ucs, sl, ui);
    TO u[2][2][W + 1];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q <= W; ++q) u[a][b][q] = (TO)ui[a][b][q];
    TO D[3][W];
    corner_grad<TO, W>(u, q0, q1, q2, D);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      VO w;
#pragma unroll
      for (int v = 0; v < W; ++v) reinterpret_cast<TO*>(&w)[v] = D[j][v];
      reinterpret_cast<VO*>(Z + (3 * c + j) * N)[g] = w;
    }
  }
}

// Per-block partial sums of |D U|^2 (U: 3 components ucs apart, uis per
// item; grid (ceil(N / (256 W)), items)), items with idle[b] != 0 skipped:
// the norm of the projection G*X = D U(X) from its potential.
template <typename T, int W>
__global__ void __launch_bounds__(256)
k_grad_norm(const T* __restrict__ U, long ucs, long uis, const int* __restrict__ idle, double* __restrict__ partials,
            int n0, int n1, int n2, T q0, T q1, T q2) {
  __shared__ double red[16];
  const int item = blockIdx.y;
  if (idle && idle[item]) return;
  const long N = (long)n0 * n1 * n2;
  U += (long)item * uis;
  const int G = n2 / W;
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (g < N / W) {
    const long line = g / G;
    const StencilLines sl = stencil_lines(line, W * (int)(g - line * G), n0, n1, n2);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T u[2][2][W + 1];
      load_corners<T, W>(U + c * ucs, sl, u);
      T Z[3][W];
      corner_grad<T, W>(u, q0, q1, q2, Z);
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int v = 0; v < W; ++v) acc += (double)Z[j][v] * (double)Z[j][v];
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[(long)item * gridDim.x + blockIdx.x] = s;
}

// CG start of an item: rho (half 0) = sign * U (U: 3 components ucs apart in
// double precision, uis per item), xi = 0.  grid.y = item.
template <typename T>
__global__ void __launch_bounds__(256)
k_cg_start_pot(T* __restrict__ rbuf, T* __restrict__ xbuf, const double* __restrict__ U, long ucs, long uis,
               double sign, const int* __restrict__ idle, long n) {
  const int b = blockIdx.y;
  if (idle && idle[b]) return;
  T* rho = rbuf + (long)b * 9 * n;
  T* xi = xbuf + (long)b * 9 * n;
  U += (long)b * uis;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n; i += stride) {
    const long c = i / n, k = i - c * n;
    rho[i] = (T)(sign * U[c * ucs + k]);
    xi[i] = T(0);
  }
}

inline int stencil_width(int n2, int elem_bytes) { return (elem_bytes == 4 && n2 % 4 == 0) ? 4 : 2; }

// Planes per thread of the marching residual update: 32 in single precision
// (the residual update 124 -> 119 us at 256^3: half the re-read lower planes
// and partial sums), 16 in double precision (32 there: 244 -> 246 us).
template <typename T> constexpr int rupd_planes() { return sizeof(T) == 4 ? 32 : 16; }

// CG residual update (mode 0) or initial |D rho|^2 (mode 2) over all items;
// returns the number of partials per item.
template <typename T>
int launch_cg_rupd(const T* U, long ucs, T* rbuf, const KrylovScalars* ks, const int* idle, double* partials, int n0,
                   int n1, int n2, int nitems, const double h[3], int mode, hipStream_t s, hipEvent_t ev0 = nullptr,
                   hipEvent_t ev1 = nullptr) {
  const T q0 = (T)(0.25 / h[0]), q1 = (T)(0.25 / h[1]), q2 = (T)(0.25 / h[2]);
  if ((double)9 * n0 * n1 * n2 * sizeof(T) >= 4294967296.0)
    throw std::invalid_argument("grid too large for 32-bit offsets in the residual update");
  const int K = rupd_planes<T>();
  const long nseg = (n0 + K - 1) / K;
  const int W = stencil_width(n2, (int)sizeof(T));
  const long bx = ((long)n1 * (n2 / W) + 255) / 256;
  const dim3 grid((unsigned)(3 * bx * nseg * nitems));
  // a line of n2 / W = 64 groups is exactly one wave of a workgroup
  const bool lanes = n2 / W == 64;
  auto go = [&](auto kernel) {
    launch_ev(kernel, grid, dim3(256), 0, s, ev0, ev1, U, ucs, rbuf, ks, idle, partials, n0, n1, n2, K, q0, q1, q2,
              mode);
  };
  if constexpr (sizeof(T) == 4) {
    if (W == 4) {
      if (lanes)
        go(k_cg_rupd_march<T, 4, true>);
      else
        go(k_cg_rupd_march<T, 4, false>);
      return (int)(3 * bx * nseg);
    }
  }
  if (lanes)
    go(k_cg_rupd_march<T, 2, true>);
  else
    go(k_cg_rupd_march<T, 2, false>);
  return (int)(3 * bx * nseg);
}

// |D U|^2 partial sums over all items (two voxels per thread); returns the
// partials per item.
inline int launch_grad_norm(const double* U, long ucs, long uis, const int* idle, double* partials, int n0, int n1,
                            int n2, int nitems, const double h[3], hipStream_t s) {
  const long N = (long)n0 * n1 * n2;
  const dim3 grid((unsigned)((N / 2 + 255) / 256), (unsigned)nitems);
  hipLaunchKernelGGL((k_grad_norm<double, 2>), grid, dim3(256), 0, s, U, ucs, uis, idle, partials, n0, n1, n2,
                     0.25 / h[0], 0.25 / h[1], 0.25 / h[2]);
  return (int)grid.x;
}

// Z = D U over all items (two voxels per thread).
template <typename TI, typename TO>
void launch_grad_store(const TI* U, long ucs, long uis, TO* Z, long zis, const int* idle, int n0, int n1, int n2,
                       int nitems, const double h[3], hipStream_t s) {
  const long N = (long)n0 * n1 * n2;
  const TO q0 = (TO)(0.25 / h[0]), q1 = (TO)(0.25 / h[1]), q2 = (TO)(0.25 / h[2]);
  const dim3 grid((unsigned)((N / 2 + 255) / 256), (unsigned)nitems);
  hipLaunchKernelGGL((k_grad_store<TI, TO, 2>), grid, dim3(256), 0, s, U, ucs, uis, Z, zis, idle, n0, n1, n2, q0, q1,
                     q2);
}

}  // namespace fg
