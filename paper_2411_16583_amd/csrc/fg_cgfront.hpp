// Front kernel of one CG iteration on the operator of eq. (30), fused, with
// the CG vectors held as 3-component potentials (r = D rho, p = D pi,
// x = D xi, D the corner-stencil gradient of fg_potential.hpp):
//   xi <- xi + alpha_{k-1} pi_{k-1}        (deferred solution update, k > 0)
//   pi <- rho (k = 0) or rho + beta pi     (search direction)
//   p  = D pi                              (9 components, never stored)
//   Y  = K : p                             (tangent contraction from the law's
//                                           state: 12 words Neo-Hookean, 18 SVK)
//   p . Y per block (FP64)                 (= p . G(K p) since p is compatible)
//   Y -> packed real-to-complex transform along N2, written as the spectrum.
// The contracted field never goes to HBM: it is staged in LDS, line by line,
// and transformed there.
//
// A workgroup owns LB grid lines (i0, i1) and all 9 components of them:
// phase A is one thread per 2 or 4 voxels (coalesced along N2; in single
// precision, where a line is a whole number of waves, only full waves take
// part and the stencil's lower corner comes from the neighbouring lane),
// phase B is the
// two-stage line FFT of the 9 LB complex lines with T threads each
// (9 LB T = 144 threads).  The stencil needs pi at the corners of the lines
// (i0 - 1, i1), (i0, i1 - 1), (i0 - 1, i1 - 1) too; it recomputes them from
// rho and the old pi there (read through the caches), and the new pi goes to
// the other parity half, so no workgroup reads what another one writes.
#pragma once
#include "fg_fft.hpp"
#include "fg_potential.hpp"
#include "fg_tangent.hpp"

namespace fg {

// W consecutive voxels of one plane in one 16-byte (or 8-byte) access.
template <typename R, int W> struct FrontPack;
template <> struct FrontPack<double, 2> { using type = double2; };
template <> struct FrontPack<float, 2> { using type = float2; };
template <> struct FrontPack<float, 4> { using type = float4; };
// voxels per thread and step in phase A: 16-byte accesses where possible
template <typename R, int M> constexpr int front_width() { return (sizeof(R) == 4 && M % 2 == 0) ? 4 : 2; }

template <typename R, typename PV> __device__ __forceinline__ R pk_get(const PV& v, int w) {
  return reinterpret_cast<const R*>(&v)[w];
}
template <typename R, typename PV> __device__ __forceinline__ void pk_set(PV& v, int w, R a) {
  reinterpret_cast<R*>(&v)[w] = a;
}
// nontemporal store of a W-vector (write streams read back only by a later kernel)
template <typename R, int W, typename PV> __device__ __forceinline__ void pk_stream(PV* p, const PV& v) {
  typedef R nvw __attribute__((ext_vector_type(W)));
  nvw a;
#pragma unroll
  for (int w = 0; w < W; ++w) a[w] = pk_get<R>(v, w);
  __builtin_nontemporal_store(a, reinterpret_cast<nvw*>(p));
}

// nontemporal load of a W-vector (streams read once: the tangent state and
// the solution potential), so that they do not push the stencil's neighbour
// lines of rho and pi out of the caches
template <typename R, int W, typename PV> __device__ __forceinline__ PV pk_load_nt(const PV* p) {
  typedef R nvw __attribute__((ext_vector_type(W)));
  const nvw a = __builtin_nontemporal_load(reinterpret_cast<const nvw*>(p));
  PV v;
#pragma unroll
  for (int w = 0; w < W; ++w) pk_set<R>(v, w, a[w]);
  return v;
}

template <int M> struct FrontShape {
  static constexpr int T = Line<M>::T;
  static constexpr int LB = (16 / T) > 0 ? (16 / T) : 1;  // lines per workgroup
  static constexpr int THREADS = 9 * LB * T;
  // Complex pad per line buffer.  A wave touches 64/T lines at once, T
  // consecutive elements each; a line stride of T (mod 32) starts them T
  // elements apart in the banks instead of one (a pad of one element puts
  // line l + 1's element t on the banks of line l's element t + 1).  In
  // single precision this removed most of the front's LDS bank conflicts
  // (counted conflict cycles 4.5e7 -> 0.7e7 at 256^3).  Double precision
  // takes a one-element pad: its buffers (with the stage twiddles) then fit
  // four workgroups per CU instead of three (the front 948 -> 930 us at
  // 256^3).
  static constexpr bool kBankPad = M % 32 == 0 && (T == 4 || T == 8 || T == 16);
  static constexpr int PADC = kBankPad ? T : ((M >= 16) ? 1 : 0);
  template <typename R> static constexpr int lstride() { return sizeof(R) == 8 ? M + 1 : M + PADC; }
};

template <typename R, int M, int LAW>
__global__ void __launch_bounds__(FrontShape<M>::THREADS)
k_cg_front(R* __restrict__ spec, R* __restrict__ pbuf, R* __restrict__ xbuf, const R* __restrict__ rbuf,
           const R* __restrict__ st, const KrylovScalars* __restrict__ ksb, double* __restrict__ partials,
           long N, int n0, int n1, SpecTables<R> tb, R q0, R q1, R q2) {
  using C = cplx<R>;
  using LS = Line<M>;
  using FS = FrontShape<M>;
  constexpr int N2 = 2 * M;
  constexpr int LB = FS::LB;
  constexpr int LSTRIDE = FS::template lstride<R>();  // complex elements per line buffer
  __shared__ C buf[9 * LB * LSTRIDE];
  __shared__ double red[16];
  // the R2C post-processing factors in LDS in single precision only (double
  // precision reads them from the caches, once per output element, to keep
  // four workgroups per CU)
  constexpr bool kPostLds = sizeof(R) == 4;
  __shared__ C stw[M], spost[kPostLds ? M : 1];
  const long nlines = (long)n0 * n1;
  // batch item of this workgroup (items are nlines lines of 9 components
  // each, item-major; ceil(nlines / LB) workgroups per item)
  const long bpi = (nlines + LB - 1) / LB;
  const int item = (int)(blockIdx.x / bpi);
  const KrylovScalars* ks = ksb + item;
  if (ks->done) return;
  spec += (long)item * 9 * N;
  pbuf += (long)item * 9 * N;
  xbuf += (long)item * 9 * N;
  rbuf += (long)item * 9 * N;
  st += (long)item * state_words(LAW) * N;
  const int tid = threadIdx.x;
  // the N2 line's stage twiddles (and the R2C post-processing factors) in
  // LDS, read once per workgroup (phase A's barrier below orders them); read
  // from the caches inside phase B they cost the single-precision front
  // 525 -> 488 us at 256^3 (FP64 950 -> 940 us)
  for (int k = tid; k < M; k += FS::THREADS) {
    stw[k] = tb.twM[k];
    if constexpr (kPostLds) spost[k] = tb.post[k];
  }
  const long line0 = ((long)blockIdx.x - (long)item * bpi) * LB;
  const int iter = ks->iter;
  const bool first = iter == 0;
  const R alpha = (R)ks->alpha;
  const R beta = (R)ks->beta;
  const R* rho = rbuf + pot_half(iter, N);
  const R* po = pbuf + pot_half(iter + 1, N);
  R* pn = pbuf + pot_half(iter, N);
  double acc = 0.0;
  // ---- phase A: pointwise, W voxels per thread and step (one W-vector
  // access per plane; W = 4 in single precision, else 2)
  constexpr int W = front_width<R, M>();
  using PV = typename FrontPack<R, W>::type;
  constexpr int GPL = 2 * M / W;  // voxel groups per line
  // single precision, lines of whole waves: the stencil's corner x - 1 comes
  // from the lane below, and phase A runs on the full waves only (lane k =
  // group k mod 64).  (In double precision this raised the kernel from 148
  // to 184 VGPRs and made it slower.)
  constexpr bool kLanes = sizeof(R) == 4 && GPL % 64 == 0;
  constexpr int PA = kLanes ? (FS::THREADS / 64) * 64 : FS::THREADS;
  static_assert(PA > 0, "phase A threads");
  const bool edge = kLanes && GPL > 64 && (tid & 63) == 0;
  const long Nw = N / W;
  const PV* sv = reinterpret_cast<const PV*>(st);
#pragma unroll 1
  for (int v = tid; tid < PA && v < LB * GPL; v += PA) {
    const int l = v / GPL;
    const int n = v % GPL;  // voxels W n .. W n + W - 1 of line l
    if (line0 + l >= nlines) continue;
    const long g = (line0 + l) * GPL + n;
    const StencilLines sl = stencil_lines(line0 + l, W * n, n0, n1, N2);
    R X[W][9];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      R u[2][2][W + 1];
      if constexpr (kLanes)
        load_corners_lanes<R, W>(rho + c * N, sl, u, edge);
      else
        load_corners<R, W>(rho + c * N, sl, u);
      if (!first) {
        R uo[2][2][W + 1];
        if constexpr (kLanes)
          load_corners_lanes<R, W>(po + c * N, sl, uo, edge);
        else
          load_corners<R, W>(po + c * N, sl, uo);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q <= W; ++q) u[a][b][q] += beta * uo[a][b][q];
        // deferred solution update at the thread's own voxels
        PV* xv = reinterpret_cast<PV*>(xbuf + c * N) + g;
        PV xo = pk_load_nt<R, W>(xv);
#pragma unroll
        for (int w = 0; w < W; ++w) pk_set<R>(xo, w, pk_get<R>(xo, w) + alpha * uo[0][0][w + 1]);
        pk_stream<R, W>(xv, xo);
      }
      PV pk;
#pragma unroll
      for (int w = 0; w < W; ++w) pk_set<R>(pk, w, u[0][0][w + 1]);
      pk_stream<R, W>(reinterpret_cast<PV*>(pn + c * N) + g, pk);
      R Z[3][W];
      corner_grad<R, W>(u, q0, q1, q2, Z);
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int w = 0; w < W; ++w) X[w][3 * c + j] = Z[j][w];
    }
    constexpr int NS = (LAW == kLawSVK) ? 17 : 12;  // state words read
    PV A[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) A[k] = pk_load_nt<R, W>(sv + k * Nw + g);
#pragma unroll
    for (int w = 0; w < W; w += 2) {
      R A0[9], A1[9], Y0[9], Y1[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        A0[k] = pk_get<R>(A[k], w);
        A1[k] = pk_get<R>(A[k], w + 1);
      }
      if constexpr (LAW == kLawSVK) {
        R S0[6], S1[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          S0[k] = pk_get<R>(A[9 + k], w);
          S1[k] = pk_get<R>(A[9 + k], w + 1);
        }
        svk_apply<R>(A0, S0, pk_get<R>(A[15], w), pk_get<R>(A[16], w), X[w], Y0);
        svk_apply<R>(A1, S1, pk_get<R>(A[15], w + 1), pk_get<R>(A[16], w + 1), X[w + 1], Y1);
      } else {
        tangent_apply<R>(A0, pk_get<R>(A[9], w), pk_get<R>(A[10], w), pk_get<R>(A[11], w), X[w], Y0);
        tangent_apply<R>(A1, pk_get<R>(A[9], w + 1), pk_get<R>(A[10], w + 1), pk_get<R>(A[11], w + 1), X[w + 1],
                         Y1);
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        acc += (double)X[w][k] * (double)Y0[k] + (double)X[w + 1][k] * (double)Y1[k];
        buf[(k * LB + l) * LSTRIDE + n * (W / 2) + w / 2] = mk<C>(Y0[k], Y1[k]);
      }
    }
  }
  __syncthreads();
  // ---- phase B: R2C along N2 of the 9 LB lines held in LDS
  const int lt = tid / LS::T;  // line task: component * LB + line
  const int t = tid % LS::T;
  const int comp = lt / LB;
  const int l = lt % LB;
  C* my = buf + lt * LSTRIDE;
  const bool active = (line0 + l) < nlines;
  C v[LS::E];
#pragma unroll
  for (int e = 0; e < LS::E; ++e) v[e] = my[LS::idxA(t, e)];
  // from here on a line's buffer is touched by its own T threads only, which
  // sit in one wave (T divides 64): wave-level ordering suffices
  static_assert(64 % LS::T == 0, "lines within one wave");
  lds_sync<true>();  // every line fully read before the exchange writes into it
  line_fft_AB<M, false, C, true>(v, my, 1, t, stw);
#pragma unroll
  for (int e = 0; e < LS::E; ++e) my[LS::idxB(t, e)] = v[e];
  lds_sync<true>();
  C* dst = reinterpret_cast<C*>(spec) + ((long)comp * nlines + line0 + l) * M;
  // X_k of the real line from the packed transform z (k = 0 carries both
  // ends of the spectrum)
  auto post = [&](int k) {
    const C zk = my[k];
    if (k == 0) return mk<C>(zk.x + zk.y, zk.x - zk.y);
    const C zm = my[M - k];
    const C ev = cscale(cadd(zk, cconj(zm)), R(0.5));
    const C od = cscale(mul_mi(csub(zk, cconj(zm))), R(0.5));
    if constexpr (kPostLds)
      return cadd(ev, cmul(od, spost[k]));
    else
      return cadd(ev, cmul(od, tb.post[k]));
  };
  if constexpr (sizeof(R) == 4 && M % (2 * LS::T) == 0) {
    // single precision: two adjacent elements per thread and store, so that
    // a line's T threads write 16 T contiguous bytes (whole 128-byte lines at
    // T = 8); the nontemporal half-line stores of one element per thread
    // counted 15% more written bytes than the spectrum and cost the front
    // 494 -> 440 us at 256^3
#pragma unroll
    for (int j = 0; j < M / (2 * LS::T); ++j) {
      const int k = 2 * (j * LS::T + t);
      const C x0 = post(k), x1 = post(k + 1);
      if (active) st_stream_f4(dst + k, make_float4(x0.x, x0.y, x1.x, x1.y));
    }
  } else {
#pragma unroll
    for (int e = 0; e < LS::E; ++e) {
      const int k = LS::idxB(t, e);
      const C X = post(k);
      if (active) st_stream(dst + k, X);
    }
  }
  const double s = block_sum(acc, red);
  if (tid == 0) partials[blockIdx.x] = s;
}

// xi += alpha pi once after the CG loop (the last deferred update, with pi of
// the last iteration), unless the loop ended on a breakdown (then the front
// kernel already applied the last valid step).  grid.y = batch item; n = N
// values per component; items with idle[b] != 0 are left alone.
template <typename T>
__global__ void __launch_bounds__(256)
k_cg_final_xi(T* __restrict__ xbuf, const T* __restrict__ pbuf, const KrylovScalars* __restrict__ ks,
              const int* __restrict__ idle, long n) {
  const int b = blockIdx.y;
  if (idle && idle[b]) return;
  const KrylovScalars* k = ks + b;
  if (k->flag == 1 || k->iter == 0) return;
  const T alpha = (T)k->alpha;
  T* xi = xbuf + (long)b * 9 * n;
  const T* pi = pbuf + (long)b * 9 * n + pot_half(k->iter - 1, n);
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n; i += stride) xi[i] += alpha * pi[i];
}

}  // namespace fg
