// Three-stage line FFT (L = R1 R2 R3) with more threads per line and fewer
// elements per thread than the two-stage version; used by the N0 pass fused
// with the projection, whose per-thread accumulator would otherwise double
// the register footprint.
//
// Forward, with Q = R2 R3:
//   stage 1: butterfly b in [0, Q):        x[b + Q n1]            -> Y1[b][k1]  * W_L^{b k1}
//   stage 2: butterfly (k1, b2):            Y1[b2 + R3 n2][k1]     -> Y2[k1][b2][k2] * W_Q^{b2 k2}
//   stage 3: butterfly (k1, k2):            Y2[k1][b2][k2] over b2 -> X[k1 + R1 (k2 + R2 k3)]
// Layout A (natural): thread t holds x[(t + T u) + Q n1], e = u R1 + n1.
// Layout B (spectral): thread t holds X[k1 + R1 (k2 + R2 k3)] with
// (k1, k2) = (g % R1, g / R1), g = t + T z, e = z R3 + k3.
// The inverse runs the stages backwards with conjugate twiddles (B -> A).
#pragma once
#include <type_traits>

#include "fg_fft.hpp"

namespace fg {

template <int L> struct Line3Shape;
template <> struct Line3Shape<256> {
  static constexpr int R1 = 8, R2 = 8, R3 = 4, T = 32;
};
template <> struct Line3Shape<128> {
  static constexpr int R1 = 4, R2 = 4, R3 = 8, T = 16;
};
template <> struct Line3Shape<96> {
  static constexpr int R1 = 4, R2 = 4, R3 = 6, T = 8;
};
template <> struct Line3Shape<512> {
  static constexpr int R1 = 8, R2 = 8, R3 = 8, T = 64;
};

// CPT adjacent columns of one LDS row position in one access (two
// single-precision complex values: one 16-byte access, the same bank pattern
// as one double-precision column).
template <int CPT, typename C> __device__ __forceinline__ void lds_put(C* p, const C (&x)[CPT]) {
  if constexpr (CPT == 2) {
    static_assert(sizeof(C) == 8, "column pairs in single precision");
    *reinterpret_cast<float4*>(p) = make_float4(x[0].x, x[0].y, x[CPT - 1].x, x[CPT - 1].y);
  } else {
    *p = x[0];
  }
}
template <int CPT, typename C> __device__ __forceinline__ void lds_get(const C* p, C (&x)[CPT]) {
  if constexpr (CPT == 2) {
    const float4 w = *reinterpret_cast<const float4*>(p);
    x[0] = mk<C>(w.x, w.y);
    x[CPT - 1] = mk<C>(w.z, w.w);
  } else {
    x[0] = *p;
  }
}

template <int L> struct Line3 {
  static constexpr int R1 = Line3Shape<L>::R1, R2 = Line3Shape<L>::R2, R3 = Line3Shape<L>::R3;
  static constexpr int T = Line3Shape<L>::T;
  static constexpr int Q = R2 * R3;
  static constexpr int U1 = Q / T, U2 = R1 * R3 / T, U3 = R1 * R2 / T;
  static constexpr int E = L / T;
  static_assert(U1 * T == Q && U2 * T == R1 * R3 && U3 * T == R1 * R2, "thread split");
  static_assert(U1 * R1 == E && U2 * R2 == E && U3 * R3 == E, "element split");
  __device__ __forceinline__ static int idxA(int t, int e) { return t + T * (e / R1) + Q * (e % R1); }
  __device__ __forceinline__ static int idxB(int t, int e) {
    const int g = t + T * (e / R3);
    return (g % R1) + R1 * ((g / R1) + R2 * (e % R3));
  }
  // LDS positions of the intermediate arrays
  __device__ __forceinline__ static int pos1(int b, int k1) { return b * R1 + k1; }
  __device__ __forceinline__ static int pos2(int k1, int b2, int k2) { return (k2 * R3 + b2) * R1 + k1; }

  template <bool INV, typename C>
  __device__ __forceinline__ static void fwd(C (&v)[E], C* lds, int ls, int t, const C* tw) {
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int b = t + T * u;
      Dft<R1, 1, INV, C>::run(v + u * R1);
#pragma unroll
      for (int k1 = 1; k1 < R1; ++k1) v[u * R1 + k1] = twiddle_tab<INV>(v[u * R1 + k1], tw, (b * k1) % L);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) lds[pos1(b, k1) * ls] = v[u * R1 + k1];
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < U2; ++w) {
      const int g = t + T * w;
      const int k1 = g % R1, b2 = g / R1;
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) v[w * R2 + n2] = lds[pos1(b2 + R3 * n2, k1) * ls];
      Dft<R2, 1, INV, C>::run(v + w * R2);
#pragma unroll
      for (int k2 = 1; k2 < R2; ++k2) v[w * R2 + k2] = twiddle_tab<INV>(v[w * R2 + k2], tw, (R1 * b2 * k2) % L);
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < U2; ++w) {
      const int g = t + T * w;
      const int k1 = g % R1, b2 = g / R1;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) lds[pos2(k1, b2, k2) * ls] = v[w * R2 + k2];
    }
    __syncthreads();
#pragma unroll
    for (int z = 0; z < U3; ++z) {
      const int g = t + T * z;
      const int k1 = g % R1, k2 = g / R1;
#pragma unroll
      for (int b2 = 0; b2 < R3; ++b2) v[z * R3 + b2] = lds[pos2(k1, b2, k2) * ls];
      Dft<R3, 1, INV, C>::run(v + z * R3);
    }
    __syncthreads();
  }

  template <typename C>
  __device__ __forceinline__ static void inv(C (&v)[E], C* lds, int ls, int t, const C* tw) {
#pragma unroll
    for (int z = 0; z < U3; ++z) {
      const int g = t + T * z;
      const int k1 = g % R1, k2 = g / R1;
      Dft<R3, 1, true, C>::run(v + z * R3);  // over k3 -> b2
#pragma unroll
      for (int b2 = 0; b2 < R3; ++b2) {
        C a = v[z * R3 + b2];
        if (b2 != 0 && k2 != 0) a = twiddle_tab<true>(a, tw, (R1 * b2 * k2) % L);
        lds[pos2(k1, b2, k2) * ls] = a;
      }
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < U2; ++w) {
      const int g = t + T * w;
      const int k1 = g % R1, b2 = g / R1;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[w * R2 + k2] = lds[pos2(k1, b2, k2) * ls];
      Dft<R2, 1, true, C>::run(v + w * R2);  // over k2 -> n2
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < U2; ++w) {
      const int g = t + T * w;
      const int k1 = g % R1, b2 = g / R1;
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) {
        const int b = b2 + R3 * n2;
        C a = v[w * R2 + n2];
        if (k1 != 0) a = twiddle_tab<true>(a, tw, (b * k1) % L);
        lds[pos1(b, k1) * ls] = a;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int b = t + T * u;
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) v[u * R1 + k1] = lds[pos1(b, k1) * ls];
      Dft<R1, 1, true, C>::run(v + u * R1);  // over k1 -> n1
    }
    __syncthreads();
  }

  // fwd and inv of CPT adjacent columns together (lds points at the first
  // column, which is CPT-aligned; one CPT-wide LDS access per position).
  template <bool INV, int CPT, typename C>
  __device__ __forceinline__ static void fwd_cols(C (&v)[CPT][E], C* lds, int ls, int t, const C* tw) {
    if constexpr (CPT == 1) {
      fwd<INV>(v[0], lds, ls, t, tw);
    } else {
#pragma unroll
      for (int u = 0; u < U1; ++u) {
        const int b = t + T * u;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          Dft<R1, 1, INV, C>::run(v[c] + u * R1);
#pragma unroll
          for (int k1 = 1; k1 < R1; ++k1) v[c][u * R1 + k1] = twiddle_tab<INV>(v[c][u * R1 + k1], tw, (b * k1) % L);
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
          C x[CPT];
#pragma unroll
          for (int c = 0; c < CPT; ++c) x[c] = v[c][u * R1 + k1];
          lds_put<CPT>(lds + pos1(b, k1) * ls, x);
        }
      }
      __syncthreads();
#pragma unroll
      for (int w = 0; w < U2; ++w) {
        const int g = t + T * w;
        const int k1 = g % R1, b2 = g / R1;
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
          C x[CPT];
          lds_get<CPT>(lds + pos1(b2 + R3 * n2, k1) * ls, x);
#pragma unroll
          for (int c = 0; c < CPT; ++c) v[c][w * R2 + n2] = x[c];
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          Dft<R2, 1, INV, C>::run(v[c] + w * R2);
#pragma unroll
          for (int k2 = 1; k2 < R2; ++k2)
            v[c][w * R2 + k2] = twiddle_tab<INV>(v[c][w * R2 + k2], tw, (R1 * b2 * k2) % L);
        }
      }
      __syncthreads();
#pragma unroll
      for (int w = 0; w < U2; ++w) {
        const int g = t + T * w;
        const int k1 = g % R1, b2 = g / R1;
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
          C x[CPT];
#pragma unroll
          for (int c = 0; c < CPT; ++c) x[c] = v[c][w * R2 + k2];
          lds_put<CPT>(lds + pos2(k1, b2, k2) * ls, x);
        }
      }
      __syncthreads();
#pragma unroll
      for (int z = 0; z < U3; ++z) {
        const int g = t + T * z;
        const int k1 = g % R1, k2 = g / R1;
#pragma unroll
        for (int b2 = 0; b2 < R3; ++b2) {
          C x[CPT];
          lds_get<CPT>(lds + pos2(k1, b2, k2) * ls, x);
#pragma unroll
          for (int c = 0; c < CPT; ++c) v[c][z * R3 + b2] = x[c];
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) Dft<R3, 1, INV, C>::run(v[c] + z * R3);
      }
      __syncthreads();
    }
  }

  template <int CPT, typename C>
  __device__ __forceinline__ static void inv_cols(C (&v)[CPT][E], C* lds, int ls, int t, const C* tw) {
    if constexpr (CPT == 1) {
      inv(v[0], lds, ls, t, tw);
    } else {
#pragma unroll
      for (int z = 0; z < U3; ++z) {
        const int g = t + T * z;
        const int k1 = g % R1, k2 = g / R1;
#pragma unroll
        for (int c = 0; c < CPT; ++c) Dft<R3, 1, true, C>::run(v[c] + z * R3);  // over k3 -> b2
#pragma unroll
        for (int b2 = 0; b2 < R3; ++b2) {
          C x[CPT];
#pragma unroll
          for (int c = 0; c < CPT; ++c) {
            x[c] = v[c][z * R3 + b2];
            if (b2 != 0 && k2 != 0) x[c] = twiddle_tab<true>(x[c], tw, (R1 * b2 * k2) % L);
          }
          lds_put<CPT>(lds + pos2(k1, b2, k2) * ls, x);
        }
      }
      __syncthreads();
#pragma unroll
      for (int w = 0; w < U2; ++w) {
        const int g = t + T * w;
        const int k1 = g % R1, b2 = g / R1;
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
          C x[CPT];
          lds_get<CPT>(lds + pos2(k1, b2, k2) * ls, x);
#pragma unroll
          for (int c = 0; c < CPT; ++c) v[c][w * R2 + k2] = x[c];
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) Dft<R2, 1, true, C>::run(v[c] + w * R2);  // over k2 -> n2
      }
      __syncthreads();
#pragma unroll
      for (int w = 0; w < U2; ++w) {
        const int g = t + T * w;
        const int k1 = g % R1, b2 = g / R1;
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
          const int b = b2 + R3 * n2;
          C x[CPT];
#pragma unroll
          for (int c = 0; c < CPT; ++c) {
            x[c] = v[c][w * R2 + n2];
            if (k1 != 0) x[c] = twiddle_tab<true>(x[c], tw, (b * k1) % L);
          }
          lds_put<CPT>(lds + pos1(b, k1) * ls, x);
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < U1; ++u) {
        const int b = t + T * u;
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
          C x[CPT];
          lds_get<CPT>(lds + pos1(b, k1) * ls, x);
#pragma unroll
          for (int c = 0; c < CPT; ++c) v[c][u * R1 + k1] = x[c];
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) Dft<R1, 1, true, C>::run(v[c] + u * R1);  // over k1 -> n1
      }
      __syncthreads();
    }
  }
};

// The two-stage transform behind the same interface.
template <int L> struct Line2Ops {
  using LS = Line<L>;
  static constexpr int T = LS::T, E = LS::E;
  __device__ __forceinline__ static int idxA(int t, int e) { return LS::idxA(t, e); }
  __device__ __forceinline__ static int idxB(int t, int e) { return LS::idxB(t, e); }
  template <bool INV, typename C>
  __device__ __forceinline__ static void fwd(C (&v)[E], C* lds, int ls, int t, const C* tw) {
    line_fft_AB<L, INV>(v, lds, ls, t, tw);
  }
  template <typename C>
  __device__ __forceinline__ static void inv(C (&v)[E], C* lds, int ls, int t, const C* tw) {
    line_ifft_BA<L>(v, lds, ls, t, tw);
  }
  // columns one after the other (one element per LDS access)
  template <bool INV, int CPT, typename C>
  __device__ __forceinline__ static void fwd_cols(C (&v)[CPT][E], C* lds, int ls, int t, const C* tw) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) fwd<INV>(v[c], lds + c, ls, t, tw);
  }
  template <int CPT, typename C>
  __device__ __forceinline__ static void inv_cols(C (&v)[CPT][E], C* lds, int ls, int t, const C* tw) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) inv(v[c], lds + c, ls, t, tw);
  }
};

// Line transform used by the fused N0 passes.
template <int L> struct ZLineSel {
  using type = Line2Ops<L>;
};
template <> struct ZLineSel<256> {
  using type = Line3<256>;
};
template <> struct ZLineSel<128> {
  using type = Line3<128>;
};
template <> struct ZLineSel<96> {
  using type = Line3<96>;
};
template <> struct ZLineSel<512> {
  using type = Line3<512>;
};
template <int L> using ZLine = typename ZLineSel<L>::type;
// Line of the potential-form N0 pass: ZLine, except the two-stage 16 x 16
// line in single precision at L = 256 (one column per thread there).
template <typename R, int L> struct ZGradSel {
  using type = ZLine<L>;
};
template <> struct ZGradSel<float, 256> {
  using type = Line2Ops<256>;
};

template <typename R, int L>
__global__ void __launch_bounds__(256)
k_fft_z_proj(R* data, int N1, int M, int B, SpecTables<R> tb, R scale, Skip skip, int kymajor) {
  using C = cplx<R>;
  using LS = ZLine<L>;
  extern __shared__ __align__(16) char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  C* stw = lds + L * B;
  R* scz = reinterpret_cast<R*>(stw + L);
  R* ssz = scz + L;
  if (skip(blockIdx.z)) return;
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    stw[k] = tb.tw0[k];
    scz[k] = tb.cz[k];
    ssz[k] = tb.sz[k];
  }
  __syncthreads();
  const int col = threadIdx.x % B;
  const int t = threadIdx.x / B;
  // workgroup order: kx tiles fastest (grid M/B x N1), or ky fastest
  // (grid N1 x M/B: consecutive workgroups then sit 16 M bytes apart
  // instead of 16 B bytes, spreading concurrent accesses over the plane)
  const int kx = (kymajor ? blockIdx.y : blockIdx.x) * B + col;
  const int ky = kymajor ? blockIdx.x : blockIdx.y;
  const int i = blockIdx.z;
  const long plane = (long)N1 * M;
  const long comp = (long)L * plane;
  // (ky, kx) factors of the rotated vector: r = (sz cy cx, cz sy cx, cz cy sx)
  const R cy = tb.cy[ky], sy = tb.sy[ky], cx = tb.cx[kx], sx = tb.sx[kx];
  const R fx0 = cy * cx, fx1 = sy * cx, fx2 = cy * sx;
  C* base = reinterpret_cast<C*>(data) + (long)ky * M + kx;
  C acc[LS::E];
#pragma unroll
  for (int e = 0; e < LS::E; ++e) acc[e] = mk<C>(R(0), R(0));
#pragma unroll 1
  for (int l = 0; l < 3; ++l) {
    const C* src = base + (3 * i + l) * comp;
    C v[LS::E];
#pragma unroll
    for (int e = 0; e < LS::E; ++e) v[e] = src[LS::idxA(t, e) * plane];
    LS::template fwd<false>(v, lds + col, B, t, stw);
#pragma unroll
    for (int e = 0; e < LS::E; ++e) {
      const int kz = LS::idxB(t, e);
      const R rl = (l == 0) ? ssz[kz] * fx0 : scz[kz] * (l == 1 ? fx1 : fx2);
      acc[e] = mk<C>(acc[e].x + v[e].x * rl, acc[e].y + v[e].y * rl);
    }
  }
#pragma unroll
  for (int e = 0; e < LS::E; ++e) {
    const int kz = LS::idxB(t, e);
    const R a = ssz[kz] * fx0, b = scz[kz] * fx1, c = scz[kz] * fx2;
    const R r2 = a * a + b * b + c * c;
    const R f = (r2 > R(0)) ? scale / r2 : R(0);
    acc[e] = cscale(acc[e], f);
  }
#pragma unroll 1
  for (int j = 0; j < 3; ++j) {
    C v[LS::E];
#pragma unroll
    for (int e = 0; e < LS::E; ++e) {
      const int kz = LS::idxB(t, e);
      const R rj = (j == 0) ? ssz[kz] * fx0 : scz[kz] * (j == 1 ? fx1 : fx2);
      v[e] = cscale(acc[e], rj);
    }
    LS::inv(v, lds + col, B, t, stw);
    if (kx != 0) {
      C* dst = base + (3 * i + j) * comp;
#pragma unroll
      for (int e = 0; e < LS::E; ++e) dst[LS::idxA(t, e) * plane] = v[e];
    }
  }
}


// Forward N1 pass of the projection in its potential form, one row i of the
// 3x3 field per workgroup.  With the rotated-scheme vector r of eq. (28),
//   sum_l A_il r_l = sz (cy cx A_i0) + cz (sy cx A_i1 + cy sx A_i2)
// (c* = cos(q/2), s* = (2/h) sin(q/2) per axis), so the two terms sharing the
// N0 factor cz are merged here, after their N1 transform, and the fused N0
// pass transforms two fields per row instead of three.  Writes
//   slot 3i     <- cy cx A_i0
//   slot 3i + 1 <- sy cx A_i1 + cy sx A_i2
// and leaves slot 3i + 2, which nothing reads afterwards.  The kx = 0 column
// packs the real columns kx = 0 and kx = N2/2, whose factors differ: it is
// stored transformed, unscaled and unmerged in all three slots (k_fft_z_dc
// separates it).  Grid (M/B, N0, 3 rows per item); element e of component l
// of the row: data + blockIdx.z * zstride + blockIdx.y * ystride + l * cstride
// + e * estride + kx.  The line transform's twiddles are staged in LDS.
// The loads of the next component are issued before the current one is
// transformed (its registers are free by then).
// Line transform of k_fft_axis_rows: the three-stage line where there is one
// (N1 = 96, 128, 256: two lines of 8 complex per thread); single precision
// takes two adjacent columns per thread, exchanged through LDS together.
template <typename R, int L> using RowLine = ZLine<L>;

template <typename R, int L, int CPT>
__global__ void __launch_bounds__(256)
k_fft_axis_rows(R* data, long estride, long ystride, long zstride, long cstride, int B, SpecTables<R> tb,
                Skip skip, const double* __restrict__ pap_partials, int nparts, KrylovScalars* ks, R* dcb) {
  static_assert(CPT == 1 || (CPT == 2 && sizeof(R) == 4), "column pairs in single precision");
  using C = cplx<R>;
  using LS = RowLine<R, L>;
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ double red[16];
  C* lds = reinterpret_cast<C*>(smem_raw);
  C* stw = lds + L * B;
  if (skip((long)blockIdx.y + (long)gridDim.y * blockIdx.z)) return;
  if (pap_partials && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z % 3 == 0) {
    // in the CG: the step length of the item from the front's partial sums
    // of p.Ap (nothing before the residual update reads it)
    const int item = blockIdx.z / 3;
    const double s = sum_partials(pap_partials + (long)item * nparts, nparts, red);
    if (threadIdx.x == 0) krylov_alpha(ks + item, s, 0);
  }
  for (int k = threadIdx.x; k < L; k += blockDim.x) stw[k] = tb.tw1[k];
  __syncthreads();
  const R* scy = tb.cy;
  const R* ssy = tb.sy;
  // CPT adjacent columns per thread (single precision: two, one 16-byte
  // access per element)
  const int BC = B / CPT;
  const int col0 = CPT * (int)(threadIdx.x % BC);
  const int t = threadIdx.x / BC;
  const int kx0 = blockIdx.x * B + col0;
  bool dc[CPT];
  R cx[CPT], sx[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    dc[c] = kx0 + c == 0;
    cx[c] = tb.cx[kx0 + c];
    sx[c] = tb.sx[kx0 + c];
  }
  // workgroup-uniform bases of the three slots and a 32-bit byte offset per
  // thread (within one plane of one component)
  C* b0 = reinterpret_cast<C*>(data) + (long)blockIdx.z * zstride + (long)blockIdx.y * ystride + (long)blockIdx.x * B;
  C* b1 = b0 + cstride;
  C* b2 = b1 + cstride;
  const unsigned ues = (unsigned)(estride * (long)sizeof(C));
  const unsigned ucol = (unsigned)(col0 * sizeof(C));
  auto offA = [&](int e) { return ucol + (unsigned)LS::idxA(t, e) * ues; };
  auto offB = [&](int e) { return ucol + (unsigned)LS::idxB(t, e) * ues; };
  // double precision: streaming loads and stores (measured at 256^3: 426 ->
  // 418 us; in single precision they made the pass slower, 210 -> 219 us);
  // single precision streams its stores only (the pass unchanged, the N0 pass
  // that reads them 144 -> 140 us)
  auto load = [&](C* b, unsigned off, C (&x)[CPT]) {
    if constexpr (CPT == 2) {
      const float4 w = at_bytes(reinterpret_cast<float4*>(b), off);
      x[0] = mk<C>(w.x, w.y);
      x[CPT - 1] = mk<C>(w.z, w.w);
    } else if constexpr (sizeof(R) == 8) {
      x[0] = ld_stream(&at_bytes(b, off));
    } else {
      x[0] = at_bytes(b, off);
    }
  };
  auto store = [&](C* b, unsigned off, const C (&x)[CPT]) {
    if constexpr (CPT == 2)
      st_stream_f4(&at_bytes(reinterpret_cast<float4*>(b), off), make_float4(x[0].x, x[0].y, x[CPT - 1].x, x[CPT - 1].y));
    else if constexpr (sizeof(R) == 8)
      st_stream(&at_bytes(b, off), x[0]);
    else
      at_bytes(b, off) = x[0];
  };
  // the kx = 0 column also goes to dcb (when given): slot s of row
  // blockIdx.z at ((3 blockIdx.z + s) L + ky) N0 + i0, N0 = gridDim.y,
  // i0 = blockIdx.y (a uniform base per row and a 32-bit byte offset)
  const bool dcl = dcb != nullptr && dc[0];
  C* dcw = dcb ? reinterpret_cast<C*>(dcb) + (long)blockIdx.z * 3 * L * gridDim.y : nullptr;
  const unsigned dcs = gridDim.y * (unsigned)sizeof(C);  // ky stride in bytes
  const unsigned dci = blockIdx.y * (unsigned)sizeof(C);
  auto dc_off = [&](int s, int ky) { return (unsigned)(s * L + ky) * dcs + dci; };
  C v[CPT][LS::E], acc[CPT][LS::E];
#pragma unroll
  for (int e = 0; e < LS::E; ++e) {
    C x[CPT], y[CPT];
    load(b0, offA(e), x);
    load(b1, offA(e), y);
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      v[c][e] = x[c];
      acc[c][e] = y[c];
    }
  }
  LS::template fwd_cols<false, CPT>(v, lds + col0, B, t, stw);
#pragma unroll
  for (int e = 0; e < LS::E; ++e) {
    const R cyk = scy[LS::idxB(t, e)];
    C x[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) x[c] = dc[c] ? v[c][e] : cscale(v[c][e], cyk * cx[c]);
    store(b0, offB(e), x);
    if (dcl) at_bytes(dcw, dc_off(0, LS::idxB(t, e))) = v[0][e];
  }
#pragma unroll
  for (int e = 0; e < LS::E; ++e) {
    C x[CPT];
    load(b2, offA(e), x);
#pragma unroll
    for (int c = 0; c < CPT; ++c) v[c][e] = x[c];
  }
  LS::template fwd_cols<false, CPT>(acc, lds + col0, B, t, stw);
  LS::template fwd_cols<false, CPT>(v, lds + col0, B, t, stw);
#pragma unroll
  for (int e = 0; e < LS::E; ++e) {
    const int ky = LS::idxB(t, e);
    C x[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      if (dc[c]) {
        at_bytes(b2, offB(e) + (unsigned)(c * sizeof(C))) = v[c][e];
        x[c] = acc[c][e];
        if (dcl) {
          at_bytes(dcw, dc_off(1, ky)) = acc[c][e];
          at_bytes(dcw, dc_off(2, ky)) = v[c][e];
        }
      } else {
        const R f1 = ssy[ky] * cx[c], f2 = scy[ky] * sx[c];
        x[c] = mk<C>(acc[c][e].x * f1 + v[c][e].x * f2, acc[c][e].y * f1 + v[c][e].y * f2);
      }
    }
    store(b1, offB(e), x);
  }
}

// LDS bytes of k_fft_z_grad3 beyond the L x B exchange buffer: the stage
// twiddles and two kz tables (cos, scaled sin).
template <typename R> constexpr size_t zgrad_extra_lds(int L) {
  return (size_t)L * sizeof(cplx<R>) + 2 * (size_t)L * sizeof(R);
}

// N0 pass fused with the projection, potential form (eq. (28) with the
// rotated scheme).  The projected field Z_ij = w_i r_j, w_i = (sum_l A_il r_l)
// scale / |r|^2, is the corner-stencil gradient of the 3-component potential
// U_i = -i e^{i Phi} w_i, Phi = (q0 + q1 + q2) / 2: the stencil
//   (D_j U)[n] = 1/(4 h_j) sum over the 4 edges of the voxel parallel to j
//                of the corner difference (corner n - 1/2 stored at n - 1)
// has the symbol i e^{-i Phi} r_j.  Only U is transformed back (one inverse
// per row instead of three); U_i is stored in component slot 3 i of the item,
// and its gradient is formed in real space by the corner stencil
// (k_cg_rupd_march, k_grad_store).  The input is the output of
// k_fft_axis_rows: slot 3i holds cy cx A_i0 and slot 3i + 1 holds
// sy cx A_i1 + cy sx A_i2, so that sum_l A_il r_l = sz X_0 + cz X_1 with X_0,
// X_1 the N0 transforms of the two slots x0, x1.  With sz = (2 / h0)
// sin(qz / 2) and cz = cos(qz / 2), e^{i qz / 2} (sz X_0 + cz X_1) is the
// transform of the two-point stencil along N0
//   c[n] = (x1[n] + x1[n + 1]) / 2 - i (x0[n + 1] - x0[n]) / h0,
// so each row takes one forward transform (of c) and one inverse instead of
// two and one, and the phase e^{i qz / 2} of U needs no kz factor (measured
// at 256^3 with the kx = 0 pairs: 272 -> 271 us FP64; 141 -> 132 us FP32,
// where the freed registers also allow 4 waves per SIMD).  Grid (M/B, N1,
// 3 rows per item), or (N1, M/B, rows) with kymajor.  The kx = 0 column is
// left to k_fft_z_dc<OP = 2>, or with DC to a leading slice z = 0 of this
// launch that runs the same body (dc_lead pairs); the rows then start at
// z = 1.  The rows' workgroups read the kx = 0 column too but never use or
// store what they compute for it.
template <typename R, int L, int CPT, bool DC = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((sizeof(R) == 4 && CPT == 1) ? 4 : 1)))
k_fft_z_grad3(R* data, int N1, int M, int B, SpecTables<R> tb, R scale, Skip skip, int kymajor, int dc_lead = 0,
              const R* dcb = nullptr) {
  static_assert(CPT == 1 || (CPT == 2 && sizeof(R) == 4), "column pairs in single precision");
  using C = cplx<R>;
  using LS = typename ZGradSel<R, L>::type;
  extern __shared__ __align__(16) char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  C* stw = lds + L * B;
  R* scz = reinterpret_cast<R*>(stw + L);
  R* ssz = scz + L;
  if constexpr (DC) {
    // leading slice: the kx = 0 column pairs (the body of k_fft_z_dc<OP = 2>,
    // one pair per workgroup), so that they start first and overlap the rest
    if (blockIdx.z == 0) {
      const int b = (int)(blockIdx.y * gridDim.x + blockIdx.x);
      if (b < dc_lead) {
        const int ky0 = b % (N1 / 2 + 1), row = b / (N1 / 2 + 1);
        if (!skip(row))
          z_dc_body<R, L, 2>(data, N1, M, tb, scale, 0.0, 0.0, ky0, row, lds, lds + z_dc_groups<2>() * 2 * L,
                             reinterpret_cast<const C*>(dcb));
      }
      return;
    }
  }
  const int i = (int)blockIdx.z - (DC ? 1 : 0);  // row of the 3x3 field, items consecutive
  if (skip(i)) return;
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    stw[k] = tb.tw0[k];
    scz[k] = tb.cz[k];
    ssz[k] = tb.sz[k];
  }
  __syncthreads();
  // CPT adjacent columns per thread (single precision: two, one 16-byte
  // access per row, so that a tile row is a whole 128-byte line)
  const int BC = B / CPT;
  const int col0 = CPT * (int)(threadIdx.x % BC);
  const int t = threadIdx.x / BC;
  const int kx0 = (kymajor ? blockIdx.y : blockIdx.x) * B + col0;
  const int ky = kymajor ? blockIdx.x : blockIdx.y;
  const long plane = (long)N1 * M;
  const long comp = (long)L * plane;
  // workgroup-uniform base of the row's first slot and a 32-bit element
  // offset per thread (col + kz plane; a component is < 2^32 bytes)
  C* base = reinterpret_cast<C*>(data) + (long)(3 * i) * comp + (long)ky * M + (kx0 - col0);
  const unsigned uplane = (unsigned)plane;
  const unsigned ucomp = (unsigned)comp;
  // every element is read once and written once: streaming loads and stores
  // in both precisions (measured at 256^3: 306 -> 284 us FP64, 180 -> 167 us
  // FP32, this pass with its kx = 0 kernel; the following inverse N1 pass also
  // ran faster, 148 -> 133 us)
  // the unit's (ky, kx) factors are loaded with its data, not after the
  // transforms (a second memory latency per workgroup)
  R cxs[CPT], sxs[CPT], snxs[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    cxs[c] = tb.cx[kx0 + c];
    sxs[c] = tb.sx[kx0 + c];
    snxs[c] = tb.snx[kx0 + c];
  }
  const R cy = tb.cy[ky], sy = tb.sy[ky], sny = tb.sny[ky];
  C v[CPT][LS::E], acc[CPT][LS::E];
  if constexpr (CPT == 2) {
#pragma unroll
    for (int e = 0; e < LS::E; ++e) {
      const float4 a = ld_stream_f4(base + (unsigned)col0 + (unsigned)LS::idxA(t, e) * uplane);
      const float4 b = ld_stream_f4(base + ucomp + (unsigned)col0 + (unsigned)LS::idxA(t, e) * uplane);
      v[0][e] = mk<C>(a.x, a.y);
      v[1][e] = mk<C>(a.z, a.w);
      acc[0][e] = mk<C>(b.x, b.y);
      acc[1][e] = mk<C>(b.z, b.w);
    }
  } else {
#pragma unroll
    for (int e = 0; e < LS::E; ++e) v[0][e] = ld_stream(base + (unsigned)col0 + (unsigned)LS::idxA(t, e) * uplane);
#pragma unroll
    for (int e = 0; e < LS::E; ++e) acc[0][e] = ld_stream(base + ucomp + (unsigned)col0 + (unsigned)LS::idxA(t, e) * uplane);
  }
  // every load is issued before the first transform: the scheduler would
  // otherwise put the first column's arithmetic (and a wait for it) ahead of
  // the second slot's loads (measured at 256^3: 294 -> 281 us FP64, 167 ->
  // 162 us FP32, with the kx = 0 kernel)
  __builtin_amdgcn_sched_barrier(0);
  // the stencil c[n] = p[n] + s[n + 1] with p = x1 / 2 + i x0 / h0 and
  // s = x1 / 2 - i x0 / h0 (s[n + 1] from the thread that holds it, through
  // LDS; 1 / h0 from the tables: sz[1] = (2 / h0) snz[1])
  const R rh0 = (L >= 2) ? tb.sz[1] / (R(2) * tb.snz[1]) : R(0);
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int e = 0; e < LS::E; ++e) {
      const C x0 = v[c][e], x1 = acc[c][e];
      const C ix0 = mk<C>(-x0.y * rh0, x0.x * rh0);  // i x0 / h0
      v[c][e] = mk<C>(R(0.5) * x1.x + ix0.x, R(0.5) * x1.y + ix0.y);    // p
      acc[c][e] = mk<C>(R(0.5) * x1.x - ix0.x, R(0.5) * x1.y - ix0.y);  // s
      lds[LS::idxA(t, e) * B + col0 + c] = acc[c][e];
    }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int e = 0; e < LS::E; ++e) {
      const int n = LS::idxA(t, e) + 1;
      v[c][e] = cadd(v[c][e], lds[(n == L ? 0 : n) * B + col0 + c]);
    }
  __syncthreads();  // every s read before the transform's exchange
  LS::template fwd_cols<false, CPT>(v, lds + col0, B, t, stw);
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const R cx = cxs[c], sx = sxs[c];
    const R fx0 = cy * cx, fx1 = sy * cx, fx2 = cy * sx;
    // -i e^{i (qy + qx) / 2} (the kz half of the phase is in the stencil)
    const C eyx = mul_mi(cmul(mk<C>(cy, sny), mk<C>(cx, snxs[c])));
#pragma unroll
    for (int e = 0; e < LS::E; ++e) {
      const int kz = LS::idxB(t, e);
      const R sz = ssz[kz], cz = scz[kz];
      const R a = sz * fx0, b = cz * fx1, cc = cz * fx2;
      const R r2 = a * a + b * b + cc * cc;
      const R f = (r2 > R(0)) ? scale / r2 : R(0);
      acc[c][e] = cmul(cscale(v[c][e], f), eyx);
    }
  }
  LS::template inv_cols<CPT>(acc, lds + col0, B, t, stw);
  // the kx = 0 column is k_fft_z_dc's
  if constexpr (CPT == 2) {
#pragma unroll
    for (int e = 0; e < LS::E; ++e) {
      C* dst = base + (unsigned)col0 + (unsigned)LS::idxA(t, e) * uplane;
      if (kx0 != 0)
        st_stream_f4(dst, make_float4(acc[0][e].x, acc[0][e].y, acc[1][e].x, acc[1][e].y));
      else
        dst[1] = acc[1][e];
    }
  } else {
    if (kx0 != 0) {
#pragma unroll
      for (int e = 0; e < LS::E; ++e) st_stream(base + (unsigned)col0 + (unsigned)LS::idxA(t, e) * uplane, acc[0][e]);
    }
  }
}

}  // namespace fg
