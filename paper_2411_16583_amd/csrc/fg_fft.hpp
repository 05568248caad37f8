// Batched 1-D FFTs of one line length L inside a workgroup, and the three
// axis passes of the 3-D real transform used by the Fourier-Galerkin
// operator (Sec. 3.2 "FFT resolution algorithms", eq. (30)).
//
// Line algorithm: two-stage Cooley-Tukey with L = R1 * R2.  T threads share a
// line (T = gcd(R1, R2)); each thread keeps E = L / T elements in registers
// and the only exchange between the stages goes through LDS:
//   layout A (natural): thread t holds x[(t + T u) + R2 n1], e = u R1 + n1
//   layout B (spectral): thread t holds X[(t + T v) + R1 k2], e = v R2 + k2
// fwd: A -> B (stage 1 radix R1 over n1, twiddle W_L^{b k1}, stage 2 radix R2)
// inv: B -> A (the mirror image), so a spectrum produced by fwd can be
// multiplied pointwise and transformed back without any reordering.
//
// 3-D real layout: (C, N0, N1, N2) with N2 fastest.  The half spectrum is
// stored "packed" in exactly the same bytes, (C, N0, N1, M) complex with
// M = N2 / 2: along N2 the DC and Nyquist coefficients of a real line are
// both real, and X[0] holds (Re X_0, Re X_M).  After the N1 and N0 passes
// the kx = 0 column therefore carries A + i B, A and B being the 2-D spectra
// of the kx = 0 and kx = M planes; the pointwise operator separates them with
// the partner column at (-kz, -ky) (kernel k_fft_z_dc).
#pragma once
#include "fg_complex.hpp"

namespace fg {

// Device-side scalars of one Krylov solve (FP64, in the workspace).
struct KrylovScalars {
  double rr;     // current r.r
  double rr0;    // b.b
  double rz;     // r.z (preconditioned solves)
  double pAp;
  double alpha;
  double beta;
  double tol2;   // tol^2 (0: run to maxit)
  int iter;
  int maxit;
  int done;      // 1 when converged, broken down or out of iterations
  int flag;      // 0 running/converged, 1 breakdown, 2 max iterations
};

// Which batch item a workgroup belongs to and whether that item is masked
// off; workgroups of masked items return at once.  The mask is one int word
// per item (nonzero: skip), either the done flag of the item's Krylov
// scalars or a separate per-item flag array.  A plan is a batch of one item.
struct Skip {
  const int* gate = nullptr;  // nullptr: never skip
  int stride = 0;             // ints between the words of consecutive items
  long per_item = 1L << 62;   // grid units (lines, planes or rows) per item
  long item_stride = 0;       // real passes: lines between the first lines of consecutive items (0: per_item)
  int sub = 1;                // real passes: per_item counts sub-items, sub of them per gated item
  __host__ __device__ int item(long unit) const { return (int)(unit / per_item); }
  __device__ __forceinline__ bool operator()(long unit) const {
    return gate && gate[(long)item(unit) * stride] != 0;
  }
  // skip items whose Krylov solve is done
  static Skip done(const KrylovScalars* ks, long per_item = 1L << 62) {
    Skip s;
    s.gate = &ks->done;
    s.stride = (int)(sizeof(KrylovScalars) / sizeof(int));
    s.per_item = per_item;
    return s;
  }
  // skip items with flags[b] != 0
  static Skip flags(const int* f, long per_item = 1L << 62) {
    Skip s;
    s.gate = f;
    s.stride = 1;
    s.per_item = per_item;
    return s;
  }
  Skip unit(long per) const {
    Skip s = *this;
    s.per_item = per;
    return s;
  }
  __device__ __forceinline__ bool masked(int item) const { return gate && gate[(long)(item / sub) * stride] != 0; }
  // Workgroups of lpb lines over nlines lines (per_item lines per item) that
  // never straddle two items: ceil(lines per item / lpb) workgroups per item.
  __host__ __device__ long item_lines(long nlines) const { return per_item < nlines ? per_item : nlines; }
  __host__ __device__ long line_blocks(long nlines, int lpb) const {
    const long lpi = item_lines(nlines);
    return (nlines / lpi) * ((lpi + lpb - 1) / lpb);
  }
};

// Line of thread row ll of this workgroup under the item-aligned split.
struct LineMap {
  long line;    // global line index
  bool active;  // inside its item
  int item;
};
__device__ __forceinline__ LineMap map_line(const Skip& sk, long nlines, int lpb, int ll) {
  const long lpi = sk.item_lines(nlines);
  const long bpi = (lpi + lpb - 1) / lpb;
  const long it = (long)blockIdx.x / bpi;
  const long lin = ((long)blockIdx.x - it * bpi) * lpb + ll;
  return LineMap{it * (sk.item_stride > 0 ? sk.item_stride : lpi) + lin, lin < lpi, (int)it};
}
static_assert(sizeof(KrylovScalars) % sizeof(int) == 0, "gate stride");

template <int L> struct LineShape;
#define FG_LINE_SHAPE(L_, R1_, R2_) \
  template <> struct LineShape<L_> { static constexpr int R1 = R1_, R2 = R2_; };
FG_LINE_SHAPE(1, 1, 1)
FG_LINE_SHAPE(2, 2, 1)
FG_LINE_SHAPE(3, 3, 1)
FG_LINE_SHAPE(4, 4, 1)
FG_LINE_SHAPE(6, 6, 1)
FG_LINE_SHAPE(8, 8, 1)
FG_LINE_SHAPE(12, 12, 1)
FG_LINE_SHAPE(16, 4, 4)
FG_LINE_SHAPE(24, 6, 4)
FG_LINE_SHAPE(32, 8, 4)
FG_LINE_SHAPE(48, 12, 4)
FG_LINE_SHAPE(64, 8, 8)
FG_LINE_SHAPE(96, 12, 8)
FG_LINE_SHAPE(128, 16, 8)
FG_LINE_SHAPE(256, 16, 16)
FG_LINE_SHAPE(512, 32, 16)
#undef FG_LINE_SHAPE

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

template <int L> struct Line {
  static constexpr int R1 = LineShape<L>::R1;
  static constexpr int R2 = LineShape<L>::R2;
  static constexpr int T = (R2 == 1) ? 1 : cgcd(R1, R2);
  static constexpr int U = R2 / T;
  static constexpr int V = R1 / T;
  static constexpr int E = L / T;
  __device__ __forceinline__ static int idxA(int t, int e) {
    return t + T * (e / R1) + R2 * (e % R1);
  }
  __device__ __forceinline__ static int idxB(int t, int e) {
    return t + T * (e / R2) + R1 * (e % R2);
  }
};

// Multiply by the stage twiddle W_L^{j} (table tw[j] = e^{-2 pi i j / L}).
template <bool INV, typename C>
__device__ __forceinline__ C twiddle_tab(C a, const C* __restrict__ tw, int j) {
  C w = tw[j];
  return INV ? cmulc(a, w) : cmul(a, w);
}

// Forward (or, with INV, inverse) DFT of a line, layout A -> layout B.
// lds: the line's exchange buffer, element i at lds[i * ls].  Ends with a
// barrier so that the caller may reuse the buffer immediately.
// Order LDS accesses: across the workgroup, or (WAVE) within the wave only,
// for lines that no other wave touches.
template <bool WAVE> __device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int L, bool INV, typename C, bool WAVE = false>
__device__ __forceinline__ void line_fft_AB(C (&v)[Line<L>::E], C* lds, int ls, int t,
                                            const C* __restrict__ tw) {
  using LS = Line<L>;
  if constexpr (LS::R2 == 1) {
    Dft<LS::R1, 1, INV, C>::run(v);
  } else {
#pragma unroll
    for (int u = 0; u < LS::U; ++u) {
      const int b = t + LS::T * u;
      Dft<LS::R1, 1, INV, C>::run(v + u * LS::R1);
#pragma unroll
      for (int k1 = 1; k1 < LS::R1; ++k1)
        v[u * LS::R1 + k1] = twiddle_tab<INV>(v[u * LS::R1 + k1], tw, (b * k1) % L);
#pragma unroll
      for (int k1 = 0; k1 < LS::R1; ++k1) lds[(k1 * LS::R2 + b) * ls] = v[u * LS::R1 + k1];
    }
    lds_sync<WAVE>();
#pragma unroll
    for (int w = 0; w < LS::V; ++w) {
      const int k1 = t + LS::T * w;
#pragma unroll
      for (int n2 = 0; n2 < LS::R2; ++n2) v[w * LS::R2 + n2] = lds[(k1 * LS::R2 + n2) * ls];
      Dft<LS::R2, 1, INV, C>::run(v + w * LS::R2);
    }
    lds_sync<WAVE>();
  }
}

// Inverse DFT of a line, layout B -> layout A (mirror of line_fft_AB).
template <int L, typename C>
__device__ __forceinline__ void line_ifft_BA(C (&v)[Line<L>::E], C* lds, int ls, int t,
                                             const C* __restrict__ tw) {
  using LS = Line<L>;
  if constexpr (LS::R2 == 1) {
    Dft<LS::R1, 1, true, C>::run(v);
  } else {
#pragma unroll
    for (int w = 0; w < LS::V; ++w) {
      const int k1 = t + LS::T * w;
      Dft<LS::R2, 1, true, C>::run(v + w * LS::R2);
#pragma unroll
      for (int n2 = 1; n2 < LS::R2; ++n2)
        v[w * LS::R2 + n2] = twiddle_tab<true>(v[w * LS::R2 + n2], tw, (n2 * k1) % L);
#pragma unroll
      for (int n2 = 0; n2 < LS::R2; ++n2) lds[(n2 * LS::R1 + k1) * ls] = v[w * LS::R2 + n2];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < LS::U; ++u) {
      const int n2 = t + LS::T * u;
#pragma unroll
      for (int k1 = 0; k1 < LS::R1; ++k1) v[u * LS::R1 + k1] = lds[(n2 * LS::R1 + k1) * ls];
      Dft<LS::R1, 1, true, C>::run(v + u * LS::R1);
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// Deterministic block reduction of one double per thread.  Fixed shuffle tree
// within a wave, then wave partials summed in order by thread 0.
__device__ __forceinline__ double block_sum(double v, double* red /*>= 16 doubles in LDS*/) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < nw; ++k) s += red[k];
  return s;  // valid in thread 0 only
}

// Sum of nparts partials in a fixed order by one block (deterministic).
// Each thread keeps eight independent running sums, so that eight loads are
// in flight per thread instead of one (the partials come from other XCDs'
// L2 or from HBM).
__device__ __forceinline__ double sum_partials(const double* __restrict__ partials, int nparts, double* red) {
  const int bd = blockDim.x;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int k = threadIdx.x;
  for (; k + 7 * bd < nparts; k += 8 * bd) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += partials[k + u * bd];
  }
  for (; k < nparts; k += bd) a[0] += partials[k];
  const double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  return block_sum(acc, red);
}

// CG step length from s = p.Ap (or p.Aq): alpha = r.r / s (r.z / s
// preconditioned), or breakdown when s <= 0.  One thread.
__device__ __forceinline__ void krylov_alpha(KrylovScalars* ks, double s, int pcg) {
  ks->pAp = s;
  if (!(s > 0.0)) {
    ks->done = 1;
    ks->flag = 1;
  } else {
    ks->alpha = (pcg ? ks->rz : ks->rr) / s;
  }
}

// Tables of one 3-D plan (device pointers), in the working precision R.
template <typename R> struct SpecTables {
  const cplx<R>* tw0;   // W_{N0}^j, j < N0
  const cplx<R>* tw1;   // W_{N1}^j
  const cplx<R>* twM;   // W_M^j, M = N2/2
  const cplx<R>* post;  // W_{N2}^k, k < M (real <-> half-length complex)
  const R* cz;          // cos(pi kz / N0), exact 0 at kz = N0/2
  const R* sz;          // (2/h0) sin(pi kz / N0)
  const R* cy;          // cos(pi ky / N1)
  const R* sy;          // (2/h1) sin(pi ky / N1)
  const R* cx;          // cos(pi kx / N2), kx = 0..M, exact 0 at kx = M
  const R* sx;          // (2/h2) sin(pi kx / N2)
  const R* snz;         // sin(pi kz / N0)  (half-voxel phase factors e^{i q / 2})
  const R* sny;         // sin(pi ky / N1)
  const R* snx;         // sin(pi kx / N2), kx = 0..M
};

// ----------------------------------------------------------------------------
// Pass 1: real-to-complex along N2 for nlines lines (in place allowed).
// Workgroups of the two real passes have XBLOCK threads (LPB lines).
constexpr int XBLOCK = 128;

template <typename R, int M>
__global__ void __launch_bounds__(XBLOCK)
k_fft_x_r2c(const R* in, R* out, long nlines, SpecTables<R> tb, Skip skip) {
  using C = cplx<R>;
  using LS = Line<M>;
  constexpr int LPB = XBLOCK / LS::T;
  constexpr int PAD = (M >= 16) ? 1 : 0;
  __shared__ C lds[LPB * (M + PAD)];
  const int t = threadIdx.x % LS::T;
  const int ll = threadIdx.x / LS::T;
  const LineMap lm = map_line(skip, nlines, LPB, ll);
  if (skip.masked(lm.item)) return;
  const long line = lm.line;
  const bool active = lm.active;
  const C* src = reinterpret_cast<const C*>(in) + line * M;
  C* dst = reinterpret_cast<C*>(out) + line * M;
  C* my = lds + ll * (M + PAD);
  C v[LS::E];
#pragma unroll
  for (int e = 0; e < LS::E; ++e) v[e] = active ? src[LS::idxA(t, e)] : mk<C>(R(0), R(0));
  line_fft_AB<M, false>(v, my, 1, t, tb.twM);
#pragma unroll
  for (int e = 0; e < LS::E; ++e) my[LS::idxB(t, e)] = v[e];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < LS::E; ++e) {
    const int k = LS::idxB(t, e);
    const C zk = my[k];
    C X;
    if (k == 0) {
      X = mk<C>(zk.x + zk.y, zk.x - zk.y);  // (Re X_0, Re X_M)
    } else {
      const C zm = my[M - k];
      const C ev = cscale(cadd(zk, cconj(zm)), R(0.5));
      const C od = cscale(mul_mi(csub(zk, cconj(zm))), R(0.5));
      X = cadd(ev, cmul(od, tb.post[k]));
    }
    if (active) dst[k] = X;
  }
}

// Epilogue of the inverse real pass: y = scale * x_out is stored (type R,
// into out) and sum(y * dotv) (or sum(y*y) when dotv == nullptr) is reduced
// per block into partials[blockIdx.x] (FP64).  A block skips everything when
// *skip is nonzero.
struct C2REpi {
  double scale;
  const void* dotv;  // same type R as the output, or nullptr
  bool self_dot;     // sum y*y
  double* partials;  // nullptr: no reduction
  Skip skip;         // per-item early exit (units: lines)
};

template <typename R, int M>
__global__ void __launch_bounds__(XBLOCK)
k_fft_x_c2r(const R* in, R* out, long nlines, SpecTables<R> tb, C2REpi epi) {
  using C = cplx<R>;
  using LS = Line<M>;
  constexpr int LPB = XBLOCK / LS::T;
  constexpr int PAD = (M >= 16) ? 1 : 0;
  __shared__ C lds[LPB * (M + PAD)];
  __shared__ double red[16];
  // the line's stage twiddles and the C2R pre-processing factors, read once
  // per workgroup (the barrier after the line load orders them); from the
  // caches they cost the pass 71 -> 65 us in single precision at 256^3
  __shared__ C stw[M], spost[M];
  for (int k = threadIdx.x; k < M; k += XBLOCK) {
    stw[k] = tb.twM[k];
    spost[k] = tb.post[k];
  }
  const int t = threadIdx.x % LS::T;
  const int ll = threadIdx.x / LS::T;
  const LineMap lm = map_line(epi.skip, nlines, LPB, ll);
  if (epi.skip.masked(lm.item)) return;
  const long line = lm.line;
  const bool active = lm.active;
  const C* src = reinterpret_cast<const C*>(in) + line * M;
  C* my = lds + ll * (M + PAD);
  // one global load per element; the mirror X[M - k] comes from LDS.  Double
  // precision streams both ways (measured at 256^3 on the 3-component
  // potential: 159 -> 143 us; single precision got slower, 71 -> 103 us)
  C v[LS::E];
#pragma unroll
  for (int e = 0; e < LS::E; ++e)
    v[e] = active ? (sizeof(R) == 8 ? ld_stream(src + LS::idxA(t, e)) : src[LS::idxA(t, e)]) : mk<C>(R(0), R(0));
#pragma unroll
  for (int e = 0; e < LS::E; ++e) my[LS::idxA(t, e)] = v[e];
  __syncthreads();
#pragma unroll
  for (int e = 0; e < LS::E; ++e) {
    const int k = LS::idxA(t, e);
    const C xk = v[e];
    if (k == 0) {
      v[e] = mk<C>(xk.x + xk.y, xk.x - xk.y);
    } else {
      const C xm = my[M - k];
      const C s = cadd(xk, cconj(xm));
      const C d = cmulc(csub(xk, cconj(xm)), spost[k]);  // * W^{-k}
      v[e] = cadd(s, mul_pi(d));
    }
  }
  __syncthreads();  // mirrors read before the exchange overwrites the buffer
  line_fft_AB<M, true>(v, my, 1, t, stw);
  // v[e] = N2 * (x[2n] + i x[2n+1]) with n = idxB(t, e)
  C* dst = reinterpret_cast<C*>(out) + line * M;
  const C* dv = reinterpret_cast<const C*>(epi.dotv) + line * M;
  const R sg = (R)epi.scale;
  double acc = 0.0;
#pragma unroll
  for (int e = 0; e < LS::E; ++e) {
    const int n = LS::idxB(t, e);
    const C y = cscale(v[e], sg);
    if (active) {
      if constexpr (sizeof(R) == 8)
        st_stream(dst + n, y);
      else
        dst[n] = y;
      if (epi.partials) {
        if (epi.self_dot) {
          acc += (double)y.x * (double)y.x + (double)y.y * (double)y.y;
        } else {
          const C q = dv[n];
          acc += (double)y.x * (double)q.x + (double)y.y * (double)q.y;
        }
      }
    }
  }
  if (epi.partials) {
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) epi.partials[blockIdx.x] = s;
  }
}

// ----------------------------------------------------------------------------
// Complex FFT of length L along one axis for tiles of B adjacent kx columns.
// Element e of the line of column col: base + e * estride, with
// base = data + blockIdx.y * ystride + blockIdx.z * zstride + blockIdx.x * B + col
// (complex units).  Used for the N1 pass (estride = M) and, in the diagnostic
// transforms, for the N0 pass (estride = N1 M).  CPT = 2 (single precision):
// each thread owns two adjacent columns, loaded and stored as one 16-byte
// vector, so a tile of B columns takes T B / 2 threads.
// With TWL the stage twiddles are copied into LDS after the exchange buffer
// (L B + L elements of dynamic LDS) and read from there.
template <typename R, int L, bool INV, int CPT, bool TWL = false>
__global__ void __launch_bounds__(256)
k_fft_axis(R* data, long estride, long ystride, long zstride, int B, const cplx<R>* __restrict__ twg,
           Skip skip) {
  using C = cplx<R>;
  using LS = Line<L>;
  extern __shared__ char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  if (skip((long)blockIdx.y + (long)gridDim.y * blockIdx.z)) return;  // unit: plane (y) of line set (z)
  const C* tw = twg;
  if constexpr (TWL) {
    C* stw = lds + L * B;
    for (int k = threadIdx.x; k < L; k += blockDim.x) stw[k] = twg[k];
    __syncthreads();
    tw = stw;
  }
  const int BC = B / CPT;  // column groups per tile
  const int cg = threadIdx.x % BC;
  const int t = threadIdx.x / BC;
  C* base = reinterpret_cast<C*>(data) + (long)blockIdx.y * ystride + (long)blockIdx.z * zstride +
            (long)blockIdx.x * B + CPT * cg;
  if constexpr (CPT == 1) {
    C v[LS::E];
#pragma unroll
    for (int e = 0; e < LS::E; ++e) v[e] = base[(long)LS::idxA(t, e) * estride];
    line_fft_AB<L, INV>(v, lds + cg, B, t, tw);
#pragma unroll
    for (int e = 0; e < LS::E; ++e) base[(long)LS::idxB(t, e) * estride] = v[e];
  } else {
    static_assert(CPT == 2 && sizeof(R) == 4, "column pairs in single precision");
    C v0[LS::E], v1[LS::E];
#pragma unroll
    for (int e = 0; e < LS::E; ++e) {
      const float4 w = *reinterpret_cast<const float4*>(base + (long)LS::idxA(t, e) * estride);
      v0[e] = mk<C>(w.x, w.y);
      v1[e] = mk<C>(w.z, w.w);
    }
    line_fft_AB<L, INV>(v0, lds + 2 * cg, B, t, tw);
    line_fft_AB<L, INV>(v1, lds + 2 * cg + 1, B, t, tw);
#pragma unroll
    for (int e = 0; e < LS::E; ++e)
      *reinterpret_cast<float4*>(base + (long)LS::idxB(t, e) * estride) = make_float4(v0[e].x, v0[e].y, v1[e].x, v1[e].y);
  }
}

// ----------------------------------------------------------------------------
// Pass 3 with the projection (eq. (28), (30)): per row i of the 3x3 field,
// Z_ij = (sum_l A_il r_l) r_j / |r|^2 * scale, r the rotated-scheme vector.
// Grid (M/B, N1, 3 rows).  The kx = 0 column is left to k_fft_z_dc.
template <typename R> struct RVec {
  R x, y, z;
};

template <typename R>
__device__ __forceinline__ RVec<R> rot_vec(const SpecTables<R>& tb, int kz, int ky, int kx) {
  const R cz = tb.cz[kz], sz = tb.sz[kz];
  const R cy = tb.cy[ky], sy = tb.sy[ky];
  const R cx = tb.cx[kx], sx = tb.sx[kx];
  // components along axes 0 (z), 1 (y), 2 (x) of the grid = tensor index j
  RVec<R> r;
  r.x = sz * cy * cx;  // j = 0 (axis 0)
  r.y = cz * sy * cx;  // j = 1 (axis 1)
  r.z = cz * cy * sx;  // j = 2 (axis 2)
  return r;
}

template <typename R>
__device__ __forceinline__ R rget(const RVec<R>& r, int j) {
  return j == 0 ? r.x : (j == 1 ? r.y : r.z);
}

// LDS bytes of k_fft_z_proj / k_fft_z_scalar beyond the L x B exchange buffer:
// the stage twiddles and the kz tables, staged once per workgroup (reading
// them from LDS inside each transform keeps the compiler from holding them in
// registers across the six transforms of a row).
template <typename R> constexpr size_t zpass_extra_lds(int L) {
  return (size_t)L * sizeof(cplx<R>) + 2 * (size_t)L * sizeof(R);
}

// Scalar symbol variant (preconditioners of Alg. 2 / Alg. 3):
//   Z = A * scale / (a0 + a1 lambda(q)),  lambda = sum_j (2/h_j)^2 sin^2(q_j/2).
template <typename R>
__device__ __forceinline__ R lap_sym(const SpecTables<R>& tb, int kz, int ky, int kx) {
  const R a = tb.sz[kz], b = tb.sy[ky], c = tb.sx[kx];
  return a * a + b * b + c * c;
}

template <typename R, int L>
__global__ void __launch_bounds__(256)
k_fft_z_scalar(R* data, int N1, int M, int B, SpecTables<R> tb, R scale, double a0, double a1,
               Skip skip) {
  using C = cplx<R>;
  using LS = Line<L>;
  extern __shared__ char smem_raw[];
  C* lds = reinterpret_cast<C*>(smem_raw);
  C* stw = lds + L * B;
  if (skip(blockIdx.z)) return;
  for (int k = threadIdx.x; k < L; k += blockDim.x) stw[k] = tb.tw0[k];
  __syncthreads();
  const int col = threadIdx.x % B;
  const int t = threadIdx.x / B;
  const int kx = blockIdx.x * B + col;
  const int ky = blockIdx.y;
  const long plane = (long)N1 * M;
  C* base = reinterpret_cast<C*>(data) + (long)ky * M + kx;
  C v[LS::E];
#pragma unroll
  for (int e = 0; e < LS::E; ++e) v[e] = base[LS::idxA(t, e) * plane];
  line_fft_AB<L, false>(v, lds + col, B, t, stw);
#pragma unroll
  for (int e = 0; e < LS::E; ++e) {
    const double den = a0 + a1 * (double)lap_sym(tb, LS::idxB(t, e), ky, kx);
    v[e] = cscale(v[e], (R)((double)scale / den));
  }
  line_ifft_BA<L>(v, lds + col, B, t, stw);
  if (kx != 0) {
#pragma unroll
    for (int e = 0; e < LS::E; ++e) base[LS::idxA(t, e) * plane] = v[e];
  }
}

// kx = 0 column: the packed value is A + i B (A: plane kx = 0, B: plane
// kx = N2/2, both spectra of real fields).  A workgroup takes the column pair
// (ky, -ky), transforms along N0, separates
//   A(k) = (P(k) + conj P(-k)) / 2,   B(k) = (P(k) - conj P(-k)) / (2i),
// applies the operator at qx = 0 to A and at qx = pi to B, and recombines.
// OP = 0: projection, one row per workgroup (grid.y = 3 rows per item);
// OP = 1: scalar symbol (grid.y = 1);
// OP = 2: projection to the 3-component potential (see k_fft_z_grad3), one
//         row per workgroup (grid.y = 3 rows per item), U_i into slot 3 i.
// Components read per row by k_fft_z_dc, one wave per component (the
// components' loads and transforms run side by side).
template <int OP> constexpr int z_dc_groups() { return (OP == 1) ? 1 : 3; }
// LDS of z_dc_body in complex values: an exchange buffer of the column pair
// per wave and the spectra of the components read.
template <int L, int OP> constexpr int z_dc_lds() { return z_dc_groups<OP>() * 2 * L * 2; }

// Body of k_fft_z_dc for the column pair (ky0, -ky0) of row `row` (OP 0, 2)
// with xbuf (NC 2 L) and spec (NC 2 L complex) in LDS; 64 NC threads, wave g
// reading component g (lanes with t >= T take part in the barriers only).
template <typename R, int L, int OP>
__device__ __forceinline__ void z_dc_body(R* data, int N1, int M, const SpecTables<R>& tb, R scale, double a0,
                                          double a1, int ky0, int row, cplx<R>* xbuf, cplx<R>* spec,
                                          const cplx<R>* __restrict__ dcb) {
  using C = cplx<R>;
  using LS = Line<L>;
  constexpr int NC = z_dc_groups<OP>();    // components read per row
  constexpr int NOUT = (OP == 0) ? 3 : 1;  // components written per row
  static_assert(2 * LS::T <= 64, "a column pair of lines per wave");
  const int grp = threadIdx.x / 64;
  const int col = threadIdx.x % 2;
  const int t = (threadIdx.x % 64) / 2;
  // idle lanes (t >= T, and waves beyond the NC components when the body
  // runs in a larger workgroup) still take part in every barrier below
  const bool lane_ok = t < LS::T && grp < NC;
  xbuf += grp * 2 * L;
  const int ky1 = (N1 - ky0) % N1;
  const int myky = col ? ky1 : ky0;
  const long plane = (long)N1 * M;
  const long comp = (long)L * plane;
  C* base = reinterpret_cast<C*>(data) + (long)myky * M;  // kx = 0
  const bool store = lane_ok && (col == 0 || ky1 != ky0);
  {
    // first component read and written by this workgroup's row
    const int cin = (OP == 1) ? 0 : 3 * row;
    const int cout = cin;
    {
      const int l = grp;
      C v[LS::E];
#pragma unroll
      for (int e = 0; e < LS::E; ++e) {
        if (!lane_ok)
          v[e] = mk<C>(R(0), R(0));
        else if (dcb)  // the compact copy of the column: contiguous along N0
          v[e] = dcb[((long)(cin + l) * N1 + myky) * L + LS::idxA(t, e)];
        else
          v[e] = base[(cin + l) * comp + LS::idxA(t, e) * plane];
      }
      if constexpr (LS::R2 == 1) {
        Dft<LS::R1, 1, false, C>::run(v);
      } else {
        // same two-stage transform, guarded for the idle lanes
#pragma unroll
        for (int u = 0; u < LS::U; ++u) {
          const int b = t + LS::T * u;
          Dft<LS::R1, 1, false, C>::run(v + u * LS::R1);
#pragma unroll
          for (int k1 = 1; k1 < LS::R1; ++k1)
            if (lane_ok) v[u * LS::R1 + k1] = twiddle_tab<false>(v[u * LS::R1 + k1], tb.tw0, (b * k1) % L);
          if (lane_ok)
#pragma unroll
            for (int k1 = 0; k1 < LS::R1; ++k1) xbuf[(k1 * LS::R2 + b) * 2 + col] = v[u * LS::R1 + k1];
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < LS::V; ++w) {
          const int k1 = t + LS::T * w;
          if (lane_ok)
#pragma unroll
            for (int n2 = 0; n2 < LS::R2; ++n2) v[w * LS::R2 + n2] = xbuf[(k1 * LS::R2 + n2) * 2 + col];
          Dft<LS::R2, 1, false, C>::run(v + w * LS::R2);
        }
        __syncthreads();
      }
      if (lane_ok)
#pragma unroll
        for (int e = 0; e < LS::E; ++e) spec[(l * 2 + col) * L + LS::idxB(t, e)] = v[e];
    }
    __syncthreads();
    // separate, apply, recombine: thread (t, col) owns kz = idxB(t, e) of its column.
    // With one output (OP 1, 2) the recombined value goes straight into v1;
    // the projection (OP 0, three outputs) keeps tA, tB.
    constexpr int TE = (NOUT == 1) ? 1 : LS::E;
    C tA[TE], tB[TE], v1[LS::E];
#pragma unroll
    for (int e = 0; e < TE; ++e) {
      tA[e] = mk<C>(R(0), R(0));
      tB[e] = mk<C>(R(0), R(0));
    }
#pragma unroll
    for (int e = 0; e < LS::E; ++e) v1[e] = mk<C>(R(0), R(0));
    if (lane_ok) {
#pragma unroll
      for (int e = 0; e < LS::E; ++e) {
        const int kz = LS::idxB(t, e);
        const int kzm = (L - kz) % L;
        C ta = mk<C>(R(0), R(0)), tbv = mk<C>(R(0), R(0));
        if constexpr (OP != 1) {
          const RVec<R> rA = rot_vec(tb, kz, myky, 0);
          const RVec<R> rB = rot_vec(tb, kz, myky, M);
          for (int l = 0; l < 3; ++l) {
            const C P = spec[(l * 2 + col) * L + kz];
            const C Pm = spec[(l * 2 + (1 - col)) * L + kzm];
            const C A = cscale(cadd(P, cconj(Pm)), R(0.5));
            const C Bv = cscale(mul_mi(csub(P, cconj(Pm))), R(0.5));
            const R ra = rget(rA, l), rb = rget(rB, l);
            ta = mk<C>(ta.x + A.x * ra, ta.y + A.y * ra);
            tbv = mk<C>(tbv.x + Bv.x * rb, tbv.y + Bv.y * rb);
          }
          const R a2 = rA.x * rA.x + rA.y * rA.y + rA.z * rA.z;
          const R b2 = rB.x * rB.x + rB.y * rB.y + rB.z * rB.z;
          ta = cscale(ta, a2 > R(0) ? scale / a2 : R(0));
          tbv = cscale(tbv, b2 > R(0) ? scale / b2 : R(0));
        } else {
          const C P = spec[col * L + kz];
          const C Pm = spec[(1 - col) * L + kzm];
          const C A = cscale(cadd(P, cconj(Pm)), R(0.5));
          const C Bv = cscale(mul_mi(csub(P, cconj(Pm))), R(0.5));
          const double dA = a0 + a1 * (double)lap_sym(tb, kz, myky, 0);
          const double dB = a0 + a1 * (double)lap_sym(tb, kz, myky, M);
          ta = cscale(A, (R)((double)scale / dA));
          tbv = cscale(Bv, (R)((double)scale / dB));
        }
        if constexpr (OP == 2) {
          // potential U = -i e^{i Phi} w: at qx = 0, U_A = -i e^{i Phi_A} tA;
          // at qx = pi, e^{i Phi_B} = i e^{i Phi_A}, so U_B = e^{i Phi_A} tB;
          // packed as U_A + i U_B
          const C ph = cmul(mk<C>(tb.cz[kz], tb.snz[kz]), mk<C>(tb.cy[myky], tb.sny[myky]));  // e^{i Phi_A}
          v1[e] = cadd(mul_mi(cmul(ta, ph)), mul_pi(cmul(tbv, ph)));
        } else if constexpr (OP == 1) {
          v1[e] = cadd(ta, mul_pi(tbv));
        } else {
          tA[e] = ta;
          tB[e] = tbv;
        }
      }
    }
    {
      // OP 0: wave j writes output j; OP 1, 2: every wave forms the one
      // output (in its own exchange buffer), wave 0 stores it
      const int j = (NOUT == 1) ? 0 : grp;
      C v[LS::E];
#pragma unroll
      for (int e = 0; e < LS::E; ++e) {
        if constexpr (OP == 0) {
          const int kz = LS::idxB(t, e);
          const C a = cscale(tA[e], rget(rot_vec(tb, kz, myky, 0), j));
          const C b = cscale(tB[e], rget(rot_vec(tb, kz, myky, M), j));
          v[e] = cadd(a, mul_pi(b));  // A' + i B'
        } else {
          v[e] = v1[e];
        }
      }
      if constexpr (LS::R2 == 1) {
        Dft<LS::R1, 1, true, C>::run(v);
      } else {
#pragma unroll
        for (int w = 0; w < LS::V; ++w) {
          const int k1 = t + LS::T * w;
          Dft<LS::R2, 1, true, C>::run(v + w * LS::R2);
#pragma unroll
          for (int n2 = 1; n2 < LS::R2; ++n2)
            if (lane_ok) v[w * LS::R2 + n2] = twiddle_tab<true>(v[w * LS::R2 + n2], tb.tw0, (n2 * k1) % L);
          if (lane_ok)
#pragma unroll
            for (int n2 = 0; n2 < LS::R2; ++n2) xbuf[(n2 * LS::R1 + k1) * 2 + col] = v[w * LS::R2 + n2];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < LS::U; ++u) {
          const int n2 = t + LS::T * u;
          if (lane_ok)
#pragma unroll
            for (int k1 = 0; k1 < LS::R1; ++k1) v[u * LS::R1 + k1] = xbuf[(n2 * LS::R1 + k1) * 2 + col];
          Dft<LS::R1, 1, true, C>::run(v + u * LS::R1);
        }
        __syncthreads();
      }
      if (store && (NOUT > 1 || grp == 0))
#pragma unroll
        for (int e = 0; e < LS::E; ++e) base[(cout + j) * comp + LS::idxA(t, e) * plane] = v[e];
    }
  }
}

template <typename R, int L, int OP>
__global__ void __launch_bounds__(64 * z_dc_groups<OP>())
k_fft_z_dc(R* data, int N1, int M, SpecTables<R> tb, R scale, double a0, double a1, Skip skip, const R* dcb) {
  __shared__ cplx<R> lds[z_dc_lds<L, OP>()];
  if (skip(blockIdx.y)) return;
  z_dc_body<R, L, OP>(data, N1, M, tb, scale, a0, a1, (int)blockIdx.x, (int)blockIdx.y, lds,
                      lds + z_dc_groups<OP>() * 2 * L, reinterpret_cast<const cplx<R>*>(dcb));
}

}  // namespace fg
