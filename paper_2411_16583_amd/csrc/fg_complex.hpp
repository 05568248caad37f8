// Complex arithmetic on HIP vector types and compile-time small DFTs.
//
// A complex value is a double2 / float2 (x = real, y = imaginary), so that
// one element is one 16-byte (8-byte) load or store.  The small DFT
// "codelets" are fully unrolled in registers: radix 2, 3 and 4 are written
// out, composite sizes (6, 8, 12, 16) are Cooley-Tukey splits R = P * Q
// with compile-time twiddles.  Sign convention: forward uses e^{-2 pi i nk/R},
// the inverse e^{+2 pi i nk/R}; neither is normalised.
#pragma once
#include <hip/hip_runtime.h>

namespace fg {

template <typename T> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };
template <typename T> using cplx = typename vec2<T>::type;

template <typename C> __device__ __forceinline__ C mk(decltype(C::x) a, decltype(C::x) b) {
  C r; r.x = a; r.y = b; return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return mk<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return mk<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }
// Streaming store of one complex value (nontemporal: the line is not kept
// in the caches for reuse; for write streams that are read back only by a
// later kernel).
template <typename C> __device__ __forceinline__ void st_stream(C* p, C v) {
  using T = decltype(C::x);
  typedef T nv2 __attribute__((ext_vector_type(2)));
  nv2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<nv2*>(p));
}
// Streaming load of one complex value (nontemporal: for read streams that
// are used once).
template <typename C> __device__ __forceinline__ C ld_stream(const C* p) {
  using T = decltype(C::x);
  typedef T nv2 __attribute__((ext_vector_type(2)));
  const nv2 w = __builtin_nontemporal_load(reinterpret_cast<const nv2*>(p));
  return mk<C>(w[0], w[1]);
}
// The same for 16 bytes of single-precision values (two complex numbers).
__device__ __forceinline__ float4 ld_stream_f4(const void* p) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 w = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
  return make_float4(w[0], w[1], w[2], w[3]);
}
__device__ __forceinline__ void st_stream_f4(void* p, float4 v) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<f4*>(p));
}
// multiply by -i (forward quarter turn) / +i
template <typename C> __device__ __forceinline__ C mul_mi(C a) { return mk<C>(a.y, -a.x); }
template <typename C> __device__ __forceinline__ C mul_pi(C a) { return mk<C>(-a.y, a.x); }

// cos(2 pi k / 96) and sin(2 pi k / 96), k = 0..95, correctly rounded.
// Every twiddle of the radix-2/3/4/6/8/12/16/24/32/48 codelets is one of these.
constexpr double kCos96[96] = {1.0, 0.9978589232386035, 0.9914448613738104, 0.9807852804032304, 0.9659258262890683, 0.9469301294951057, 0.9238795325112867, 0.8968727415326883, 0.8660254037844386, 0.8314696123025452, 0.7933533402912352, 0.7518398074789774, 0.7071067811865476, 0.6593458151000688, 0.6087614290087207, 0.5555702330196022, 0.5, 0.4422886902190013, 0.3826834323650898, 0.3214394653031616, 0.25881904510252074, 0.19509032201612828, 0.1305261922200516, 0.06540312923014306, 0.0, -0.06540312923014306, -0.1305261922200516, -0.19509032201612828, -0.25881904510252074, -0.3214394653031616, -0.3826834323650898, -0.4422886902190013, -0.5, -0.5555702330196022, -0.6087614290087207, -0.6593458151000688, -0.7071067811865476, -0.7518398074789774, -0.7933533402912352, -0.8314696123025452, -0.8660254037844386, -0.8968727415326883, -0.9238795325112867, -0.9469301294951057, -0.9659258262890683, -0.9807852804032304, -0.9914448613738104, -0.9978589232386035, -1.0, -0.9978589232386035, -0.9914448613738104, -0.9807852804032304, -0.9659258262890683, -0.9469301294951057, -0.9238795325112867, -0.8968727415326883, -0.8660254037844386, -0.8314696123025452, -0.7933533402912352, -0.7518398074789774, -0.7071067811865476, -0.6593458151000688, -0.6087614290087207, -0.5555702330196022, -0.5, -0.4422886902190013, -0.3826834323650898, -0.3214394653031616, -0.25881904510252074, -0.19509032201612828, -0.1305261922200516, -0.06540312923014306, 0.0, 0.06540312923014306, 0.1305261922200516, 0.19509032201612828, 0.25881904510252074, 0.3214394653031616, 0.3826834323650898, 0.4422886902190013, 0.5, 0.5555702330196022, 0.6087614290087207, 0.6593458151000688, 0.7071067811865476, 0.7518398074789774, 0.7933533402912352, 0.8314696123025452, 0.8660254037844386, 0.8968727415326883, 0.9238795325112867, 0.9469301294951057, 0.9659258262890683, 0.9807852804032304, 0.9914448613738104, 0.9978589232386035};
constexpr double kSin96[96] = {0.0, 0.06540312923014306, 0.1305261922200516, 0.19509032201612828, 0.25881904510252074, 0.3214394653031616, 0.3826834323650898, 0.4422886902190013, 0.5, 0.5555702330196022, 0.6087614290087207, 0.6593458151000688, 0.7071067811865476, 0.7518398074789774, 0.7933533402912352, 0.8314696123025452, 0.8660254037844386, 0.8968727415326883, 0.9238795325112867, 0.9469301294951057, 0.9659258262890683, 0.9807852804032304, 0.9914448613738104, 0.9978589232386035, 1.0, 0.9978589232386035, 0.9914448613738104, 0.9807852804032304, 0.9659258262890683, 0.9469301294951057, 0.9238795325112867, 0.8968727415326883, 0.8660254037844386, 0.8314696123025452, 0.7933533402912352, 0.7518398074789774, 0.7071067811865476, 0.6593458151000688, 0.6087614290087207, 0.5555702330196022, 0.5, 0.4422886902190013, 0.3826834323650898, 0.3214394653031616, 0.25881904510252074, 0.19509032201612828, 0.1305261922200516, 0.06540312923014306, 0.0, -0.06540312923014306, -0.1305261922200516, -0.19509032201612828, -0.25881904510252074, -0.3214394653031616, -0.3826834323650898, -0.4422886902190013, -0.5, -0.5555702330196022, -0.6087614290087207, -0.6593458151000688, -0.7071067811865476, -0.7518398074789774, -0.7933533402912352, -0.8314696123025452, -0.8660254037844386, -0.8968727415326883, -0.9238795325112867, -0.9469301294951057, -0.9659258262890683, -0.9807852804032304, -0.9914448613738104, -0.9978589232386035, -1.0, -0.9978589232386035, -0.9914448613738104, -0.9807852804032304, -0.9659258262890683, -0.9469301294951057, -0.9238795325112867, -0.8968727415326883, -0.8660254037844386, -0.8314696123025452, -0.7933533402912352, -0.7518398074789774, -0.7071067811865476, -0.6593458151000688, -0.6087614290087207, -0.5555702330196022, -0.5, -0.4422886902190013, -0.3826834323650898, -0.3214394653031616, -0.25881904510252074, -0.19509032201612828, -0.1305261922200516, -0.06540312923014306};

// Multiply by W_R^j = e^{-+ 2 pi i j / R} with j a compile-time constant
// (after unrolling); the quarter turns are exact.
template <int R, bool INV, typename C>
__device__ __forceinline__ C twiddle_const(C a, int j) {
  using T = decltype(C::x);
  j %= R;
  if (j == 0) return a;
  if (4 * j == R) return INV ? mul_pi(a) : mul_mi(a);
  if (2 * j == R) return mk<C>(-a.x, -a.y);
  if (4 * j == 3 * R) return INV ? mul_mi(a) : mul_pi(a);
  static_assert(96 % R == 0, "constant twiddles for radices dividing 96");
  const int k = j * (96 / R);
  const T c = (T)kCos96[k];
  const T s = INV ? (T)kSin96[k] : -(T)kSin96[k];
  return cmul(a, mk<C>(c, s));
}

// In-place DFT of length R on a[0], a[S], ..., a[(R-1) S] (natural order).
template <int R, int S, bool INV, typename C> struct Dft;

template <int S, bool INV, typename C> struct Dft<1, S, INV, C> {
  __device__ __forceinline__ static void run(C*) {}
};

template <int S, bool INV, typename C> struct Dft<2, S, INV, C> {
  __device__ __forceinline__ static void run(C* a) {
    C t = a[0];
    a[0] = cadd(t, a[S]);
    a[S] = csub(t, a[S]);
  }
};

template <int S, bool INV, typename C> struct Dft<3, S, INV, C> {
  __device__ __forceinline__ static void run(C* a) {
    using T = decltype(C::x);
    const T h = (T)0.8660254037844386;  // sin(2 pi / 3)
    C s = cadd(a[S], a[2 * S]);
    C d = csub(a[S], a[2 * S]);
    C m = mk<C>(a[0].x - (T)0.5 * s.x, a[0].y - (T)0.5 * s.y);
    C rd = cscale(d, h);
    a[0] = cadd(a[0], s);
    // forward: y1 = m - i h d, y2 = m + i h d
    C q = INV ? mul_pi(rd) : mul_mi(rd);
    a[S] = cadd(m, q);
    a[2 * S] = csub(m, q);
  }
};

template <int S, bool INV, typename C> struct Dft<4, S, INV, C> {
  __device__ __forceinline__ static void run(C* a) {
    C t0 = cadd(a[0], a[2 * S]);
    C t1 = csub(a[0], a[2 * S]);
    C t2 = cadd(a[S], a[3 * S]);
    C t3 = csub(a[S], a[3 * S]);
    C r3 = INV ? mul_pi(t3) : mul_mi(t3);
    a[0] = cadd(t0, t2);
    a[2 * S] = csub(t0, t2);
    a[S] = cadd(t1, r3);
    a[3 * S] = csub(t1, r3);
  }
};

template <int R> struct FirstFactor {
  static constexpr int P = (R % 4 == 0) ? 4 : ((R % 3 == 0) ? 3 : 2);
};

// Composite R = P * Q:
//   X[k1 + P k2] = sum_{n2<Q} W_Q^{n2 k2} W_R^{n2 k1} sum_{n1<P} x[n2 + Q n1] W_P^{n1 k1}
template <int R, int S, bool INV, typename C> struct Dft {
  static constexpr int P = FirstFactor<R>::P;
  static constexpr int Q = R / P;
  __device__ __forceinline__ static void run(C* a) {
#pragma unroll
    for (int n2 = 0; n2 < Q; ++n2) Dft<P, Q * S, INV, C>::run(a + n2 * S);
#pragma unroll
    for (int n2 = 1; n2 < Q; ++n2)
#pragma unroll
      for (int k1 = 1; k1 < P; ++k1) a[(n2 + Q * k1) * S] = twiddle_const<R, INV>(a[(n2 + Q * k1) * S], n2 * k1);
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) Dft<Q, S, INV, C>::run(a + Q * k1 * S);
    // a[(Q k1 + k2) S] holds X[k1 + P k2]; permute to natural order
    C t[R];
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < Q; ++k2) t[k1 + P * k2] = a[(Q * k1 + k2) * S];
#pragma unroll
    for (int k = 0; k < R; ++k) a[k * S] = t[k];
  }
};

// Element at a 32-bit byte offset from a base pointer (a workgroup-uniform
// base plus one 32-bit register per access).
template <typename T> __device__ __forceinline__ T& at_bytes(T* base, unsigned byte_off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}
template <typename T> __device__ __forceinline__ const T& at_bytes(const T* base, unsigned byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

}  // namespace fg
