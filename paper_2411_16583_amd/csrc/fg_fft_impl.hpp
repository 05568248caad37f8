// Definitions of the FFT pass launchers (included by fg_fft_f64.hip and
// fg_fft_f32.hip, one working precision each).
#pragma once
#include <hip/hip_ext.h>
#include <algorithm>
#include <stdexcept>

#include "fg_cgfront.hpp"
#include "fg_fft3.hpp"
#include "fg_launch.hpp"

namespace fg {

#define FG_FOR_M(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(256)
#define FG_FOR_AXIS(X) X(1) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(256)
// N1 passes also take 512-long lines (plane grids of 512 x 512)
#define FG_FOR_N1(X) FG_FOR_AXIS(X) X(512)

template <typename R>
void launch_r2c(int M, const R* in, R* out, long nlines, const SpecTables<R>& tb, const Skip& skip,
                hipStream_t s) {
  switch (M) {
#define FG_CASE(L_)                                                                        \
  case L_: {                                                                               \
    constexpr int LPB = XBLOCK / Line<L_>::T;                                              \
    const long blocks = skip.line_blocks(nlines, LPB);                                     \
    hipLaunchKernelGGL((k_fft_x_r2c<R, L_>), dim3((unsigned)blocks), dim3(XBLOCK), 0, s, in, out, \
                       nlines, tb, skip);                                                  \
    return;                                                                                \
  }
    FG_FOR_M(FG_CASE)
#undef FG_CASE
  }
  throw std::invalid_argument("unsupported N2/2");
}

template <typename R>
int launch_c2r(int M, const R* in, R* out, long nlines, const SpecTables<R>& tb, const C2REpi& epi,
               hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  switch (M) {
#define FG_CASE(L_)                                                                        \
  case L_: {                                                                               \
    constexpr int LPB = XBLOCK / Line<L_>::T;                                              \
    const long blocks = epi.skip.line_blocks(nlines, LPB);                                 \
    launch_ev((k_fft_x_c2r<R, L_>), dim3((unsigned)blocks), dim3(XBLOCK), 0, s, ev0, ev1, in, out, \
              nlines, tb, epi);                                                            \
    return (int)blocks;                                                                    \
  }
    FG_FOR_M(FG_CASE)
#undef FG_CASE
  }
  throw std::invalid_argument("unsupported N2/2");
}

template <typename R>
void launch_axis(int L, bool inv, R* data, long estride, long ystride, long zstride, int M, int gy, int gz,
                 const cplx<R>* tw, const Skip& skip, hipStream_t s, int tile, hipEvent_t ev0, hipEvent_t ev1) {
  // single precision, on request: two columns per thread (16-byte accesses)
  int cpt = (sizeof(R) == 4 && (tile & kTileColumnPairs)) ? 2 : 1;
  tile &= ~kTileColumnPairs;
  const int T = line_threads(L);
  const int B = tile > 0 ? tile : column_tile_cpt(L, M, (int)sizeof(cplx<R>), cpt);
  if (B % cpt != 0) cpt = 1;
  // single precision reads the stage twiddles from LDS where they fit beside
  // the exchange buffer (the inverse N1 pass at 256^3: 94 -> 71 us); double
  // precision keeps them in the caches (its LDS is what bounds occupancy)
  const bool twl = sizeof(R) == 4 && (size_t)(L * B + L) * sizeof(cplx<R>) <= 65536;
  const size_t shm = (size_t)(L * B + (twl ? L : 0)) * sizeof(cplx<R>);
  dim3 grid((unsigned)(M / B), (unsigned)gy, (unsigned)gz);
  const dim3 block((unsigned)(T * B / cpt));
  constexpr int CP = (sizeof(R) == 4) ? 2 : 1;
  constexpr bool TW = sizeof(R) == 4;
  switch (L) {
#define FG_AXIS_GO(L_, INV_, CPT_)                                                                            \
  do {                                                                                                      \
    if (twl)                                                                                                \
      launch_ev((k_fft_axis<R, L_, INV_, CPT_, TW>), grid, block, shm, s, ev0, ev1, data, estride, ystride, \
                zstride, B, tw, skip);                                                                      \
    else                                                                                                    \
      launch_ev((k_fft_axis<R, L_, INV_, CPT_, false>), grid, block, shm, s, ev0, ev1, data, estride,       \
                ystride, zstride, B, tw, skip);                                                             \
  } while (0)
#define FG_CASE(L_)                 \
  case L_:                          \
    if (cpt == 2) {                 \
      if (inv)                      \
        FG_AXIS_GO(L_, true, CP);   \
      else                          \
        FG_AXIS_GO(L_, false, CP);  \
    } else {                        \
      if (inv)                      \
        FG_AXIS_GO(L_, true, 1);    \
      else                          \
        FG_AXIS_GO(L_, false, 1);   \
    }                               \
    return;
    FG_FOR_N1(FG_CASE)
#undef FG_CASE
#undef FG_AXIS_GO
  }
  throw std::invalid_argument("unsupported axis length");
}

template <typename R>
void launch_axis_rows(int N1, R* data, int N0, int M, const SpecTables<R>& tb, const Skip& skip, hipStream_t s,
                      int nitems, int tile, const double* pap_partials, int nparts, KrylovScalars* ks, R* dcb,
                      hipEvent_t ev0, hipEvent_t ev1) {
  tile &= ~kTileColumnPairs;
  const int T = zline_threads(N1);  // threads per line of RowLine<R, N1>
  // single precision: two adjacent columns per thread
  constexpr int CPT = (sizeof(R) == 4) ? 2 : 1;
  int B = tile > 0 ? tile : zgrad_tile(N1, M, (int)sizeof(cplx<R>));
  int cpt = (B % CPT == 0) ? CPT : 1;
  // the N1 tile is shared with launch_axis: halve it until the workgroup and
  // its LDS (exchange buffer + twiddles) fit
  while (B > 1 && (T * B / cpt > 256 || (size_t)N1 * (B + 1) * sizeof(cplx<R>) > 65536)) {
    B /= 2;
    cpt = (B % CPT == 0) ? CPT : 1;
  }
  const size_t shm = (size_t)N1 * (B + 1) * sizeof(cplx<R>);
  const long plane = (long)N1 * M;
  // planes y = i0, z = row (3 per item); components of a row n0 planes apart
  dim3 grid((unsigned)(M / B), (unsigned)N0, (unsigned)(3 * nitems));
  const Skip sk = skip.unit(3L * N0);
  switch (N1) {
#define FG_CASE(L_)                                                                                    \
  case L_:                                                                                             \
    if (cpt == 2)                                                                                      \
      launch_ev((k_fft_axis_rows<R, L_, CPT>), grid, dim3(T * B / 2), shm, s, ev0, ev1, data, (long)M, plane, \
                         3L * N0 * plane, (long)N0 * plane, B, tb, sk, pap_partials, nparts, ks, dcb); \
    else                                                                                               \
      launch_ev((k_fft_axis_rows<R, L_, 1>), grid, dim3(T * B), shm, s, ev0, ev1, data, (long)M, plane,  \
                         3L * N0 * plane, (long)N0 * plane, B, tb, sk, pap_partials, nparts, ks, dcb); \
    return;
    FG_FOR_N1(FG_CASE)
#undef FG_CASE
  }
  throw std::invalid_argument("unsupported axis length");
}

template <typename R>
void launch_zproj(int N0, R* data, int N1, int M, const SpecTables<R>& tb, R scale, const Skip& skip,
                  hipStream_t s, int nitems, int tile) {
  const int T = zline_threads(N0);
  // built-in choice (tile 0): the largest tile, workgroups ky fastest
  const int kymajor = (tile == 0 || (tile & kTileKyMajor)) ? 1 : 0;
  tile &= ~kTileKyMajor;
  int B = tile > 0 ? tile : column_tile_t(T, N0, M, (int)sizeof(cplx<R>));
  while (B > 1 && T * B > 256) B /= 2;  // a tile chosen for the column-pair N0 pass
  const size_t shm = (size_t)N0 * B * sizeof(cplx<R>) + zpass_extra_lds<R>(N0);
  dim3 grid = kymajor ? dim3((unsigned)N1, (unsigned)(M / B), (unsigned)(3 * nitems))
                      : dim3((unsigned)(M / B), (unsigned)N1, (unsigned)(3 * nitems));
  dim3 gdc((unsigned)(N1 / 2 + 1), (unsigned)(3 * nitems), 1);
  switch (N0) {
#define FG_CASE(L_)                                                                                    \
  case L_:                                                                                             \
    hipLaunchKernelGGL((k_fft_z_proj<R, L_>), grid, dim3(T * B), shm, s, data, N1, M, B, tb, scale, skip, \
                       kymajor);                                                                       \
    hipLaunchKernelGGL((k_fft_z_dc<R, L_, 0>), gdc, dim3(64 * z_dc_groups<0>()), 0, s, data, N1, M, tb, scale, \
                       0.0, 0.0, skip, (const R*)nullptr);                                            \
    return;
    FG_FOR_AXIS(FG_CASE)
#undef FG_CASE
  }
  throw std::invalid_argument("unsupported N0");
}

// The potential-form N0 pass with the kx = 0 pairs as its leading slice
// (N0 = 256 only; see launch_zgrad).
template <typename R, int L>
void launch_zgrad_fused(dim3 grid, dim3 block, size_t shm, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, R* data,
                        int N1, int M, int B, const SpecTables<R>& tb, R scale, const Skip& sk, int kymajor,
                        int dc_lead, const R* dcb) {
  if constexpr (L == 256) {
    launch_ev((k_fft_z_grad3<R, L, 1, true>), grid, block, shm, s, ev0, ev1, data, N1, M, B, tb, scale, sk, kymajor,
              dc_lead, dcb);
  } else {
    throw std::logic_error("the fused kx = 0 slice is built for N0 = 256 only");
  }
}

template <typename R>
void launch_zgrad(int N0, R* data, int N1, int M, const SpecTables<R>& tb, R scale, const Skip& skip,
                  hipStream_t s, int nitems, int tile, const R* dcb, hipEvent_t ev0, hipEvent_t ev1) {
  const int T = zgrad_threads(N0, (int)sizeof(cplx<R>));
  const int kymajor = (tile == 0 || (tile & kTileKyMajor)) ? 1 : 0;
  tile &= ~kTileKyMajor;
  // single precision: two adjacent columns per thread (one at N0 = 256)
  constexpr int CPT = (sizeof(R) == 4) ? 2 : 1;
  int B = tile > 0 ? tile : zgrad_tile(N0, M, (int)sizeof(cplx<R>));
  auto cpt_of = [&](int b) { return (b % 2 == 0) ? zgrad_cpt(N0, (int)sizeof(cplx<R>)) : 1; };
  while (B > 1 && T * B / cpt_of(B) > 256) B /= 2;  // a tile chosen for another line shape
  const int cpt = cpt_of(B);
  const size_t shm = (size_t)N0 * B * sizeof(cplx<R>) + zgrad_extra_lds<R>(N0);
  dim3 grid = kymajor ? dim3((unsigned)N1, (unsigned)(M / B), (unsigned)(3 * nitems))
                      : dim3((unsigned)(M / B), (unsigned)N1, (unsigned)(3 * nitems));
  dim3 gdc((unsigned)(N1 / 2 + 1), (unsigned)(3 * nitems), 1);
  const Skip sk = skip.unit(3);  // grid.z (grad) and grid.y (kx = 0): 3 rows per item
  // N0 = 256 with one column per thread: the kx = 0 pairs run as a leading
  // slice of the same launch when they fit in it, so that they overlap the
  // rest instead of following it (measured at 256^3, the pass with its
  // kx = 0 work: single precision 152 -> 143 us); the workgroups then take
  // the larger of the two LDS sizes (in double precision 48 KiB: 3 per CU,
  // as many as the registers allow anyway)
  const int dc_lead = (N1 / 2 + 1) * 3 * nitems;
  const size_t shm_dc = std::max(shm, (size_t)z_dc_lds<256, 2>() * sizeof(cplx<R>));
  const bool fuse_dc = N0 == 256 && cpt == 1 && T * B >= 64 * z_dc_groups<2>() &&
                       (long)dc_lead <= (long)grid.x * grid.y && shm_dc <= 65536;
  switch (N0) {
#define FG_CASE(L_)                                                                                    \
  case L_:                                                                                             \
    if (fuse_dc) {                                                                                     \
      launch_zgrad_fused<R, L_>(dim3(grid.x, grid.y, grid.z + 1), dim3(T * B), shm_dc, s, ev0, ev1, data, N1, M, B, \
                                tb, scale, sk, kymajor, dc_lead, dcb);                                 \
      return;                                                                                          \
    }                                                                                                  \
    if (cpt == 2)                                                                                      \
      launch_ev((k_fft_z_grad3<R, L_, CPT>), grid, dim3(T * B / 2), shm, s, ev0, nullptr, data, N1, M, B, tb, scale, \
                         sk, kymajor, 0, nullptr);                                                     \
    else                                                                                               \
      launch_ev((k_fft_z_grad3<R, L_, 1>), grid, dim3(T * B), shm, s, ev0, nullptr, data, N1, M, B, tb, scale, sk, \
                         kymajor, 0, nullptr);                                                         \
    launch_ev((k_fft_z_dc<R, L_, 2>), gdc, dim3(64 * z_dc_groups<2>()), 0, s, nullptr, ev1, data, N1, M, tb,   \
              scale, 0.0, 0.0, sk, dcb);                                                              \
    return;
    FG_FOR_AXIS(FG_CASE)
#undef FG_CASE
  }
  throw std::invalid_argument("unsupported N0");
}

template <typename R>
void launch_zscalar(int N0, R* data, int N1, int M, const SpecTables<R>& tb, R scale, double a0, double a1,
                    const Skip& skip, hipStream_t s) {
  const int B = column_tile(N0, M, (int)sizeof(cplx<R>));
  const int T = line_threads(N0);
  const size_t shm = (size_t)N0 * B * sizeof(cplx<R>) + zpass_extra_lds<R>(N0);
  dim3 grid((unsigned)(M / B), (unsigned)N1, 1);
  dim3 gdc((unsigned)(N1 / 2 + 1), 1, 1);
  switch (N0) {
#define FG_CASE(L_)                                                                                   \
  case L_:                                                                                            \
    hipLaunchKernelGGL((k_fft_z_scalar<R, L_>), grid, dim3(T * B), shm, s, data, N1, M, B, tb, scale, a0, \
                       a1, skip);                                                                     \
    hipLaunchKernelGGL((k_fft_z_dc<R, L_, 1>), gdc, dim3(64 * z_dc_groups<1>()), 0, s, data, N1, M, tb, scale, \
                       a0, a1, skip, (const R*)nullptr);                                              \
    return;
    FG_FOR_AXIS(FG_CASE)
#undef FG_CASE
  }
  throw std::invalid_argument("unsupported N0");
}

template <typename R>
int launch_cg_front(int M, R* spec, R* pbuf, R* xbuf, const R* rbuf, const R* st, const KrylovScalars* ks,
                    double* partials, long N, int n0, int n1, const double h[3], const SpecTables<R>& tb,
                    hipStream_t s, int nitems, hipEvent_t ev0, hipEvent_t ev1, int law) {
  const R q0 = (R)(0.25 / h[0]), q1 = (R)(0.25 / h[1]), q2 = (R)(0.25 / h[2]);
  const long nlines = (long)n0 * n1;
  switch (M) {
#define FG_CASE(L_)                                                                                   \
  case L_: {                                                                                          \
    using FS = FrontShape<L_>;                                                                        \
    const long blocks = nitems * ((nlines + FS::LB - 1) / FS::LB);                                    \
    if (law == kLawSVK)                                                                            \
      launch_ev((k_cg_front<R, L_, kLawSVK>), dim3((unsigned)blocks), dim3(FS::THREADS), 0, s, ev0, ev1, spec, \
                pbuf, xbuf, rbuf, st, ks, partials, N, n0, n1, tb, q0, q1, q2);                         \
    else                                                                                              \
      launch_ev((k_cg_front<R, L_, kLawNH>), dim3((unsigned)blocks), dim3(FS::THREADS), 0, s, ev0, ev1, spec, \
                pbuf, xbuf, rbuf, st, ks, partials, N, n0, n1, tb, q0, q1, q2);                         \
    return (int)blocks;                                                                               \
  }
    FG_FOR_M(FG_CASE)
#undef FG_CASE
  }
  throw std::invalid_argument("unsupported N2/2");
}

#define FG_INSTANTIATE_LAUNCHERS(R)                                                                     \
  template int launch_cg_front<R>(int, R*, R*, R*, const R*, const R*, const KrylovScalars*, double*, long, int, \
                                  int, const double*, const SpecTables<R>&, hipStream_t, int, hipEvent_t,   \
                                  hipEvent_t, int);                                                     \
  template void launch_r2c<R>(int, const R*, R*, long, const SpecTables<R>&, const Skip&, hipStream_t); \
  template int launch_c2r<R>(int, const R*, R*, long, const SpecTables<R>&, const C2REpi&, hipStream_t, hipEvent_t, \
                             hipEvent_t);                                                           \
  template void launch_axis<R>(int, bool, R*, long, long, long, int, int, int, const cplx<R>*, const Skip&, \
                               hipStream_t, int, hipEvent_t, hipEvent_t);                               \
  template void launch_axis_rows<R>(int, R*, int, int, const SpecTables<R>&, const Skip&, hipStream_t, int, int,    \
                                    const double*, int, KrylovScalars*, R*, hipEvent_t, hipEvent_t);            \
  template void launch_zproj<R>(int, R*, int, int, const SpecTables<R>&, R, const Skip&, hipStream_t, int, int); \
  template void launch_zgrad<R>(int, R*, int, int, const SpecTables<R>&, R, const Skip&, hipStream_t, int, int, \
                                const R*, hipEvent_t, hipEvent_t);                                       \
  template void launch_zscalar<R>(int, R*, int, int, const SpecTables<R>&, R, double, double, const Skip&, \
                                  hipStream_t);

}  // namespace fg
