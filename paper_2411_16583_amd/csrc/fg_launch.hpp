// Host-side launchers of the FFT passes (size dispatch).  Defined once per
// working precision in fg_fft_f64.hip / fg_fft_f32.hip.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fg_fft.hpp"

namespace fg {

// Launch that takes a timing event pair itself when one is given (the
// kernel's own start and end, no marker packets on the stream): ev0 is
// recorded at the start of this kernel, ev1 at its end; either may be null.
template <typename F, typename... A>
inline void launch_ev(F kernel, dim3 grid, dim3 block, unsigned shm, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1,
                      A... args) {
  if (ev0 || ev1)
    hipExtLaunchKernelGGL(kernel, grid, block, shm, s, ev0, ev1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
}

bool fft_length_supported(int L);       // complex line lengths
bool fft_axis_length_supported(int L);  // N1 (and N0 > 1)
bool fft_n0_length_supported(int L);    // N0: the axis lengths and 1 (a plane)
bool fft_n1_length_supported(int L);    // N1: the axis lengths and 512

// Largest power-of-two column tile dividing M with T * B <= 256 threads and
// an exchange buffer of L * B complex values within 64 KiB.
int column_tile(int L, int M, int elem_bytes);
int column_tile_t(int T, int L, int M, int elem_bytes);
// largest tile for cpt columns per thread: T tile / cpt <= 256 threads
int column_tile_cpt(int L, int M, int elem_bytes, int cpt);
int line_threads(int L);
int zline_threads(int L);  // threads per line of the fused N0 projection pass
// threads per line and columns per thread of the potential-form N0 pass
// (elem_bytes: bytes of one complex value of the working precision)
int zgrad_threads(int L, int elem_bytes);
int zgrad_cpt(int L, int elem_bytes);
int zgrad_tile(int L, int M, int elem_bytes);  // built-in tile of launch_zgrad

// Fused CG front on the potentials (deferred xi update, direction update,
// p = D pi, contraction, p.Kp, N2 real-to-complex pass); h: grid spacings;
// law: kLawNH or kLawSVK (the tangent state's layout); returns the
// number of partials written.
template <typename R>
int launch_cg_front(int M, R* spec, R* pbuf, R* xbuf, const R* rbuf, const R* st, const KrylovScalars* ks,
                    double* partials, long N, int n0, int n1, const double h[3], const SpecTables<R>& tb,
                    hipStream_t s, int nitems = 1, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                    int law = 0);

template <typename R>
void launch_r2c(int M, const R* in, R* out, long nlines, const SpecTables<R>& tb, const Skip& skip,
                hipStream_t s);
// returns the number of blocks (= partials written when epi.partials != nullptr)
template <typename R>
int launch_c2r(int M, const R* in, R* out, long nlines, const SpecTables<R>& tb, const C2REpi& epi,
               hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// tile: columns per workgroup (0: column_tile).
template <typename R>
void launch_axis(int L, bool inv, R* data, long estride, long ystride, long zstride, int M, int gy, int gz,
                 const cplx<R>* tw, const Skip& skip, hipStream_t s, int tile = 0, hipEvent_t ev0 = nullptr,
                 hipEvent_t ev1 = nullptr);
// Forward N1 pass of the potential-form projection for nitems 9-component
// fields: per row, the two terms sharing the N0 factor are merged (slots
// 3i, 3i + 1 written; kx = 0 column unmerged in all three slots).  tile as
// for launch_axis (a column-pair flag is ignored).  With pap_partials (in
// the CG), one workgroup per item also sets the item's step length from
// the front's nparts partial sums of p.Ap (k_finalize mode 0).  With dcb,
// the kx = 0 column of the three slots of every row is also written there,
// contiguous along N0 (complex [9 nitems][N1][N0]), for launch_zgrad.
template <typename R>
void launch_axis_rows(int N1, R* data, int N0, int M, const SpecTables<R>& tb, const Skip& skip, hipStream_t s,
                      int nitems = 1, int tile = 0, const double* pap_partials = nullptr, int nparts = 0,
                      KrylovScalars* ks = nullptr, R* dcb = nullptr, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);
// N0 pass fused with the projection, for nitems 9-component fields (3 rows
// each).
template <typename R>
void launch_zproj(int N0, R* data, int N1, int M, const SpecTables<R>& tb, R scale, const Skip& skip,
                  hipStream_t s, int nitems = 1, int tile = 0);
// N0 pass fused with the projection in the potential form, on the output of
// launch_axis_rows (the potential U_i written to slot 3i of each item), and
// its kx = 0 companion (reading the kx = 0 column from dcb when given: the
// buffer launch_axis_rows filled in the same pass).
template <typename R>
void launch_zgrad(int N0, R* data, int N1, int M, const SpecTables<R>& tb, R scale, const Skip& skip,
                  hipStream_t s, int nitems = 1, int tile = 0, const R* dcb = nullptr, hipEvent_t ev0 = nullptr,
                  hipEvent_t ev1 = nullptr);
// Flag on a projection-pass tile: workgroups ordered ky fastest.
constexpr int kTileKyMajor = 1 << 16;
// Flag on an N1-pass tile in single precision: two adjacent columns per
// thread (one 16-byte access; measured slower at 256^3, kept for the tuner).
constexpr int kTileColumnPairs = 1 << 17;
// Tile widths a pass accepts: powers of two dividing M with T tile <= 256
// threads and an L x tile exchange buffer (plus the pass's tables) within
// 64 KiB.  zproj: the fused N0 projection pass (L = N0), else the N1 pass.
bool tile_valid(bool zproj, int L, int M, int elem_bytes, int tile);
// N0 pass fused with a scalar symbol scale / (a0 + a1 lambda(q)), 1 component.
template <typename R>
void launch_zscalar(int N0, R* data, int N1, int M, const SpecTables<R>& tb, R scale, double a0, double a1,
                    const Skip& skip, hipStream_t s);

}  // namespace fg
