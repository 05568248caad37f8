// Plan, workspace, tables and the solver drivers behind the C ABI of
// include/fgfft.h.  All device work is issued on the plan's stream; the
// only host synchronisations are the scalar read-backs of convergence tests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fgfft.h"
#include "fg_launch.hpp"
#include "fg_pointwise.hpp"
#include "fg_scalar.hpp"
#include "fg_cgfront.hpp"
#include "fg_fft3.hpp"
#include "fg_batch.hpp"
#include "fg_cggrad.hpp"

using namespace fg;

namespace fg {

bool fft_length_supported(int L) {
  switch (L) {
    case 2: case 3: case 4: case 6: case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96:
    case 128: case 256:
      return true;
  }
  return false;
}
bool fft_axis_length_supported(int L) { return L >= 4 && fft_length_supported(L); }
// N0 may also be 1: a single plane (2-D problem), where the N0 transform is
// the identity and every difference along axis 0 vanishes
bool fft_n0_length_supported(int L) { return L == 1 || fft_axis_length_supported(L); }
// N1 may also be 512 (the N1 passes have 512-long lines; N0 stays <= 256)
bool fft_n1_length_supported(int L) { return L == 512 || fft_axis_length_supported(L); }

int line_threads(int L) {
  switch (L) {
    case 16: return Line<16>::T;
    case 24: return Line<24>::T;
    case 32: return Line<32>::T;
    case 48: return Line<48>::T;
    case 64: return Line<64>::T;
    case 96: return Line<96>::T;
    case 128: return Line<128>::T;
    case 256: return Line<256>::T;
    case 512: return Line<512>::T;
    default: return 1;
  }
}

int column_tile_t(int T, int L, int M, int elem_bytes) {
  int B = 1;
  while ((M % (2 * B)) == 0 && T * 2 * B <= 256 && (long)L * 2 * B * elem_bytes <= 65536) B *= 2;
  return B;
}

int column_tile(int L, int M, int elem_bytes) { return column_tile_t(line_threads(L), L, M, elem_bytes); }

int column_tile_cpt(int L, int M, int elem_bytes, int cpt) {
  const int T = line_threads(L);
  if (cpt <= 1 || M % cpt != 0) return column_tile_t(T, L, M, elem_bytes);
  int B = cpt;
  while ((M % (2 * B)) == 0 && T * 2 * B / cpt <= 256 && (long)L * 2 * B * elem_bytes <= 65536) B *= 2;
  return B;
}

// Built-in tile of the potential-form N0 pass: the largest power of two
// dividing M whose workgroup (two columns per thread in single precision)
// and LDS fit.
int zgrad_tile(int L, int M, int elem_bytes) {
  const int T = zgrad_threads(L, elem_bytes);
  const int cpt = zgrad_cpt(L, elem_bytes);
  int B = 1;
  while (M % (2 * B) == 0 && T * 2 * B / cpt <= 256 && (long)L * 2 * B * elem_bytes + 2L * L * elem_bytes <= 65536)
    B *= 2;
  return B;
}

// The potential-form N0 pass in single precision at L = 256 uses the
// two-stage 16 x 16 line with one column per thread (one LDS exchange per
// transform instead of two; the pass with its kx = 0 kernel 162 -> 154 us at
// 256^3);
// elsewhere the line of zline_threads, two columns per thread in single
// precision.
int zgrad_threads(int L, int elem_bytes) { return (elem_bytes == 8 && L == 256) ? Line<256>::T : zline_threads(L); }
int zgrad_cpt(int L, int elem_bytes) { return (elem_bytes == 8 && L != 256) ? 2 : 1; }

int zline_threads(int L) {
  if (L == 256) return Line3<256>::T;
  if (L == 128) return Line3<128>::T;
  if (L == 96) return Line3<96>::T;
  if (L == 512) return Line3<512>::T;
  return line_threads(L);
}

static_assert(kTileKyMajor == FG_TILE_KY_MAJOR, "public tile flag");
static_assert(kTileColumnPairs == FG_TILE_COLUMN_PAIRS, "public tile flag");

bool tile_valid(bool zproj, int L, int M, int elem_bytes, int tile) {
  bool pairs = false;
  if (zproj && (tile & kTileKyMajor)) tile &= ~kTileKyMajor;
  if (!zproj && elem_bytes == 8 && (tile & kTileColumnPairs)) {
    tile &= ~kTileColumnPairs;
    pairs = true;
  }
  if (tile < 1 || (tile & (tile - 1)) != 0 || M % tile != 0) return false;
  const int T = zproj ? zgrad_threads(L, elem_bytes) : line_threads(L);
  // single-precision N1 pass with column pairs: tile / 2 column groups
  if (pairs && tile % 2 != 0) return false;
  // the single-precision N0 pass takes two columns per thread (even tiles)
  // except at L = 256 (zgrad_cpt)
  const int cpt = pairs ? 2 : ((zproj && tile % 2 == 0) ? zgrad_cpt(L, elem_bytes) : 1);
  if (T * tile / cpt > 256) return false;
  // exchange buffer, plus the stage twiddles and the two kz tables of the
  // projection pass
  const long lds = (long)L * tile * elem_bytes + (zproj ? 2L * L * elem_bytes : 0L);
  return lds <= 65536;
}

}  // namespace fg

namespace {

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define FG_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) throw HipError(std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Status : std::runtime_error {
  fg_status code;
  Status(fg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

template <typename R> struct TablesDev {
  cplx<R>* tw0;
  cplx<R>* tw1;
  cplx<R>* twM;
  cplx<R>* post;
  R *cz, *sz, *cy, *sy, *cx, *sx;
  R *snz, *sny, *snx;
  SpecTables<R> spec() const {
    return SpecTables<R>{tw0, tw1, twM, post, cz, sz, cy, sy, cx, sx, snz, sny, snx};
  }
};

}  // namespace

struct fg_plan {
  int n0, n1, n2, M;
  long N;          // voxels per item
  int nitems = 1;  // batch items (independent solves on the same grid)
  bool batch_group = false;  // owned by a batch: only the tile calls are public
  // tile widths (columns per workgroup), 0 = heuristic:
  // [0] N1 pass FP64, [1] N0 projection pass FP64, [2] N1 pass FP32, [3] N0 projection pass FP32
  int tiles[4] = {0, 0, 0, 0};
  int tiles_gen = 0;  // bumped by fg_plan_set_tiles (a captured batch graph is then stale)
  int law = ::FG_LAW_NEO_HOOKE;  // material law (fg_set_law, before the workspace)
  double h[3];
  fg_precision prec;
  hipStream_t stream;
  std::string err;

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t need = 0;
  // carved regions (offsets into ws)
  TablesDev<double> t64{};
  TablesDev<float> t32{};
  KrylovScalars* ks = nullptr;   // [0, nitems) mechanics CG per item
  KrylovScalars* ksc = nullptr;  // scalar PCG (= ks + nitems)
  int* flags = nullptr;          // [0] domain
  double* dscal = nullptr;       // small FP64 scalars (norms), 64 + 16 nitems entries
  double* part = nullptr;        // partial sums
  double* part2 = nullptr;
  double* Fu = nullptr;          // uniform tensor (9)
  double* S64 = nullptr;         // 9N doubles: stress / FP64 spectra
  void* S = nullptr;             // 9N T (aliases S64 in FP64 plans)
  void* x = nullptr;             // 9N T
  void* r = nullptr;             // 9N T
  void* p = nullptr;             // 9N T
  void* st = nullptr;            // tangent state, state_words(law) N T
  void* dcb = nullptr;           // kx = 0 column of the row slots, contiguous along N0 (9 n0 n1 complex per item)
  double* sc = nullptr;          // scalar solver area, 16N doubles
  size_t part_n = 0;

  // material (caller-owned)
  const double *E = nullptr, *nu = nullptr, *Om = nullptr, *D = nullptr, *smax = nullptr;
  double gc = 0, lc = 0, RT = 0, cmax = 1;
  bool have_material = false;
  // state (caller-owned)
  double *F = nullptr, *c = nullptr, *d = nullptr, *H = nullptr;
  double* zeroN = nullptr;  // N zeros (c, d when not given) inside the scalar area
  // a linear system of one Newton correction begun by fg_newton_linear_begin
  // and open for fg_cg_iterate (cleared by every call that reuses the CG
  // workspace)
  bool lin_open = false;

  // optional per-kernel-class timing with HIP events (fg_profile_*)
  bool prof_on = false;
  unsigned prof_mask = ~0u;  // kernel classes timed while prof_on (bit = FG_PASS_*)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[FG_NPASS];
  size_t prof_used[FG_NPASS] = {};
  long prof_noop[FG_NPASS] = {};

  // pinned host scalars
  KrylovScalars* hks = nullptr;  // nitems + 1 entries
  KrylovScalars* hksc = nullptr;
  double* hd = nullptr;
  int* hflags = nullptr;
};

namespace {

template <typename T> T* carve(char* base, size_t& off, size_t count) {
  T* ptr = reinterpret_cast<T*>(base + off);
  off = align_up(off + count * sizeof(T));
  return ptr;
}

size_t layout(fg_plan* P, char* base) {
  const long N = P->N;
  const long NT = P->N * P->nitems;
  const int n0 = P->n0, n1 = P->n1, M = P->M;
  size_t off = 0;
  auto tabs = [&](auto& t, auto tag) {
    using R = decltype(tag);
    t.tw0 = carve<cplx<R>>(base, off, n0);
    t.tw1 = carve<cplx<R>>(base, off, n1);
    t.twM = carve<cplx<R>>(base, off, M);
    t.post = carve<cplx<R>>(base, off, M);
    t.cz = carve<R>(base, off, n0);
    t.sz = carve<R>(base, off, n0);
    t.cy = carve<R>(base, off, n1);
    t.sy = carve<R>(base, off, n1);
    t.cx = carve<R>(base, off, M + 1);
    t.sx = carve<R>(base, off, M + 1);
    t.snz = carve<R>(base, off, n0);
    t.sny = carve<R>(base, off, n1);
    t.snx = carve<R>(base, off, M + 1);
  };
  tabs(P->t64, double());
  tabs(P->t32, float());
  P->ks = carve<KrylovScalars>(base, off, P->nitems + 1);
  P->ksc = P->ks + P->nitems;
  P->flags = carve<int>(base, off, 4);
  P->dscal = carve<double>(base, off, 64 + 16 * P->nitems);
  P->Fu = carve<double>(base, off, 16 + 9 * P->nitems);
  // partial sums: 9 per 256-voxel block of every item, plus slack for the
  // per-item rounding of the line passes
  P->part_n = (size_t)9 * P->nitems * (N / 256 + 2) + 8192;
  P->part = carve<double>(base, off, P->part_n);
  P->part2 = carve<double>(base, off, P->part_n);
  const size_t tb = (P->prec == FG_FP64) ? sizeof(double) : sizeof(float);
  P->S64 = carve<double>(base, off, 9 * NT);
  if (P->prec == FG_FP64) {
    P->S = P->S64;
  } else {
    P->S = carve<char>(base, off, 9 * NT * tb);
  }
  P->x = carve<char>(base, off, 9 * NT * tb);
  P->r = carve<char>(base, off, 9 * NT * tb);
  P->p = carve<char>(base, off, 9 * NT * tb);
  P->st = carve<char>(base, off, (size_t)fg::state_words(P->law) * NT * tb);
  P->dcb = carve<char>(base, off, (size_t)9 * n0 * n1 * P->nitems * sizeof(cplx<double>));
  // scalar solvers (phase field, Fick) only on single plans; batches keep
  // just the zero fields standing in for c and d
  P->sc = carve<double>(base, off, P->nitems == 1 ? 16 * N : NT);
  return off;
}

// Host tables: long double trigonometry rounded once to the working type.
template <typename R> void host_tables(const fg_plan* P, std::vector<char>& blob, const TablesDev<R>& dev,
                                       char* ws_base) {
  auto put = [&](void* dptr, const void* src, size_t bytes) {
    const size_t off = (char*)dptr - ws_base;
    std::memcpy(blob.data() + off, src, bytes);
  };
  const long double PI = 3.141592653589793238462643383279502884L;
  auto roots = [&](int L, void* dptr) {
    std::vector<cplx<R>> w(L);
    for (int j = 0; j < L; ++j) {
      const long double a = 2.0L * PI * (long double)j / (long double)L;
      w[j].x = (R)std::cos(a);
      w[j].y = (R)(-std::sin(a));
      if (4 * j == L) { w[j].x = 0; w[j].y = -1; }
      if (2 * j == L) { w[j].x = -1; w[j].y = 0; }
      if (4 * j == 3 * L) { w[j].x = 0; w[j].y = 1; }
      if (j == 0) { w[j].x = 1; w[j].y = 0; }
    }
    put(dptr, w.data(), L * sizeof(cplx<R>));
  };
  roots(P->n0, dev.tw0);
  roots(P->n1, dev.tw1);
  roots(P->M, dev.twM);
  {
    std::vector<cplx<R>> w(P->M);
    for (int k = 0; k < P->M; ++k) {
      const long double a = 2.0L * PI * (long double)k / (long double)P->n2;
      w[k].x = (R)std::cos(a);
      w[k].y = (R)(-std::sin(a));
      if (k == 0) { w[k].x = 1; w[k].y = 0; }
      if (4 * k == P->n2) { w[k].x = 0; w[k].y = -1; }
    }
    put(dev.post, w.data(), P->M * sizeof(cplx<R>));
  }
  // cos(q/2), (2/h) sin(q/2) and sin(q/2) at q = 2 pi m / n (the rotated
  // vector and the half-voxel phase e^{i q/2} of the potential form)
  auto half = [&](int n, int count, double h, void* cptr, void* sptr, void* nptr) {
    std::vector<R> cc(count), ss(count), sn(count);
    for (int m = 0; m < count; ++m) {
      const long double a = PI * (long double)m / (long double)n;
      long double cv = std::cos(a), sv = std::sin(a);
      if (m == 0) sv = 0.0L;
      if (2 * m == n) {
        cv = 0.0L;  // exact values at q = pi
        sv = 1.0L;
      }
      cc[m] = (R)cv;
      ss[m] = (R)((2.0L / (long double)h) * sv);
      sn[m] = (R)sv;
    }
    put(cptr, cc.data(), count * sizeof(R));
    put(sptr, ss.data(), count * sizeof(R));
    put(nptr, sn.data(), count * sizeof(R));
  };
  half(P->n0, P->n0, P->h[0], dev.cz, dev.sz, dev.snz);
  half(P->n1, P->n1, P->h[1], dev.cy, dev.sy, dev.sny);
  half(P->n2, P->M + 1, P->h[2], dev.cx, dev.sx, dev.snx);
}

// Event pair around one launch of a kernel class (when that class is being
// timed).  With `in_launch` the scope only hands out the pair (start, stop)
// for a launch that records them itself (hipExtLaunchKernelGGL: the kernel's
// own start and end, no marker packets between kernels); otherwise the
// events are recorded on the stream around the scope.
struct ProfScope {
  fg_plan* P;
  int pass;
  hipEvent_t start = nullptr, stop = nullptr;
  bool in_launch;
  ProfScope(fg_plan* P_, int pass_, bool in_launch_ = false) : P(P_), pass(pass_), in_launch(in_launch_) {
    if (!P->prof_on || !(P->prof_mask >> pass & 1u)) return;
    auto& v = P->prof_ev[pass];
    size_t& u = P->prof_used[pass];
    if (u == v.size()) {
      hipEvent_t a, b;
      FG_HIP(hipEventCreate(&a));
      FG_HIP(hipEventCreate(&b));
      v.emplace_back(a, b);
    }
    start = v[u].first;
    stop = v[u].second;
    ++u;
    if (!in_launch) FG_HIP(hipEventRecord(start, P->stream));
  }
  ~ProfScope() {
    if (stop && !in_launch) (void)hipEventRecord(stop, P->stream);
  }
};

inline unsigned blocks_for(long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }
inline unsigned grid_stride_blocks(long n) { return (unsigned)std::min<long>(2048, (n + 255) / 256); }

void check_launch() { FG_HIP(hipGetLastError()); }

void sync_read(fg_plan* P) {
  FG_HIP(hipMemcpyAsync(P->hks, P->ks, (P->nitems + 1) * sizeof(KrylovScalars), hipMemcpyDeviceToHost, P->stream));
  FG_HIP(hipMemcpyAsync(P->hd, P->dscal, (64 + 16 * P->nitems) * sizeof(double), hipMemcpyDeviceToHost,
                        P->stream));
  FG_HIP(hipMemcpyAsync(P->hflags, P->flags, 4 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
  FG_HIP(hipStreamSynchronize(P->stream));
}

void check_domain(fg_plan* P) {
  if (P->hflags[0] & FG_FLAG_DOMAIN) {
    FG_HIP(hipMemsetAsync(P->flags, 0, 4 * sizeof(int), P->stream));
    throw Status(FG_E_DOMAIN, "det F <= 0, 1 + Omega c <= 0 or c outside (0, 1)");
  }
}

// Sum of nparts partials into dscal[slot].
void reduce_to(fg_plan* P, const double* parts, int nparts, int slot) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, parts, nparts, (KrylovScalars*)nullptr,
                     P->dscal + slot, 2, 0);
  check_launch();
}

// Per-item sums (nparts partials per item, item-major) into the item slot
// array dscal[64 + 16 b + slot]... stored as dscal[64 + slot * nitems + b].
void reduce_items(fg_plan* P, const double* parts, int nparts_per_item, int slot) {
  hipLaunchKernelGGL(k_finalize, dim3(P->nitems), dim3(1024), 0, P->stream, parts, nparts_per_item,
                     (KrylovScalars*)nullptr, P->dscal + 64 + (long)slot * P->nitems, 2, 0);
  check_launch();
}
inline double item_value(const fg_plan* P, int slot, int b) { return P->hd[64 + (long)slot * P->nitems + b]; }

// ----------------------------------------------------------------------------
// 3-D transforms on the plan grid.
template <typename R> const TablesDev<R>& tabs(const fg_plan* P);
template <> const TablesDev<double>& tabs<double>(const fg_plan* P) { return P->t64; }
template <> const TablesDev<float>& tabs<float>(const fg_plan* P) { return P->t32; }
template <typename R> int tile_axis(const fg_plan* P) { return P->tiles[sizeof(R) == 8 ? 0 : 2]; }
template <typename R> int tile_zproj(const fg_plan* P) { return P->tiles[sizeof(R) == 8 ? 1 : 3]; }

// Forward passes 1 and 2 (N2 real-to-complex, N1 complex) of ncomp fields,
// in -> data (in may equal data).  In a batch the ncomp fields are
// ncomp / nitems per item, item-major; skip masks whole items.
template <typename R>
void fwd_xy(fg_plan* P, const R* in, R* data, int ncomp, const Skip& skip) {
  const SpecTables<R> tb = tabs<R>(P).spec();
  const long cpi = ncomp / P->nitems;
  {
    ProfScope ps(P, FG_PASS_R2C);
    launch_r2c<R>(P->M, in, data, (long)ncomp * P->n0 * P->n1, tb, skip.unit(cpi * P->n0 * P->n1), P->stream);
  }
  ProfScope ps(P, FG_PASS_AXIS);
  launch_axis<R>(P->n1, false, data, P->M, (long)P->n1 * P->M, 0, P->M, ncomp * P->n0, 1, tb.tw1,
                 skip.unit(cpi * P->n0), P->stream, tile_axis<R>(P));
}

// Inverse passes 2 and 1, data -> out with the C2R epilogue; returns #partials.
template <typename R>
int inv_yx(fg_plan* P, R* data, R* out, int ncomp, const C2REpi& epi) {
  const SpecTables<R> tb = tabs<R>(P).spec();
  const long cpi = ncomp / P->nitems;
  {
    ProfScope ps(P, FG_PASS_AXIS);
    launch_axis<R>(P->n1, true, data, P->M, (long)P->n1 * P->M, 0, P->M, ncomp * P->n0, 1, tb.tw1,
                   epi.skip.unit(cpi * P->n0), P->stream, tile_axis<R>(P));
  }
  ProfScope ps(P, FG_PASS_C2R);
  C2REpi e = epi;
  e.skip = epi.skip.unit(cpi * P->n0 * P->n1);
  return launch_c2r<R>(P->M, data, out, (long)ncomp * P->n0 * P->n1, tb, e, P->stream);
}

// y = G * x for the 9-component fields of all items (projection); returns
// the number of partials (all items; nitems divides it).
template <typename R>
int project9(fg_plan* P, const R* in, R* work, R* out, const C2REpi& epi) {
  fwd_xy<R>(P, in, work, 9 * P->nitems, epi.skip);
  {
    ProfScope ps(P, FG_PASS_ZPROJ);
    launch_zproj<R>(P->n0, work, P->n1, P->M, tabs<R>(P).spec(), (R)(1.0 / (double)P->N), epi.skip.unit(3),
                    P->stream, P->nitems, tile_zproj<R>(P));
  }
  return inv_yx<R>(P, work, out, 9 * P->nitems, epi);
}

// y = F^-1[ F[x] / (a0 + a1 lambda) ] for one scalar field, returns #partials.
template <typename R>
int precond1(fg_plan* P, const R* in, R* work, R* out, double a0, double a1, const C2REpi& epi) {
  fwd_xy<R>(P, in, work, 1, epi.skip);
  {
    ProfScope ps(P, FG_PASS_ZSCALAR);
    launch_zscalar<R>(P->n0, work, P->n1, P->M, tabs<R>(P).spec(), (R)(1.0 / (double)P->N), a0, a1, epi.skip,
                      P->stream);
  }
  return inv_yx<R>(P, work, out, 1, epi);
}

// ----------------------------------------------------------------------------
// Mechanics.
void constitutive(fg_plan* P, const double* Fu, double* Pout, void* state, double* pparts,
                  const int* idle = nullptr) {
  ProfScope ps(P, FG_PASS_CONSTITUTIVE);
  const dim3 grid(blocks_for(P->N), (unsigned)P->nitems);
  const double* c = P->c ? P->c : P->zeroN;
  const double* d = P->d ? P->d : P->zeroN;
  if (P->prec == FG_FP64)
    hipLaunchKernelGGL((k_constitutive<double>), grid, dim3(256), 0, P->stream, P->F, Fu, c, d, P->E, P->nu,
                       P->Om, Pout, (double*)state, pparts, P->flags, P->N, idle, P->law);
  else
    hipLaunchKernelGGL((k_constitutive<float>), grid, dim3(256), 0, P->stream, P->F, Fu, c, d, P->E, P->nu,
                       P->Om, Pout, (float*)state, pparts, P->flags, P->N, idle, P->law);
  check_launch();
}

// ||G*P|| of the stress in S64 (in place), into dscal[slot]; G*P stays in S64.
void potential64(fg_plan* P, double* field, const Skip& skip);

// |G*P|^2 of the FP64 9-component fields in S64 (all items not idle) by the
// potential route: S64 is replaced by the potential U(P) (slot 3i of each
// item, D U = G*P) and the partial sums of |D U|^2 go to P->part; returns
// the partials per item.  A following cg_start may reuse U.
int residual_pot(fg_plan* P, const int* idle) {
  potential64(P, P->S64, idle ? Skip::flags(idle) : Skip{});
  return launch_grad_norm(P->S64, 3 * P->N, 9 * P->N, idle, P->part, P->n0, P->n1, P->n2, P->nitems, P->h,
                          P->stream);
}

// |G*P|^2 of a single-item plan into dscal[slot] (S64 ends up holding U(P)).
void residual_norm(fg_plan* P, int slot) { reduce_to(P, P->part, residual_pot(P, nullptr), slot); }

// mean of a 9-component FP64 field into dscal[8 + k]
void mean9(fg_plan* P, const double* field) {
  const unsigned nb = blocks_for(P->N);
  hipLaunchKernelGGL(k_mean9_partials, dim3(nb), dim3(256), 0, P->stream, field, P->part2, P->N);
  check_launch();
  for (int k = 0; k < 9; ++k) reduce_to(P, P->part2 + (size_t)k * nb, (int)nb, 8 + k);
}

// Iterations to launch before the next convergence read-back: half the
// number predicted from the mean contraction rate of r.r so far, so that
// few launches land after convergence (they exit at once but still cost a
// launch each).
int next_chunk(const KrylovScalars& h, long launched) {
  if (h.iter <= 0 || !(h.rr > 0.0) || !(h.rr0 > 0.0) || !(h.tol2 > 0.0)) return 8;
  const double rate = std::log(h.rr / h.rr0) / (double)h.iter;  // < 0 when converging
  const double need = std::log(h.tol2 * h.rr0 / h.rr);            // < 0 while not converged
  int k = 8;
  if (rate < -1e-12) k = (int)std::ceil(0.5 * need / rate);
  k = std::max(1, std::min(k, 64));
  if (h.maxit > 0) k = std::min(k, std::max(1, h.maxit - h.iter));
  (void)launched;
  return k;
}

// Kernel launches of the CG loop that found the solve already converged
// (they return at once); excluded from the profiled launch counts.
void note_noop_iterations(fg_plan* P, long noop) {
  if (!P->prof_on || noop <= 0) return;
  for (int pass : {FG_PASS_FRONT, FG_PASS_AXIS, FG_PASS_ZPROJ, FG_PASS_AXIS3, FG_PASS_C2R3, FG_PASS_GRAD,
                   FG_PASS_FINALIZE})
    if (P->prof_mask >> pass & 1u) P->prof_noop[pass] += noop;
}

// Grid of a per-item field kernel: up to 256 blocks per item, grid.y = item.
inline dim3 item_grid(long n, int nitems) {
  return dim3((unsigned)std::min<long>(256, (n + 255) / 256), (unsigned)nitems);
}

// Inverse half of the projection in the potential form for all items: the
// 3-component potential U (slots 0, 3, 6 of each item, spectral, written by
// launch_zgrad) back to real space: N1 pass, then N2 complex-to-real.
template <typename R>
void inv_potential(fg_plan* P, R* data, const Skip& skip) {
  const SpecTables<R> tb = tabs<R>(P).spec();
  const long lines = (long)P->n0 * P->n1;
  {
    ProfScope ps(P, FG_PASS_AXIS3, true);
    // planes y = i0, z = 3 item + c (components 3 apart)
    launch_axis<R>(P->n1, true, data, P->M, (long)P->n1 * P->M, 3L * P->n0 * P->n1 * P->M, P->M, P->n0,
                   3 * P->nitems, tb.tw1, skip.unit(3L * P->n0), P->stream, tile_axis<R>(P), ps.start, ps.stop);
  }
  ProfScope ps(P, FG_PASS_C2R3, true);
  // sub-items (item, c) of N0 N1 lines, 3 N0 N1 lines apart, 3 per item
  Skip sk = skip.unit(lines);
  sk.item_stride = 3 * lines;
  sk.sub = 3;
  C2REpi epi{1.0, nullptr, true, nullptr, sk};
  launch_c2r<R>(P->M, data, data, 3 * lines * P->nitems, tb, epi, P->stream, ps.start, ps.stop);
}

// One CG iteration for every item of the plan (items whose solve is done
// skip every kernel), on the potentials rho, pi, xi of r = D rho, p = D pi,
// x = D xi (fg_potential.hpp):
//   xi += alpha_{k-1} pi_{k-1}; pi = rho + beta pi; Y = K:(D pi); p.Y; N2
//   pass of Y; N1 pass (9 components in, the two terms of each row that
//   share the N0 factor merged; alpha = r.r / p.Kp by one workgroup per
//   item); N0 pass reducing the projection to the 3-component potential; N1
//   and N2 inverse passes of the potential U (D U = G(K p)); rho -= alpha U,
//   r.r = |D rho|^2; beta, convergence.
template <typename T>
void cg_iteration(fg_plan* P) {
  T* S = (T*)P->S;
  const int nit = P->nitems;
  KrylovScalars* ks = P->ks;
  const SpecTables<T> tb = tabs<T>(P).spec();
  const Skip skip = Skip::done(ks);
  int nbf;
  {
    ProfScope ps(P, FG_PASS_FRONT, true);
    nbf = launch_cg_front<T>(P->M, S, (T*)P->p, (T*)P->x, (const T*)P->r, (const T*)P->st, ks, P->part, P->N, P->n0,
                             P->n1, P->h, tb, P->stream, nit, ps.start, ps.stop, P->law);
  }
  {
    // alpha = r.r / p.Ap is formed by the row pass (one workgroup per item)
    ProfScope ps(P, FG_PASS_AXIS, true);
    launch_axis_rows<T>(P->n1, S, P->n0, P->M, tb, skip, P->stream, nit, tile_axis<T>(P), P->part, nbf / nit, ks,
                        (T*)P->dcb, ps.start, ps.stop);
  }
  {
    ProfScope ps(P, FG_PASS_ZPROJ, true);
    launch_zgrad<T>(P->n0, S, P->n1, P->M, tb, (T)(1.0 / (double)P->N), skip, P->stream, nit, tile_zproj<T>(P),
                    (const T*)P->dcb, ps.start, ps.stop);
  }
  inv_potential<T>(P, S, skip);
  int nbg;
  {
    ProfScope ps(P, FG_PASS_GRAD, true);
    nbg = launch_cg_rupd<T>((const T*)S, 3 * P->N, (T*)P->r, ks, nullptr, P->part2, P->n0, P->n1, P->n2, nit, P->h, 0,
                            P->stream, ps.start, ps.stop);
  }
  {
    ProfScope ps(P, FG_PASS_FINALIZE, true);
    launch_ev(k_finalize, dim3(nit), dim3(1024), 0, P->stream, ps.start, ps.stop, (const double*)P->part2, nbg, ks,
              (double*)nullptr, 1, 0);
  }
  check_launch();
}

// Potential of the 9-component FP64 fields in `field` (all items), in place:
// N2, N1 (rows merged), N0 (projection to the potential) and the inverse N1
// and N2 passes.  Afterwards slot 3i of each item holds the real U_i with
// D U = G(field).
void potential64(fg_plan* P, double* field, const Skip& skip) {
  const SpecTables<double> tb = P->t64.spec();
  {
    ProfScope ps(P, FG_PASS_R2C);
    launch_r2c<double>(P->M, field, field, 9L * P->n0 * P->n1 * P->nitems, tb, skip.unit(9L * P->n0 * P->n1),
                       P->stream);
  }
  {
    ProfScope ps(P, FG_PASS_AXIS);
    launch_axis_rows<double>(P->n1, field, P->n0, P->M, tb, skip, P->stream, P->nitems, tile_axis<double>(P), nullptr,
                             0, nullptr, (double*)P->dcb);
  }
  {
    ProfScope ps(P, FG_PASS_ZPROJ);
    launch_zgrad<double>(P->n0, field, P->n1, P->M, tb, 1.0 / (double)P->N, skip, P->stream, P->nitems,
                         tile_zproj<double>(P), (const double*)P->dcb);
  }
  inv_potential<double>(P, field, skip);
}

// CG start on the potentials for every item not idle: rho_0 = sign U with U
// the potential of the FP64 field `field` (overwritten; with potential_ready
// `field` already holds U, as residual_pot leaves it), so that
// r_0 = D rho_0 = sign G(field); xi = 0; per-block partial sums of
// |r_0|^2 = |D rho_0|^2 into P->part.  Returns the partials per item (the
// caller reduces them into the Krylov scalars).
template <typename T>
int cg_start(fg_plan* P, double* field, double sign, const int* idle, bool potential_ready = false) {
  if (!potential_ready) potential64(P, field, idle ? Skip::flags(idle) : Skip{});
  const long N = P->N;
  hipLaunchKernelGGL((k_cg_start_pot<T>), item_grid(3 * N, P->nitems), dim3(256), 0, P->stream, (T*)P->r, (T*)P->x,
                     (const double*)field, 3 * N, 9 * N, sign, idle, N);
  const int nb = launch_cg_rupd<T>((const T*)P->r, 0, (T*)P->r, P->ks, idle, P->part, P->n0, P->n1, P->n2, P->nitems,
                                   P->h, 2, P->stream);
  check_launch();
  return nb;
}

// Single-item CG start: cg_start and the Krylov scalars (rr0 = rr = |r_0|^2,
// iter = 0, done if r_0 = 0).
template <typename T>
void cg_start1(fg_plan* P, double* field, double sign, bool potential_ready = false) {
  const int nb = cg_start<T>(P, field, sign, nullptr, potential_ready);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part, nb, P->ks, (double*)nullptr, 5, 0);
  check_launch();
}

// The CG solution x = D xi of every item not idle, in double precision, into
// the 9-component field dst (after the last deferred update of xi).
template <typename T>
void cg_result(fg_plan* P, double* dst, const int* idle) {
  const long N = P->N;
  hipLaunchKernelGGL((k_cg_final_xi<T>), item_grid(3 * N, P->nitems), dim3(256), 0, P->stream, (T*)P->x,
                     (const T*)P->p, (const KrylovScalars*)P->ks, idle, N);
  launch_grad_store<T, double>((const T*)P->x, N, 9 * N, dst, 9 * N, idle, P->n0, P->n1, P->n2, P->nitems, P->h,
                               P->stream);
  check_launch();
}

template <typename T>
void cg_solve(fg_plan* P, const fg_solver_opts* o, fg_stats* stats) {
  KrylovScalars* ks = P->ks;
  // rho_0, xi = 0 and ks (rr0, rr, iter = 0, done) were set by cg_start1
  {
    // only tol2 / maxit are host-set; the rest was set on the device
    P->hd[62] = (o->fixed_lin > 0) ? 0.0 : o->tol_lin * o->tol_lin;
    ((int*)(P->hd + 63))[0] = (o->fixed_lin > 0) ? o->fixed_lin : o->max_lin;
    FG_HIP(hipMemcpyAsync(&ks->tol2, P->hd + 62, sizeof(double), hipMemcpyHostToDevice, P->stream));
    FG_HIP(hipMemcpyAsync(&ks->maxit, P->hd + 63, sizeof(int), hipMemcpyHostToDevice, P->stream));
  }
  int chunk = 8;
  long launched = 0;
  for (int guard = 0; guard < 1000000; ++guard) {
    launched += chunk;
    for (int k = 0; k < chunk; ++k) cg_iteration<T>(P);
    sync_read(P);
    if (P->hks[0].done) break;
    chunk = next_chunk(P->hks[0], launched);
  }
  const KrylovScalars& h = P->hks[0];
  note_noop_iterations(P, launched - h.iter);
  if (stats) {
    stats->lin_iters_last = h.iter;
    stats->lin_relres = h.rr0 > 0 ? std::sqrt(h.rr / h.rr0) : 0.0;
  }
  // Both precisions report a breakdown (p.Ap <= 0) and the iteration cap:
  // a correction from an indefinite or unconverged solve is not handed on.
  if (h.flag == 1) throw Status(FG_E_BREAKDOWN, "CG breakdown: p.Ap <= 0");
  if (h.flag == 2) throw Status(FG_E_NOCONV, "CG reached max_lin iterations");
}

// Normaliser of eq. (31) for the macroscopic F_macro: ||G*P(F_macro)||
// with the floors of reading A8 (max with 1e-14 ||P(F_macro)|| and 1e-300).
double residual_denominator(fg_plan* P, const double Fmacro[9]) {
  FG_HIP(hipMemcpyAsync(P->Fu, Fmacro, 9 * sizeof(double), hipMemcpyHostToDevice, P->stream));
  const unsigned nbN = blocks_for(P->N);
  constitutive(P, P->Fu, P->S64, nullptr, P->part2);
  reduce_to(P, P->part2, (int)nbN, 0);  // ||P(Fbar)||^2
  residual_norm(P, 1);                  // ||G*P(Fbar)||^2
  sync_read(P);
  check_domain(P);
  return std::max(std::max(std::sqrt(P->hd[1]), 1e-14 * std::sqrt(P->hd[0])), 1e-300);
}

// P and the tangent state at the current F, and ||G*(P - B)|| (B = 0 when
// null); S64 is left holding the potential U(P - B) (D U = G*(P - B)) that the
// CG start reuses.
double newton_residual_norm(fg_plan* P, const double* B = nullptr) {
  constitutive(P, nullptr, P->S64, P->st, nullptr);
  if (B) {
    const long n9 = 9 * P->N;
    hipLaunchKernelGGL(k_sub_f64, dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, P->S64, B, n9);
    check_launch();
  }
  residual_norm(P, 2);
  sync_read(P);
  check_domain(P);
  return std::sqrt(P->hd[2]);
}
double newton_residual(fg_plan* P, double den) { return newton_residual_norm(P) / den; }

// Newton loop of Alg. 1 at the current F (increment already applied).
// With B, the equation is G*(P(F) - B) = 0 and err_res is normalised by its
// value at the entry state (Fmacro unused).
void newton(fg_plan* P, const double Fmacro[9], const fg_solver_opts* o, fg_stats* stats,
            const double* B = nullptr) {
  const long n9 = 9 * P->N;
  double den = B ? 0.0 : residual_denominator(P, Fmacro);
  int it = 0;
  if (stats) {
    stats->newton_iters = 0;
    stats->lin_iters_total = 0;
    stats->n_history = 0;
  }
  while (true) {
    const double rn = newton_residual_norm(P, B);
    if (B && it == 0) den = (rn > 0.0) ? rn : 1.0;
    const double err = rn / den;
    if (stats) {
      if (stats->n_history < 64) stats->err_history[stats->n_history] = err;
      stats->n_history += 1;
      stats->err_res = err;
    }
    if (!(err == err)) throw Status(FG_E_NOCONV, "Newton residual is NaN");
    // The mixed form converges linearly (inner forcing 1e-6) where the FP64
    // form converges quadratically and lands well below tol_newton; refining
    // to 0.01 tol_newton gives both the same final accuracy.
    const double tol_eff = (P->prec == FG_MIXED) ? 0.01 * o->tol_newton : o->tol_newton;
    if (err <= tol_eff) break;
    if (it >= o->max_newton) throw Status(FG_E_NOCONV, "Newton reached max_newton iterations");
    // b = -G*P: r_0 = D rho_0 with rho_0 = -U(P), the potential the residual
    // pass left in S64
    if (P->prec == FG_FP64) {
      cg_start1<double>(P, P->S64, -1.0, true);
      cg_solve<double>(P, o, stats);
      cg_result<double>(P, P->S64, nullptr);
    } else {
      fg_solver_opts om = *o;
      // Inner forcing: the single-precision operator is accurate to a few
      // 1e-7 at 256^3 (FFT rounding), so CG is not asked for more than 1e-5;
      // the double-precision Newton residual refines the rest.
      if (om.fixed_lin <= 0) om.tol_lin = std::max(o->tol_lin, 1e-5);
      cg_start1<float>(P, P->S64, -1.0, true);
      cg_solve<float>(P, &om, stats);
      // dF = D xi evaluated in double precision: a discrete gradient, hence
      // compatible to rounding whatever the single-precision error of xi
      cg_result<float>(P, P->S64, nullptr);
    }
    hipLaunchKernelGGL((k_axpy_into_f64<double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, P->F,
                       (const double*)P->S64, n9);
    check_launch();
    if (stats) {
      if (it < 64) stats->lin_history[it] = stats->lin_iters_last;
      stats->lin_iters_total += stats->lin_iters_last;
    }
    ++it;
    if (stats) stats->newton_iters = it;
  }
}

// Adjoint of L = sum W_ij <P_ij> at the current (converged) state: solve
// G(K:lam) = -G(K:W) for the compatible, zero-mean lam with the same CG (lam
// = D xi), then the per-voxel gradients with respect to log E and Omega.
// <K : (W + lam)> of the adjoint solution lam into Tout (host, 9): the
// homogenised tangent applied to W (d<P>/dFbar : W), by the major symmetry
// of K the same linear solve as the adjoint.
// Y = K : X from the stored tangent state of the plan's law (one item).
template <typename T> void launch_contract(fg_plan* P, T* Y, const T* X) {
  const dim3 grid(blocks_for(P->N / 2));
  if (P->law == ::FG_LAW_SVK)
    hipLaunchKernelGGL((k_contract<T, fg::kLawSVK>), grid, dim3(256), 0, P->stream, Y, X, (const T*)P->st, P->N);
  else
    hipLaunchKernelGGL((k_contract<T, fg::kLawNH>), grid, dim3(256), 0, P->stream, Y, X, (const T*)P->st, P->N);
}

void tangent_mean(fg_plan* P, const double* lam, double* Tout) {
  const long N = P->N;
  const double* c = P->c ? P->c : P->zeroN;
  const double* d = P->d ? P->d : P->zeroN;
  hipLaunchKernelGGL(k_tangent_apply_f64, dim3(blocks_for(N)), dim3(256), 0, P->stream, P->F, c, d, P->E, P->nu,
                     P->Om, (const double*)P->Fu, lam, P->S64, P->flags, N, P->law);
  check_launch();
  mean9(P, P->S64);
  sync_read(P);
  check_domain(P);
  for (int k = 0; k < 9; ++k) Tout[k] = P->hd[8 + k] / (double)N;
}

template <typename T>
void adjoint(fg_plan* P, const double W[9], double* gE, double* gO, const fg_solver_opts* o, fg_stats* stats,
             double* Tout = nullptr) {
  const long N = P->N;
  T* S = (T*)P->S;
  T* pbuf = (T*)P->p;
  constitutive(P, nullptr, nullptr, P->st, nullptr);
  FG_HIP(hipMemcpyAsync(P->Fu, W, 9 * sizeof(double), hipMemcpyHostToDevice, P->stream));
  hipLaunchKernelGGL((k_fill_uniform9<T>), dim3(blocks_for(N)), dim3(256), 0, P->stream, pbuf, (const double*)P->Fu,
                     N);
  launch_contract<T>(P, S, (const T*)pbuf);
  check_launch();
  static_assert(sizeof(T) == 8, "the single-precision adjoint is adjoint_mixed");
  {
    // b = -G*(K:W): r_0 = D rho_0 with rho_0 = -U, U the potential of K:W
    // (D U = G*(K:W))
    cg_start1<double>(P, (double*)S, -1.0);
  }
  sync_read(P);
  check_domain(P);
  if (!P->hks[0].done) cg_solve<T>(P, o, stats);
  // lam = D xi (zero when the right-hand side vanishes: xi = 0)
  double* lam = (double*)P->r;
  cg_result<double>(P, lam, nullptr);
  const double* c = P->c ? P->c : P->zeroN;
  const double* d = P->d ? P->d : P->zeroN;
  if (gE || gO) {
    hipLaunchKernelGGL((k_adjoint_grad<T>), dim3(blocks_for(N)), dim3(256), 0, P->stream, P->F, c, d, P->E, P->nu,
                       P->Om, (const T*)lam, (const double*)P->Fu, gE, gO, P->flags, N, P->law);
    check_launch();
  }
  if (Tout) tangent_mean(P, lam, Tout);
  sync_read(P);
  check_domain(P);
}

// Mixed form of the adjoint: the system G*(K:lam) = -G*(K:W) is refined in
// double precision, lam_{k+1} = lam_k + G*(d_k), where d_k solves
// G*(K:d) = R_k by CG with the single-precision operator and
//   R_k = -G*(G*(K:(W + lam_k)))
// is the double-precision residual (K evaluated from F on the fly).  Stops
// when ||R_k|| <= tol_lin ||R_0||, the criterion of the double-precision CG.
// lam lives in the (otherwise unused) scalar-solver area.
void adjoint_mixed(fg_plan* P, const double W[9], double* gE, double* gO, const fg_solver_opts* o,
                   fg_stats* stats, double* Tout = nullptr) {
  const long N = P->N, n9 = 9 * N;
  double* lam = P->sc;
  const double* c = P->c ? P->c : P->zeroN;
  const double* d = P->d ? P->d : P->zeroN;
  constitutive(P, nullptr, nullptr, P->st, nullptr);  // single-precision state for the inner CG
  FG_HIP(hipMemcpyAsync(P->Fu, W, 9 * sizeof(double), hipMemcpyHostToDevice, P->stream));
  hipLaunchKernelGGL((k_fill<double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, lam, 0.0, n9);
  check_launch();
  const unsigned nbN = blocks_for(N);
  double rr0 = 0.0, rr = 0.0;
  int refine = 0;
  for (;; ++refine) {
    hipLaunchKernelGGL(k_tangent_apply_f64, dim3(nbN), dim3(256), 0, P->stream, P->F, c, d, P->E, P->nu, P->Om,
                       (const double*)P->Fu, (const double*)lam, P->S64, P->flags, N, P->law);
    check_launch();
    C2REpi e1{1.0, nullptr, true, nullptr, Skip{}};
    project9<double>(P, P->S64, P->S64, P->S64, e1);
    C2REpi e2{-1.0, nullptr, true, P->part, Skip{}};
    const int nb = project9<double>(P, P->S64, P->S64, P->S64, e2);
    // rr = R.R, and the inner CG starts from it (rr0 of the correction)
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part, nb, P->ks, (double*)nullptr, 5, 0);
    check_launch();
    sync_read(P);
    check_domain(P);
    rr = P->hks[0].rr0;
    if (refine == 0) rr0 = rr;
    if (rr0 == 0.0 || std::sqrt(rr / rr0) <= o->tol_lin) break;
    if (refine >= 30) throw Status(FG_E_NOCONV, "mixed adjoint: refinement did not converge");
    // inner CG on R_k (compatible, in S64): rho_0 = U of R_k, r_0 = D rho_0
    cg_start1<float>(P, P->S64, 1.0);
    fg_solver_opts om = *o;
    // the correction reduces R_k by 1e-5 at most (single-precision operator),
    // and by no more than what is left to reach tol_lin ||R_0||
    om.fixed_lin = 0;
    om.tol_lin = std::max(1e-5, o->tol_lin * std::sqrt(rr0 / rr));
    fg_stats inner{};
    cg_solve<float>(P, &om, &inner);
    if (stats) stats->lin_iters_total += inner.lin_iters_last;
    // lam += G*(d) in double precision, d = D xi
    cg_result<float>(P, P->S64, nullptr);
    project9<double>(P, P->S64, P->S64, P->S64, e1);
    hipLaunchKernelGGL((k_axpy_into_f64<double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, lam,
                       (const double*)P->S64, n9);
    check_launch();
  }
  if (stats) {
    stats->newton_iters = refine;  // double-precision refinements
    stats->lin_iters_last = stats->lin_iters_total;
    stats->lin_relres = rr0 > 0 ? std::sqrt(rr / rr0) : 0.0;
  }
  if (gE || gO) {
    hipLaunchKernelGGL((k_adjoint_grad<double>), dim3(nbN), dim3(256), 0, P->stream, P->F, c, d, P->E, P->nu, P->Om,
                       (const double*)lam, (const double*)P->Fu, gE, gO, P->flags, N, P->law);
    check_launch();
  }
  if (Tout) tangent_mean(P, lam, Tout);
  sync_read(P);
  check_domain(P);
}

// ----------------------------------------------------------------------------
// Scalar PCG (shared by the phase-field and Fick solves).  Vectors in the
// scalar area: x, r, z, p, q, work (spectral).  ks[1] holds the scalars; the
// caller has set r = b, x = 0 and ks[1] (rr0) via mode 5.
enum class ScalarOp { PFF, FICK };

struct ScalarVecs {
  double *x, *r, *z, *p, *q, *work, *a, *w, *mu, *A6, *ct;
};

ScalarVecs scalar_vecs(fg_plan* P) {
  const long N = P->N;
  double* b = P->sc;
  ScalarVecs v;
  v.x = b + 0 * N;
  v.r = b + 1 * N;
  v.z = b + 2 * N;
  v.p = b + 3 * N;
  v.q = b + 4 * N;
  v.work = b + 5 * N;
  v.a = b + 6 * N;
  v.w = b + 6 * N;  // Fick uses w where PFF uses a
  v.mu = b + 7 * N;
  v.ct = b + 8 * N;
  v.A6 = b + 9 * N;  // 6N
  // b + 15 N: zeros
  return v;
}

void scalar_pcg(fg_plan* P, ScalarOp op, double a0, double a1, double dt, const fg_solver_opts* o,
                fg_stats* stats) {
  ScalarVecs v = scalar_vecs(P);
  KrylovScalars* ks = P->ksc;
  P->hd[60] = (o->fixed_lin > 0) ? 0.0 : o->tol_lin * o->tol_lin;
  ((int*)(P->hd + 61))[0] = (o->fixed_lin > 0) ? o->fixed_lin : o->max_lin;
  FG_HIP(hipMemcpyAsync(&ks->tol2, P->hd + 60, sizeof(double), hipMemcpyHostToDevice, P->stream));
  FG_HIP(hipMemcpyAsync(&ks->maxit, P->hd + 61, sizeof(int), hipMemcpyHostToDevice, P->stream));
  const Skip skip = Skip::done(ks);
  const unsigned nbN = blocks_for(P->N);
  const unsigned nbu = grid_stride_blocks(P->N);
  const Grid3 g{P->n0, P->n1, P->n2, 1.0 / P->h[0], 1.0 / P->h[1], 1.0 / P->h[2]};
  // z = M r, rz
  auto apply_prec = [&]() {
    C2REpi epi{1.0, v.r, false, P->part, skip};
    const int nb = precond1<double>(P, v.r, v.work, v.z, a0, a1, epi);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part, nb, ks, (double*)nullptr, 4, 1);
  };
  apply_prec();
  check_launch();
  int chunk = 4;
  for (int guard = 0; guard < 1000000; ++guard) {
    for (int k = 0; k < chunk; ++k) {
      hipLaunchKernelGGL(k_pcg_dir, dim3(nbN), dim3(256), 0, P->stream, v.p, v.z, ks, P->N);
      if (op == ScalarOp::PFF)
        hipLaunchKernelGGL(k_pff_apply, dim3(nbN), dim3(256), 0, P->stream, v.p, v.a, P->gc * P->lc, g, v.q,
                           P->part, ks, P->N);
      else
        hipLaunchKernelGGL(k_fick_apply, dim3(nbN), dim3(256), 0, P->stream, v.p, v.w, v.A6, dt, g, v.q, P->part,
                           ks, P->N);
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part, (int)nbN, ks, (double*)nullptr, 0,
                         1);
      hipLaunchKernelGGL((k_cg_update<double>), dim3(nbu), dim3(256), 0, P->stream, v.x, v.r, v.p, v.q, ks,
                         P->part2, P->N);
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part2, (int)nbu, ks, (double*)nullptr, 3,
                         1);
      apply_prec();
      check_launch();
    }
    sync_read(P);
    if (P->hksc[0].done) break;
    chunk = next_chunk(P->hksc[0], 0);
  }
  const KrylovScalars& h = P->hksc[0];
  if (stats) {
    stats->lin_iters_last = h.iter;
    stats->lin_relres = h.rr0 > 0 ? std::sqrt(h.rr / h.rr0) : 0.0;
    stats->lin_iters_total += h.iter;
  }
  if (h.flag == 1) throw Status(FG_E_BREAKDOWN, "PCG breakdown: p.Ap <= 0");
  if (h.flag == 2) throw Status(FG_E_NOCONV, "PCG reached max_lin iterations");
}

void pff(fg_plan* P, const fg_solver_opts* o, fg_stats* stats) {
  if (!P->smax || !P->H || !P->d) throw Status(FG_E_STATE, "pff_solve needs sigma_max, d and H");
  ScalarVecs v = scalar_vecs(P);
  const unsigned nbN = blocks_for(P->N);
  const double* c = P->c ? P->c : P->zeroN;
  hipLaunchKernelGGL(k_pff_history, dim3(nbN), dim3(256), 0, P->stream, P->F, c, P->E, P->nu, P->Om, P->smax, P->H,
                     v.a, v.r, v.x, P->gc, P->lc, P->part, P->part2, P->flags, P->N, P->law);
  check_launch();
  reduce_to(P, P->part, (int)nbN, 0);  // sum H
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part2, (int)nbN, P->ksc, (double*)nullptr,
                     5, 1);
  check_launch();
  sync_read(P);
  check_domain(P);
  if (stats) stats->lin_iters_total = 0;
  const double Hbar = P->hd[0] / (double)P->N;
  if (!P->hksc[0].done) {
    scalar_pcg(P, ScalarOp::PFF, P->gc / P->lc + 2.0 * Hbar, P->gc * P->lc, 0.0, o, stats);
  } else if (stats) {
    stats->lin_iters_last = 0;
    stats->lin_relres = 0.0;
  }
  FG_HIP(hipMemcpyAsync(P->d, v.x, P->N * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
}

void fick(fg_plan* P, double dt, const double* cdot, const fg_solver_opts* o, fg_stats* stats,
          int full_jacobian = 0) {
  if (!P->c || !P->D) throw Status(FG_E_STATE, "fick_step needs c and D");
  ScalarVecs v = scalar_vecs(P);
  const long N = P->N;
  const unsigned nbN = blocks_for(N);
  const Grid3 g{P->n0, P->n1, P->n2, 1.0 / P->h[0], 1.0 / P->h[1], 1.0 / P->h[2]};
  FG_HIP(hipMemcpyAsync(v.ct, P->c, N * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
  const double* d = P->d ? P->d : P->zeroN;
  hipLaunchKernelGGL(k_fick_coef, dim3(nbN), dim3(256), 0, P->stream, P->F, d, v.ct, P->D, P->RT, v.A6, P->part,
                     P->part2, N);
  check_launch();
  reduce_to(P, P->part, (int)nbN, 0);   // sum tr(Aplus)
  reduce_to(P, P->part2, (int)nbN, 1);  // ||c_t||^2
  sync_read(P);
  const double abar = P->hd[0] / (double)N / 3.0;
  const double nct = std::sqrt(P->hd[1]);
  if (stats) {
    stats->newton_iters = 0;
    stats->lin_iters_total = 0;
    stats->n_history = 0;
  }
  for (int it = 0; it < o->max_newton; ++it) {
    hipLaunchKernelGGL(k_fick_mu, dim3(nbN), dim3(256), 0, P->stream, P->c, P->F, d, P->E, P->nu, P->Om, P->RT,
                       P->cmax, v.mu, v.w, P->part, P->flags, N, full_jacobian, P->law);
    check_launch();
    reduce_to(P, P->part, (int)nbN, 2);  // sum 1/w
    hipLaunchKernelGGL(k_fick_residual, dim3(nbN), dim3(256), 0, P->stream, P->c, v.ct, v.mu, v.A6, cdot, dt, g,
                       v.r, v.x, P->part2, N);
    check_launch();
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part2, (int)nbN, P->ksc,
                       (double*)nullptr, 5, 1);
    check_launch();
    sync_read(P);
    check_domain(P);
    const double winv = P->hd[2] / (double)N;
    if (!P->hksc[0].done) scalar_pcg(P, ScalarOp::FICK, winv, dt * abar, dt, o, stats);
    hipLaunchKernelGGL(k_fick_update, dim3(nbN), dim3(256), 0, P->stream, P->c, v.x, v.w, P->part, N);
    check_launch();
    reduce_to(P, P->part, (int)nbN, 3);
    sync_read(P);
    const double rel = std::sqrt(P->hd[3]) / nct;
    if (stats) {
      if (stats->n_history < 64) {
        stats->err_history[stats->n_history] = rel;
        stats->lin_history[stats->n_history] = stats->lin_iters_last;
      }
      stats->n_history += 1;
      stats->newton_iters = it + 1;
      stats->err_res = rel;
    }
    if (rel < o->tol_newton) return;
  }
  throw Status(FG_E_NOCONV, "Fick Newton reached max_newton iterations");
}

}  // namespace

namespace {
// F^0 = F_t + (F_macro - <F_t>): the macroscopic increment of Alg. 1.
void apply_macro(fg_plan* P, const double F_macro[9]) {
  mean9(P, P->F);
  sync_read(P);
  for (int k = 0; k < 9; ++k) P->hd[32 + k] = F_macro[k] - P->hd[8 + k] / (double)P->N;
  FG_HIP(hipMemcpyAsync(P->Fu, P->hd + 32, 9 * sizeof(double), hipMemcpyHostToDevice, P->stream));
  hipLaunchKernelGGL(k_add_uniform9, dim3(blocks_for(P->N)), dim3(256), 0, P->stream, P->F, (const double*)P->Fu,
                     P->N, P->N);
  check_launch();
}

}  // namespace

// ------------------------------------------------------------------ C ABI --
fg_status plan_set_workspace(fg_plan* P, void* dev, size_t bytes);
void plan_delete(fg_plan* P);

namespace {
fg_status run(fg_plan* P, const std::function<void()>& fn) {
  try {
    fn();
    if (P) P->err.clear();
    return FG_OK;
  } catch (const Status& s) {
    if (P) P->err = s.what();
    return s.code;
  } catch (const HipError& e) {
    if (P) P->err = e.what();
    return FG_E_HIP;
  } catch (const std::invalid_argument& e) {
    if (P) P->err = e.what();
    return FG_E_SIZE;
  } catch (const std::exception& e) {
    if (P) P->err = e.what();
    return FG_E_HIP;
  }
}

fg_status plan_new(const int grid[3], const double spacing[3], fg_precision prec, void* stream, int nitems,
                   fg_plan** out) {
  if (!grid || !spacing || !out) return FG_E_ARG;
  *out = nullptr;
  if (prec != FG_FP64 && prec != FG_MIXED) return FG_E_ARG;
  if (nitems < 1) return FG_E_ARG;
  for (int k = 0; k < 3; ++k)
    if (!(spacing[k] > 0.0) || !std::isfinite(spacing[k])) return FG_E_ARG;
  if (!fg::fft_n0_length_supported(grid[0]) || !fg::fft_n1_length_supported(grid[1])) return FG_E_SIZE;
  if (grid[2] % 2 != 0 || !fg::fft_length_supported(grid[2] / 2) || grid[2] < 4) return FG_E_SIZE;
  fg_plan* P = new (std::nothrow) fg_plan();
  if (!P) return FG_E_HIP;
  P->n0 = grid[0];
  P->n1 = grid[1];
  P->n2 = grid[2];
  P->M = grid[2] / 2;
  P->N = (long)grid[0] * grid[1] * grid[2];
  for (int k = 0; k < 3; ++k) P->h[k] = spacing[k];
  P->nitems = nitems;
  P->prec = prec;
  P->stream = (hipStream_t)stream;
  P->need = layout(P, nullptr) + kAlign;
  if (hipHostMalloc((void**)&P->hks, (nitems + 1) * sizeof(KrylovScalars), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&P->hd, (64 + 16 * nitems) * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&P->hflags, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    plan_delete(P);
    return FG_E_HIP;
  }
  P->hksc = P->hks + nitems;
  *out = P;
  return FG_OK;
}

void need_ready(fg_plan* P, bool need_state) {
  if (P->batch_group) throw Status(FG_E_ARG, "a batch group plan takes only the tile calls");
  P->lin_open = false;  // every solver call reuses the CG workspace
  if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
  if (!P->have_material) throw Status(FG_E_STATE, "material not set");
  if (need_state && !P->F) throw Status(FG_E_STATE, "state not set");
}
}  // namespace

extern "C" {

fg_status fg_plan_create(const int grid[3], const double spacing[3], fg_precision prec, void* stream,
                         fg_plan** out) {
  return plan_new(grid, spacing, prec, stream, 1, out);
}

size_t fg_plan_workspace_bytes(const fg_plan* P) { return P ? P->need : 0; }

static_assert(FG_LAW_NEO_HOOKE == fg::kLawNH && FG_LAW_SVK == fg::kLawSVK, "law codes");

fg_status fg_set_law(fg_plan* P, int law) {
  if (!P || P->batch_group || (law != ::FG_LAW_NEO_HOOKE && law != ::FG_LAW_SVK)) return FG_E_ARG;
  if (P->ws) {
    P->err = "the law must be set before the workspace";
    return FG_E_STATE;
  }
  P->law = law;
  P->need = layout(P, nullptr) + kAlign;
  return FG_OK;
}

fg_status fg_plan_set_workspace(fg_plan* P, void* dev, size_t bytes) {
  if (!P || !dev || P->batch_group) return FG_E_ARG;
  return plan_set_workspace(P, dev, bytes);
}

}  // extern "C"

fg_status plan_set_workspace(fg_plan* P, void* dev, size_t bytes) {
  if (((uintptr_t)dev) % kAlign != 0) {
    P->err = "workspace must be 256-byte aligned";
    return FG_E_ARG;
  }
  if (bytes < P->need) {
    P->err = "workspace too small";
    return FG_E_SIZE;
  }
  return run(P, [&]() {
    P->ws = (char*)dev;
    P->ws_bytes = bytes;
    layout(P, P->ws);
    // tables: built on the host in one blob covering the table region
    const size_t tab_end = (size_t)((char*)P->ks - P->ws);
    std::vector<char> blob(tab_end, 0);
    host_tables<double>(P, blob, P->t64, P->ws);
    host_tables<float>(P, blob, P->t32, P->ws);
    FG_HIP(hipMemcpyAsync(P->ws, blob.data(), tab_end, hipMemcpyHostToDevice, P->stream));
    FG_HIP(hipMemsetAsync(P->ks, 0, (P->nitems + 1) * sizeof(KrylovScalars), P->stream));
    FG_HIP(hipMemsetAsync(P->flags, 0, 4 * sizeof(int), P->stream));
    P->zeroN = (P->nitems == 1) ? P->sc + 15 * P->N : P->sc;
    FG_HIP(hipMemsetAsync(P->zeroN, 0, P->N * P->nitems * sizeof(double), P->stream));
    FG_HIP(hipStreamSynchronize(P->stream));  // the host blob goes out of scope
  });
}

extern "C" {

fg_status fg_set_material(fg_plan* P, const double* E, const double* nu, const double* Omega, const double* D,
                          const double* sigma_max, double gc, double lc, double RT, double c_max) {
  if (!P || !E || !nu || !Omega || P->batch_group) return FG_E_ARG;
  if (!(gc > 0) || !(lc > 0) || !(RT > 0) || !(c_max > 0)) {
    P->err = "gc, lc, RT and c_max must be positive";
    return FG_E_ARG;
  }
  P->E = E;
  P->nu = nu;
  P->Om = Omega;
  P->D = D;
  P->smax = sigma_max;
  P->gc = gc;
  P->lc = lc;
  P->RT = RT;
  P->cmax = c_max;
  P->have_material = true;
  return FG_OK;
}

fg_status fg_set_state(fg_plan* P, double* F, double* c, double* d, double* H) {
  if (!P || !F || P->batch_group) return FG_E_ARG;
  P->F = F;
  P->c = c;
  P->d = d;
  P->H = H;
  return FG_OK;
}

fg_status fg_apply_macro(fg_plan* P, const double F_macro[9]) {
  if (!P || !F_macro) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    apply_macro(P, F_macro);
    FG_HIP(hipStreamSynchronize(P->stream));
  });
}

fg_status fg_newton_solve(fg_plan* P, const double F_macro[9], const fg_solver_opts* opts, fg_stats* stats) {
  if (!P || !F_macro || !opts) return FG_E_ARG;
  if (opts->max_lin <= 0 && opts->fixed_lin <= 0) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    if (stats) std::memset(stats, 0, sizeof(fg_stats));
    apply_macro(P, F_macro);
    newton(P, F_macro, opts, stats);
    FG_HIP(hipStreamSynchronize(P->stream));
  });
}

fg_status fg_newton_solve_shifted(fg_plan* P, const double* B, const fg_solver_opts* opts, fg_stats* stats) {
  if (!P || !B || !opts) return FG_E_ARG;
  if (opts->max_lin <= 0 && opts->fixed_lin <= 0) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    if (stats) std::memset(stats, 0, sizeof(fg_stats));
    newton(P, nullptr, opts, stats, B);
    FG_HIP(hipStreamSynchronize(P->stream));
  });
}

fg_status fg_newton_linear_begin(fg_plan* P, const double F_macro[9], double* err_res) {
  if (!P || !F_macro) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    const double err = newton_residual(P, residual_denominator(P, F_macro));
    // b = -G*P: rho_0 = -U(P), the potential newton_residual left in S64
    if (P->prec == FG_FP64)
      cg_start1<double>(P, P->S64, -1.0, true);
    else
      cg_start1<float>(P, P->S64, -1.0, true);
    sync_read(P);
    if (err_res) *err_res = err;
    P->lin_open = true;
  });
}

fg_status fg_cg_iterate(fg_plan* P, int n, int apply, fg_stats* stats) {
  if (!P || n < 0 || P->batch_group) return FG_E_ARG;
  return run(P, [&]() {
    if (!P->lin_open) throw Status(FG_E_STATE, "no linear system open (fg_newton_linear_begin)");
    // P->hks[0] holds the scalars of the last read-back (every call here
    // ends with one): continue from them for exactly n more iterations
    KrylovScalars& h = P->hks[0];
    if (n > 0 && h.flag != 1 && h.rr0 > 0.0) {
      h.tol2 = 0.0;
      h.maxit = h.iter + n;
      h.done = 0;
      h.flag = 0;
      FG_HIP(hipMemcpyAsync(P->ks, &h, sizeof(KrylovScalars), hipMemcpyHostToDevice, P->stream));
      for (int left = n; left > 0;) {
        const int chunk = std::min(left, 8);
        for (int k = 0; k < chunk; ++k) {
          if (P->prec == FG_FP64)
            cg_iteration<double>(P);
          else
            cg_iteration<float>(P);
        }
        left -= chunk;
        sync_read(P);
        if (P->hks[0].flag == 1) break;
      }
    }
    const KrylovScalars& k = P->hks[0];
    if (stats) {
      stats->lin_iters_last = k.iter;
      stats->lin_relres = k.rr0 > 0 ? std::sqrt(k.rr / k.rr0) : 0.0;
    }
    if (k.flag == 1) throw Status(FG_E_BREAKDOWN, "CG breakdown: p.Ap <= 0");
    if (apply) {
      P->lin_open = false;
      if (P->prec == FG_FP64)
        cg_result<double>(P, P->S64, nullptr);
      else
        cg_result<float>(P, P->S64, nullptr);
      const long n9 = 9 * P->N;
      hipLaunchKernelGGL((k_axpy_into_f64<double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, P->F,
                         (const double*)P->S64, n9);
      check_launch();
      FG_HIP(hipStreamSynchronize(P->stream));
    }
  });
}

fg_status fg_adjoint_gradient(fg_plan* P, const double dL_dPavg[9], double* dL_dlogE, double* dL_dOmega,
                              const fg_solver_opts* opts, fg_stats* stats) {
  if (!P || !dL_dPavg || !opts) return FG_E_ARG;
  if (!dL_dlogE && !dL_dOmega) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    if (stats) std::memset(stats, 0, sizeof(fg_stats));
    if (P->prec == FG_FP64)
      adjoint<double>(P, dL_dPavg, dL_dlogE, dL_dOmega, opts, stats);
    else
      adjoint_mixed(P, dL_dPavg, dL_dlogE, dL_dOmega, opts, stats);
    FG_HIP(hipStreamSynchronize(P->stream));
  });
}

fg_status fg_homogenized_tangent(fg_plan* P, const double W[9], double T_out[9], const fg_solver_opts* opts,
                                 fg_stats* stats) {
  if (!P || !W || !T_out || !opts) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    if (stats) std::memset(stats, 0, sizeof(fg_stats));
    if (P->prec == FG_FP64)
      adjoint<double>(P, W, nullptr, nullptr, opts, stats, T_out);
    else
      adjoint_mixed(P, W, nullptr, nullptr, opts, stats, T_out);
    FG_HIP(hipStreamSynchronize(P->stream));
  });
}

fg_status fg_residual(fg_plan* P, const double F_macro[9], double* err_res) {
  if (!P || !F_macro || !err_res) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    FG_HIP(hipMemcpyAsync(P->Fu, F_macro, 9 * sizeof(double), hipMemcpyHostToDevice, P->stream));
    const unsigned nbN = blocks_for(P->N);
    constitutive(P, P->Fu, P->S64, nullptr, P->part2);
    reduce_to(P, P->part2, (int)nbN, 0);
    residual_norm(P, 1);
    constitutive(P, nullptr, P->S64, nullptr, nullptr);
    residual_norm(P, 2);
    sync_read(P);
    check_domain(P);
    const double den = std::max(std::max(std::sqrt(P->hd[1]), 1e-14 * std::sqrt(P->hd[0])), 1e-300);
    *err_res = std::sqrt(P->hd[2]) / den;
  });
}

fg_status fg_homogenized_stress(fg_plan* P, double P_avg[9]) {
  if (!P || !P_avg) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    constitutive(P, nullptr, P->S64, nullptr, nullptr);
    mean9(P, P->S64);
    sync_read(P);
    check_domain(P);
    for (int k = 0; k < 9; ++k) P_avg[k] = P->hd[8 + k] / (double)P->N;
  });
}

fg_status fg_stress(fg_plan* P, double* Pout) {
  if (!P || !Pout) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    constitutive(P, nullptr, Pout, nullptr, nullptr);
    sync_read(P);
    check_domain(P);
  });
}

fg_status fg_apply_operator(fg_plan* P, const double* x, double* y) {
  if (!P || !x || !y || x == y) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    const long n9 = 9 * P->N;
    const unsigned nbN = blocks_for(P->N);
    if (P->prec == FG_FP64) {
      constitutive(P, nullptr, nullptr, P->st, nullptr);
      launch_contract<double>(P, y, x);
      check_launch();
      C2REpi epi{1.0, nullptr, true, nullptr, Skip{}};
      project9<double>(P, y, y, y, epi);
    } else {
      constitutive(P, nullptr, nullptr, P->st, nullptr);
      float* xf = (float*)P->p;
      float* yf = (float*)P->S;
      hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, xf, x,
                         n9);
      launch_contract<float>(P, yf, (const float*)xf);
      check_launch();
      C2REpi epi{1.0, nullptr, true, nullptr, Skip{}};
      project9<float>(P, yf, yf, yf, epi);
      hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, y,
                         (const float*)yf, n9);
    }
    check_launch();
  });
}

fg_status fg_project(fg_plan* P, const double* x, double* y) {
  if (!P || !x || !y || P->batch_group) return FG_E_ARG;
  return run(P, [&]() {
    if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
    P->lin_open = false;
    C2REpi epi{1.0, nullptr, true, nullptr, Skip{}};
    project9<double>(P, x, P->S64, y, epi);
    check_launch();
  });
}

fg_status fg_project_grad(fg_plan* P, const double* x, double* y) {
  if (!P || !x || !y || P->batch_group) return FG_E_ARG;
  return run(P, [&]() {
    if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
    P->lin_open = false;
    {
      ProfScope ps(P, FG_PASS_R2C);
      launch_r2c<double>(P->M, x, P->S64, 9L * P->n0 * P->n1, P->t64.spec(), Skip{}, P->stream);
    }
    launch_axis_rows<double>(P->n1, P->S64, P->n0, P->M, P->t64.spec(), Skip{}, P->stream, 1, tile_axis<double>(P),
                             nullptr, 0, nullptr, (double*)P->dcb);
    launch_zgrad<double>(P->n0, P->S64, P->n1, P->M, P->t64.spec(), 1.0 / (double)P->N, Skip{}, P->stream, 1,
                         tile_zproj<double>(P), (const double*)P->dcb);
    inv_potential<double>(P, P->S64, Skip{});
    launch_grad_store<double, double>((const double*)P->S64, 3 * P->N, 9 * P->N, y, 9 * P->N, nullptr, P->n0, P->n1,
                                      P->n2, 1, P->h, P->stream);
    check_launch();
  });
}

fg_status fg_fft_r2c(fg_plan* P, double* data, int ncomp) {
  if (!P || !data || ncomp <= 0 || P->batch_group) return FG_E_ARG;
  return run(P, [&]() {
    if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
    P->lin_open = false;
    const SpecTables<double> tb = P->t64.spec();
    fwd_xy<double>(P, data, data, ncomp, Skip{});
    launch_axis<double>(P->n0, false, data, (long)P->n1 * P->M, P->M, (long)P->n0 * P->n1 * P->M, P->M, P->n1,
                        ncomp, tb.tw0, Skip{}, P->stream);
    check_launch();
  });
}

fg_status fg_fft_c2r(fg_plan* P, double* data, int ncomp) {
  if (!P || !data || ncomp <= 0 || P->batch_group) return FG_E_ARG;
  return run(P, [&]() {
    if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
    P->lin_open = false;
    const SpecTables<double> tb = P->t64.spec();
    launch_axis<double>(P->n0, true, data, (long)P->n1 * P->M, P->M, (long)P->n0 * P->n1 * P->M, P->M, P->n1,
                        ncomp, tb.tw0, Skip{}, P->stream);
    C2REpi epi{1.0 / (double)P->N, nullptr, true, nullptr, Skip{}};
    inv_yx<double>(P, data, data, ncomp, epi);
    check_launch();
  });
}

fg_status pff_solve(fg_plan* P, const fg_solver_opts* opts, fg_stats* stats) {
  if (!P || !opts) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    if (stats) std::memset(stats, 0, sizeof(fg_stats));
    pff(P, opts, stats);
    FG_HIP(hipStreamSynchronize(P->stream));
  });
}

fg_status fick_step(fg_plan* P, double dt, const double* cdot_B, const fg_solver_opts* opts, fg_stats* stats) {
  if (!P || !opts || !(dt > 0)) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    if (stats) std::memset(stats, 0, sizeof(fg_stats));
    fick(P, dt, cdot_B, opts, stats);
    FG_HIP(hipStreamSynchronize(P->stream));
  });
}

fg_status fick_step_full(fg_plan* P, double dt, const double* cdot_B, const fg_solver_opts* opts, fg_stats* stats) {
  if (!P || !opts || !(dt > 0)) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    if (stats) std::memset(stats, 0, sizeof(fg_stats));
    fick(P, dt, cdot_B, opts, stats, 1);
    FG_HIP(hipStreamSynchronize(P->stream));
  });
}

fg_status fg_profile_begin(fg_plan* P) {
  if (!P || P->batch_group) return FG_E_ARG;
  return run(P, [&]() {
    FG_HIP(hipStreamSynchronize(P->stream));
    P->prof_on = true;
    for (int k = 0; k < FG_NPASS; ++k) {
      P->prof_used[k] = 0;
      P->prof_noop[k] = 0;
    }
  });
}

fg_status fg_profile_passes(fg_plan* P, unsigned mask) {
  if (!P || P->batch_group || P->prof_on) return FG_E_ARG;
  P->prof_mask = mask;
  return FG_OK;
}

fg_status fg_profile_end(fg_plan* P, double ms[], long launches[]) {
  if (!P || !ms || !launches) return FG_E_ARG;
  return run(P, [&]() {
    P->prof_on = false;
    FG_HIP(hipStreamSynchronize(P->stream));
    for (int k = 0; k < FG_NPASS; ++k) {
      double tot = 0.0;
      for (size_t u = 0; u < P->prof_used[k]; ++u) {
        float t = 0.f;
        FG_HIP(hipEventElapsedTime(&t, P->prof_ev[k][u].first, P->prof_ev[k][u].second));
        tot += t;
      }
      ms[k] = tot;
      launches[k] = (long)P->prof_used[k] - P->prof_noop[k];
      P->prof_used[k] = 0;
      P->prof_noop[k] = 0;
    }
  });
}

const char* fg_status_string(fg_status s) {
  switch (s) {
    case FG_OK: return "ok";
    case FG_E_ARG: return "invalid argument";
    case FG_E_SIZE: return "unsupported size";
    case FG_E_HIP: return "HIP runtime error";
    case FG_E_NOCONV: return "no convergence";
    case FG_E_BREAKDOWN: return "Krylov breakdown";
    case FG_E_DOMAIN: return "domain error";
    case FG_E_STATE: return "plan not ready";
  }
  return "unknown status";
}

const char* fg_last_error(const fg_plan* P) { return P ? P->err.c_str() : "null plan"; }

void fg_plan_destroy(fg_plan* P) {
  if (!P || P->batch_group) return;  // a batch owns its group plans
  plan_delete(P);
}

}  // extern "C"

void plan_delete(fg_plan* P) {
  for (int k = 0; k < FG_NPASS; ++k)
    for (auto& e : P->prof_ev[k]) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  if (P->hks) (void)hipHostFree(P->hks);
  if (P->hd) (void)hipHostFree(P->hd);
  if (P->hflags) (void)hipHostFree(P->hflags);
  delete P;
}

// ------------------------------------------------------------ batched form --
// Many independent (RVE, load case) items, possibly on different grids.
// Items of one grid form a group: one plan whose fields hold all its items
// item-major, so every kernel of the CG and Newton passes covers the whole
// group in one launch, with finished items masked.  Each group runs on a
// stream of its own; one tick advances every item of every group by one step
// (a CG iteration or a Newton step), and a captured graph holds several ticks
// of all groups (forked from and joined into the batch stream).
struct fg_batch {
  int n_rve = 0, n_cases = 0;
  fg_precision prec = FG_FP64;
  hipStream_t user = nullptr;  // caller's stream: inputs are ordered on it
  hipStream_t s0 = nullptr;    // batch stream (fork / join, graph launch)
  hipEvent_t ev_in = nullptr, ev_fork = nullptr;
  struct Group {
    int grid[3];
    double h[3];
    std::vector<std::pair<int, int>> items;  // (rve, case) of each item
    fg_plan* P = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t ev_join = nullptr;
    size_t off = 0, plan_bytes = 0, bytes = 0;
    double *E = nullptr, *nu = nullptr, *Om = nullptr, *c = nullptr, *F = nullptr;
    NewtonCtl* nc = nullptr;
    int* idle = nullptr;
    int* active = nullptr;
  };
  std::vector<Group> groups;
  std::vector<std::pair<int, int>> where;  // (rve, case) -> (group, item)
  std::vector<char> have_mat;              // per RVE
  size_t need = 0;
  char* ws = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_ticks = 0;
  int graph_every = 0;         // newton_every at capture
  int newton_every = 1;        // the Newton step runs in every k-th tick
  std::vector<int> graph_gen;  // tiles_gen of each group at capture
  NewtonCtl* hnc = nullptr;  // pinned, max items of a group
  int* hactive = nullptr;    // pinned, one per group
  std::string err;
};

namespace {

// Items per group: bounded by the grid limits of the N1 pass (9 N0 planes
// per item on grid.y) and the N0 pass (3 rows per item on grid.z).
int max_items_per_group(const int grid[3]) { return std::max(1, 65535 / (9 * grid[0])); }

fg_status batch_run(fg_batch* B, const std::function<void()>& fn) {
  try {
    fn();
    B->err.clear();
    return FG_OK;
  } catch (const Status& s) {
    B->err = s.what();
    return s.code;
  } catch (const HipError& e) {
    B->err = e.what();
    return FG_E_HIP;
  } catch (const std::invalid_argument& e) {
    B->err = e.what();
    return FG_E_SIZE;
  } catch (const std::exception& e) {
    B->err = e.what();
    return FG_E_HIP;
  }
}


// One tick of a group: a CG iteration for the items whose solve runs, then
// the Newton step for the items whose solve has ended.
template <typename T>
void batch_tick(fg_plan* P, fg_batch::Group& g, bool newton) {
  cg_iteration<T>(P);
  if (!newton) return;
  const int nit = P->nitems;
  const long n9 = 9 * P->N;
  const dim3 gi = item_grid(n9, nit);
  hipLaunchKernelGGL(k_newton_gate, dim3(1), dim3(1024), 0, P->stream, (const KrylovScalars*)P->ks, g.nc, g.idle,
                     g.active, nit, (int)FG_E_BREAKDOWN, (int)FG_E_NOCONV);
  // F += D xi, evaluated in double precision (a discrete gradient: compatible
  // to rounding also in the mixed form)
  cg_result<T>(P, P->S64, g.idle);
  hipLaunchKernelGGL((k_items_axpy<double>), gi, dim3(256), 0, P->stream, P->F, (const double*)P->S64,
                     (const int*)g.idle, n9);
  constitutive(P, nullptr, P->S64, P->st, nullptr, g.idle);
  {
    // err_res of eq. (31) from |D U(P)| = |G*P| and the Newton test
    const int nb = residual_pot(P, g.idle);
    hipLaunchKernelGGL(k_newton_check, dim3(nit), dim3(1024), 0, P->stream, (const double*)P->part, nb, g.nc,
                       g.idle, (int)FG_E_NOCONV);
  }
  {
    // b = -G*P: rho_0 = -U(P) (left in S64), xi = 0, and a fresh CG
    const int nb = cg_start<T>(P, P->S64, -1.0, g.idle, true);
    hipLaunchKernelGGL(k_newton_cg_start, dim3(nit), dim3(1024), 0, P->stream, (const double*)P->part, nb, P->ks, g.nc,
                       (const int*)g.idle);
  }
  check_launch();
}

// ticks of every group, forked from s0 and joined back into it
void batch_enqueue(fg_batch* B, int ticks) {
  FG_HIP(hipEventRecord(B->ev_fork, B->s0));
  for (auto& g : B->groups) {
    FG_HIP(hipStreamWaitEvent(g.s, B->ev_fork, 0));
    for (int t = 0; t < ticks; ++t) {
      const bool newton = (t % B->newton_every) == 0;
      if (B->prec == FG_FP64)
        batch_tick<double>(g.P, g, newton);
      else
        batch_tick<float>(g.P, g, newton);
    }
    FG_HIP(hipEventRecord(g.ev_join, g.s));
    FG_HIP(hipStreamWaitEvent(B->s0, g.ev_join, 0));
  }
}

void batch_capture(fg_batch* B, int ticks) {
  std::vector<int> gen;
  for (auto& g : B->groups) gen.push_back(g.P->tiles_gen);
  if (B->exec && B->graph_ticks == ticks && B->graph_every == B->newton_every && gen == B->graph_gen) return;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  FG_HIP(hipStreamBeginCapture(B->s0, hipStreamCaptureModeThreadLocal));
  try {
    batch_enqueue(B, ticks);
  } catch (...) {
    hipGraph_t tmp = nullptr;
    (void)hipStreamEndCapture(B->s0, &tmp);
    if (tmp) (void)hipGraphDestroy(tmp);
    throw;
  }
  FG_HIP(hipStreamEndCapture(B->s0, &B->graph));
  FG_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  B->graph_ticks = ticks;
  B->graph_every = B->newton_every;
  B->graph_gen = gen;
}

// Start of the solve for a group: F = F_macro of the item's load case
// (uniform), the normaliser of eq. (31) per item, Newton and CG control.
void batch_prologue(fg_batch* B, fg_batch::Group& g, const double* F_macro, const fg_solver_opts* o) {
  fg_plan* P = g.P;
  const int nit = P->nitems;
  const long N = P->N;
  for (int b = 0; b < nit; ++b)
    for (int k = 0; k < 9; ++k) P->hd[64 + 9 * b + k] = F_macro[9 * g.items[b].second + k];
  FG_HIP(hipMemcpyAsync(P->Fu, P->hd + 64, 9 * nit * sizeof(double), hipMemcpyHostToDevice, P->stream));
  hipLaunchKernelGGL((k_fill<double>), dim3(grid_stride_blocks(9 * N * nit)), dim3(256), 0, P->stream, P->F, 0.0,
                     9 * N * nit);
  hipLaunchKernelGGL(k_add_uniform9, dim3(blocks_for(N * nit)), dim3(256), 0, P->stream, P->F,
                     (const double*)P->Fu, N, N * nit);
  hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(64), 0, P->stream, P->flags, 0, 4L);
  check_launch();
  // ||P(Fbar)||^2 and ||G*P(Fbar)||^2 per item
  constitutive(P, P->Fu, P->S64, nullptr, P->part2);
  reduce_items(P, P->part2, (int)blocks_for(N), 0);
  reduce_items(P, P->part, residual_pot(P, nullptr), 1);
  sync_read(P);
  check_domain(P);
  const bool mixed = (P->prec == FG_MIXED);
  fg_solver_opts om = *o;
  if (mixed && om.fixed_lin <= 0) om.tol_lin = std::max(o->tol_lin, 1e-5);
  for (int b = 0; b < nit; ++b) {
    NewtonCtl& c = B->hnc[b];
    std::memset(&c, 0, sizeof(NewtonCtl));
    const double p2 = item_value(P, 0, b), gp2 = item_value(P, 1, b);
    c.den = std::max(std::max(std::sqrt(gp2), 1e-14 * std::sqrt(p2)), 1e-300);
    c.tol = mixed ? 0.01 * o->tol_newton : o->tol_newton;
    c.max_newton = o->max_newton;
    c.mixed = mixed ? 1 : 0;
    KrylovScalars& k = P->hks[b];
    std::memset(&k, 0, sizeof(KrylovScalars));
    k.done = 1;  // the first tick starts with the Newton step
    k.tol2 = (om.fixed_lin > 0) ? 0.0 : om.tol_lin * om.tol_lin;
    k.maxit = (om.fixed_lin > 0) ? om.fixed_lin : om.max_lin;
  }
  FG_HIP(hipMemcpyAsync(g.nc, B->hnc, nit * sizeof(NewtonCtl), hipMemcpyHostToDevice, P->stream));
  FG_HIP(hipMemcpyAsync(P->ks, P->hks, nit * sizeof(KrylovScalars), hipMemcpyHostToDevice, P->stream));
  const long n9 = 9 * N * nit;
  if (P->prec == FG_FP64)
    hipLaunchKernelGGL((k_fill<double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, (double*)P->x, 0.0,
                       n9);
  else
    hipLaunchKernelGGL((k_fill<float>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, (float*)P->x, 0.0f,
                       n9);
  check_launch();
  FG_HIP(hipStreamSynchronize(P->stream));  // pinned control blocks are reused
}

// <P> and statistics of a group after the solve; returns the first failure.
void batch_epilogue(fg_batch* B, fg_batch::Group& g, double* P_avg, fg_stats* stats, fg_status& first,
                    std::string& first_msg) {
  fg_plan* P = g.P;
  const int nit = P->nitems;
  const long N = P->N;
  constitutive(P, nullptr, P->S64, nullptr, nullptr);
  const unsigned nb = blocks_for(N);
  hipLaunchKernelGGL(k_mean9_partials, dim3(nb, (unsigned)nit), dim3(256), 0, P->stream, (const double*)P->S64,
                     P->part2, N);
  check_launch();
  for (int k = 0; k < 9; ++k) reduce_items(P, P->part2 + (size_t)k * nit * nb, (int)nb, k);
  FG_HIP(hipMemcpyAsync(B->hnc, g.nc, nit * sizeof(NewtonCtl), hipMemcpyDeviceToHost, P->stream));
  sync_read(P);
  const bool domain = P->hflags[0] & FG_FLAG_DOMAIN;
  for (int b = 0; b < nit; ++b) {
    const int rve = g.items[b].first, lc = g.items[b].second;
    const long idx = (long)rve * B->n_cases + lc;
    if (P_avg)
      for (int k = 0; k < 9; ++k) P_avg[9 * idx + k] = item_value(P, k, b) / (double)N;
    const NewtonCtl& c = B->hnc[b];
    const KrylovScalars& h = P->hks[b];
    if (stats) {
      fg_stats& s = stats[idx];
      std::memset(&s, 0, sizeof(fg_stats));
      s.newton_iters = c.it;
      s.lin_iters_total = c.lin_total;
      s.lin_iters_last = c.lin_last;
      s.n_history = c.n_hist;
      s.err_res = c.err;
      s.lin_relres = h.rr0 > 0 ? std::sqrt(h.rr / h.rr0) : 0.0;
      for (int k = 0; k < std::min(c.n_hist, FG_NHIST); ++k) s.err_history[k] = c.err_hist[k];
      for (int k = 0; k < std::min(c.it, FG_NHIST); ++k) s.lin_history[k] = c.lin_hist[k];
    }
    fg_status st = (fg_status)c.status;
    if (st == FG_OK && !c.finished) st = FG_E_NOCONV;
    if (st != FG_OK && first == FG_OK) {
      first = st;
      first_msg = "item (rve " + std::to_string(rve) + ", case " + std::to_string(lc) + "): " +
                  (st == FG_E_BREAKDOWN ? "CG breakdown" : "Newton did not converge");
    }
  }
  if (domain && first == FG_OK) {
    first = FG_E_DOMAIN;
    first_msg = "det F <= 0 or 1 + Omega c <= 0 in a batch item";
  }
}

void batch_destroy_parts(fg_batch* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  for (auto& g : B->groups) {
    if (g.P) plan_delete(g.P);
    if (g.ev_join) (void)hipEventDestroy(g.ev_join);
    if (g.s) (void)hipStreamDestroy(g.s);
  }
  if (B->ev_in) (void)hipEventDestroy(B->ev_in);
  if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
  if (B->s0) (void)hipStreamDestroy(B->s0);
  if (B->hnc) (void)hipHostFree(B->hnc);
  if (B->hactive) (void)hipHostFree(B->hactive);
}

}  // namespace

extern "C" {

fg_status fg_batch_create(int n_rve, const int* grids, const double* spacings, int n_cases, fg_precision prec,
                          void* stream, fg_batch** out) {
  if (!out) return FG_E_ARG;
  *out = nullptr;
  if (n_rve < 1 || n_cases < 1 || !grids || !spacings) return FG_E_ARG;
  if (prec != FG_FP64 && prec != FG_MIXED) return FG_E_ARG;
  fg_batch* B = new (std::nothrow) fg_batch();
  if (!B) return FG_E_HIP;
  B->n_rve = n_rve;
  B->n_cases = n_cases;
  B->prec = prec;
  B->user = (hipStream_t)stream;
  B->where.assign((size_t)n_rve * n_cases, {-1, -1});
  B->have_mat.assign(n_rve, 0);
  // group the items by grid and spacing, in RVE order
  for (int r = 0; r < n_rve; ++r) {
    const int* gr = grids + 3 * r;
    const double* sp = spacings + 3 * r;
    for (int lc = 0; lc < n_cases; ++lc) {
      int gidx = -1;
      for (size_t k = 0; k < B->groups.size(); ++k) {
        const auto& g = B->groups[k];
        if (g.grid[0] == gr[0] && g.grid[1] == gr[1] && g.grid[2] == gr[2] && g.h[0] == sp[0] && g.h[1] == sp[1] &&
            g.h[2] == sp[2] && (int)g.items.size() < max_items_per_group(gr))
          gidx = (int)k;
      }
      if (gidx < 0) {
        fg_batch::Group g;
        for (int k = 0; k < 3; ++k) {
          g.grid[k] = gr[k];
          g.h[k] = sp[k];
        }
        B->groups.push_back(g);
        gidx = (int)B->groups.size() - 1;
      }
      auto& g = B->groups[gidx];
      B->where[(size_t)r * n_cases + lc] = {gidx, (int)g.items.size()};
      g.items.push_back({r, lc});
    }
  }
  fg_status st = FG_OK;
  int max_items = 1;
  for (auto& g : B->groups) {
    st = plan_new(g.grid, g.h, prec, nullptr, (int)g.items.size(), &g.P);
    if (st != FG_OK) break;
    if (hipStreamCreateWithFlags(&g.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g.ev_join, hipEventDisableTiming) != hipSuccess) {
      st = FG_E_HIP;
      break;
    }
    g.P->stream = g.s;
    g.P->batch_group = true;
    max_items = std::max(max_items, (int)g.items.size());
  }
  if (st == FG_OK && (hipStreamCreateWithFlags(&B->s0, hipStreamNonBlocking) != hipSuccess ||
                      hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess ||
                      hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming) != hipSuccess ||
                      hipHostMalloc((void**)&B->hnc, max_items * sizeof(NewtonCtl), hipHostMallocDefault) !=
                          hipSuccess ||
                      hipHostMalloc((void**)&B->hactive, B->groups.size() * sizeof(int), hipHostMallocDefault) !=
                          hipSuccess))
    st = FG_E_HIP;
  if (st != FG_OK) {
    batch_destroy_parts(B);
    delete B;
    return st;
  }
  // workspace: per group the plan workspace, then E, nu, Omega, c (N each
  // per item), F (9 N per item), the Newton control blocks and flags
  size_t off = 0;
  for (auto& g : B->groups) {
    const long NT = g.P->N * g.P->nitems;
    g.off = off;
    g.plan_bytes = align_up(g.P->need);
    size_t b = g.plan_bytes;
    b += align_up(4 * NT * sizeof(double));
    b += align_up(9 * NT * sizeof(double));
    b += align_up(g.items.size() * sizeof(NewtonCtl));
    b += align_up((g.items.size() + 64) * sizeof(int));
    g.bytes = b;
    off += b;
  }
  B->need = off + kAlign;
  *out = B;
  return FG_OK;
}

size_t fg_batch_workspace_bytes(const fg_batch* B) { return B ? B->need : 0; }

int fg_batch_groups(const fg_batch* B) { return B ? (int)B->groups.size() : 0; }

fg_status fg_batch_set_workspace(fg_batch* B, void* dev, size_t bytes) {
  if (!B || !dev) return FG_E_ARG;
  if (((uintptr_t)dev) % kAlign != 0) {
    B->err = "workspace must be 256-byte aligned";
    return FG_E_ARG;
  }
  if (bytes < B->need) {
    B->err = "workspace too small";
    return FG_E_SIZE;
  }
  return batch_run(B, [&]() {
    B->ws = (char*)dev;
    for (auto& g : B->groups) {
      char* base = B->ws + g.off;
      const fg_status st = plan_set_workspace(g.P, base, g.plan_bytes);
      if (st != FG_OK) throw Status(st, std::string("group workspace: ") + fg_last_error(g.P));
      const long NT = g.P->N * g.P->nitems;
      size_t o = g.plan_bytes;
      g.E = reinterpret_cast<double*>(base + o);
      g.nu = g.E + NT;
      g.Om = g.nu + NT;
      g.c = g.Om + NT;
      o += align_up(4 * NT * sizeof(double));
      g.F = reinterpret_cast<double*>(base + o);
      o += align_up(9 * NT * sizeof(double));
      g.nc = reinterpret_cast<NewtonCtl*>(base + o);
      o += align_up(g.items.size() * sizeof(NewtonCtl));
      g.idle = reinterpret_cast<int*>(base + o);
      g.active = g.idle + g.items.size();
      FG_HIP(hipMemsetAsync(g.c, 0, NT * sizeof(double), g.s));
      FG_HIP(hipMemsetAsync(g.idle, 0, (g.items.size() + 64) * sizeof(int), g.s));
      g.P->E = g.E;
      g.P->nu = g.nu;
      g.P->Om = g.Om;
      g.P->c = g.c;
      g.P->F = g.F;
      g.P->gc = g.P->lc = g.P->RT = g.P->cmax = 1.0;
      g.P->have_material = true;
      FG_HIP(hipStreamSynchronize(g.s));
    }
    // a new workspace invalidates a captured graph
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->graph_ticks = 0;
  });
}

fg_status fg_batch_set_material(fg_batch* B, int rve, const double* E, const double* nu, const double* Omega,
                                const double* c) {
  if (!B || !E || !nu || !Omega || rve < 0 || rve >= B->n_rve) return FG_E_ARG;
  return batch_run(B, [&]() {
    if (!B->ws) throw Status(FG_E_STATE, "workspace not set");
    FG_HIP(hipEventRecord(B->ev_in, B->user));
    for (int lc = 0; lc < B->n_cases; ++lc) {
      const auto w = B->where[(size_t)rve * B->n_cases + lc];
      auto& g = B->groups[w.first];
      const long N = g.P->N;
      const size_t nb = N * sizeof(double);
      FG_HIP(hipStreamWaitEvent(g.s, B->ev_in, 0));
      FG_HIP(hipMemcpyAsync(g.E + w.second * N, E, nb, hipMemcpyDeviceToDevice, g.s));
      FG_HIP(hipMemcpyAsync(g.nu + w.second * N, nu, nb, hipMemcpyDeviceToDevice, g.s));
      FG_HIP(hipMemcpyAsync(g.Om + w.second * N, Omega, nb, hipMemcpyDeviceToDevice, g.s));
      if (c)
        FG_HIP(hipMemcpyAsync(g.c + w.second * N, c, nb, hipMemcpyDeviceToDevice, g.s));
      else
        FG_HIP(hipMemsetAsync(g.c + w.second * N, 0, nb, g.s));
      FG_HIP(hipStreamSynchronize(g.s));  // the caller may free or reuse its buffers
    }
    B->have_mat[rve] = 1;
  });
}

fg_status fg_batch_newton_solve(fg_batch* B, const double* F_macro, const fg_solver_opts* opts, int graph_ticks,
                                double* P_avg, fg_stats* stats) {
  if (!B || !F_macro || !opts) return FG_E_ARG;
  if (opts->max_lin <= 0 && opts->fixed_lin <= 0) return FG_E_ARG;
  if (graph_ticks < 0) return FG_E_ARG;
  if (graph_ticks > 0 && graph_ticks % B->newton_every != 0) {
    B->err = "graph_ticks must be a multiple of the Newton schedule (fg_batch_set_schedule)";
    return FG_E_ARG;
  }
  return batch_run(B, [&]() {
    if (!B->ws) throw Status(FG_E_STATE, "workspace not set");
    for (int r = 0; r < B->n_rve; ++r)
      if (!B->have_mat[r]) throw Status(FG_E_STATE, "material not set for every RVE");
    FG_HIP(hipEventRecord(B->ev_in, B->user));
    for (auto& g : B->groups) {
      FG_HIP(hipStreamWaitEvent(g.s, B->ev_in, 0));
      batch_prologue(B, g, F_macro, opts);
    }
    const int maxit = (opts->fixed_lin > 0) ? opts->fixed_lin : opts->max_lin;
    const int k = B->newton_every;
    // every Newton step takes at most maxit CG ticks, then waits at most k
    // ticks for a tick with the Newton step
    const long cap = (long)(opts->max_newton + 1) * (maxit + k) + 2 * k;
    const int per = graph_ticks > 0 ? graph_ticks : 8 * k;
    if (graph_ticks > 0) batch_capture(B, graph_ticks);
    for (long ticks = 0; ticks < cap; ticks += per) {
      if (graph_ticks > 0)
        FG_HIP(hipGraphLaunch(B->exec, B->s0));
      else
        batch_enqueue(B, per);
      for (size_t k = 0; k < B->groups.size(); ++k)
        FG_HIP(hipMemcpyAsync(B->hactive + k, B->groups[k].active, sizeof(int), hipMemcpyDeviceToHost, B->s0));
      FG_HIP(hipStreamSynchronize(B->s0));
      int act = 0;
      for (size_t k = 0; k < B->groups.size(); ++k) act += B->hactive[k];
      if (act == 0) break;
    }
    fg_status first = FG_OK;
    std::string msg;
    for (auto& g : B->groups) batch_epilogue(B, g, P_avg, stats, first, msg);
    if (first != FG_OK) throw Status(first, msg);
  });
}

fg_status fg_batch_state(fg_batch* B, int rve, int lcase, double* F) {
  if (!B || !F || rve < 0 || rve >= B->n_rve || lcase < 0 || lcase >= B->n_cases) return FG_E_ARG;
  return batch_run(B, [&]() {
    if (!B->ws) throw Status(FG_E_STATE, "workspace not set");
    const auto w = B->where[(size_t)rve * B->n_cases + lcase];
    auto& g = B->groups[w.first];
    const long n9 = 9 * g.P->N;
    FG_HIP(hipMemcpyAsync(F, g.F + w.second * n9, n9 * sizeof(double), hipMemcpyDeviceToDevice, g.s));
    FG_HIP(hipStreamSynchronize(g.s));
  });
}

fg_status fg_batch_set_schedule(fg_batch* B, int newton_every) {
  if (!B || newton_every < 1 || newton_every > 64) return FG_E_ARG;
  B->newton_every = newton_every;
  return FG_OK;
}

fg_plan* fg_batch_plan(fg_batch* B, int group) {
  if (!B || group < 0 || group >= (int)B->groups.size()) return nullptr;
  return B->groups[group].P;
}

int fg_batch_group_info(const fg_batch* B, int group, int grid[3], int* nitems) {
  if (!B || group < 0 || group >= (int)B->groups.size()) return -1;
  const auto& g = B->groups[group];
  if (grid)
    for (int k = 0; k < 3; ++k) grid[k] = g.grid[k];
  if (nitems) *nitems = (int)g.items.size();
  return 0;
}

const char* fg_batch_last_error(const fg_batch* B) { return B ? B->err.c_str() : "null batch"; }

void fg_batch_destroy(fg_batch* B) {
  if (!B) return;
  batch_destroy_parts(B);
  delete B;
}

}  // extern "C"

// ------------------------------------------------------------ tile tuning --
namespace {
struct TilePass {
  bool zproj;
  int elem;  // bytes of one complex value
};
TilePass tile_pass(int which) { return TilePass{(which & 1) != 0, (which < 2) ? 16 : 8}; }
int tile_len(const fg_plan* P, int which) { return (which & 1) ? P->n0 : P->n1; }

template <typename R>
void time_pass_impl(fg_plan* P, bool zproj, int tile, int reps, double* ms) {
  R* S = (sizeof(R) == 8) ? (R*)P->S64 : (R*)P->S;
  const long n = 9 * P->N * P->nitems;
  hipLaunchKernelGGL((k_fill<R>), dim3(grid_stride_blocks(n)), dim3(256), 0, P->stream, S, (R)1e-3, n);
  check_launch();
  const SpecTables<R> tb = tabs<R>(P).spec();
  auto launch = [&]() {
    if (zproj) {
      launch_zgrad<R>(P->n0, S, P->n1, P->M, tb, (R)(1.0 / (double)P->N), Skip{}, P->stream, P->nitems, tile);
    } else {
      // the N1 work of a CG iteration: the forward row pass and the inverse
      // pass of the potential
      launch_axis_rows<R>(P->n1, S, P->n0, P->M, tb, Skip{}, P->stream, P->nitems, tile);
      launch_axis<R>(P->n1, true, S, P->M, (long)P->n1 * P->M, 3L * P->n0 * P->n1 * P->M, P->M, P->n0,
                     3 * P->nitems, tb.tw1, Skip{}, P->stream, tile);
    }
  };
  hipEvent_t e0, e1;
  FG_HIP(hipEventCreate(&e0));
  FG_HIP(hipEventCreate(&e1));
  try {
    launch();  // warm-up
    FG_HIP(hipEventRecord(e0, P->stream));
    for (int k = 0; k < reps; ++k) launch();
    FG_HIP(hipEventRecord(e1, P->stream));
    check_launch();
    FG_HIP(hipEventSynchronize(e1));
    float el = 0.f;
    FG_HIP(hipEventElapsedTime(&el, e0, e1));
    *ms = (double)el / reps;
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}
}  // namespace

extern "C" {

int fg_plan_tile_candidates(const fg_plan* P, int which, int* out, int cap) {
  if (!P || which < 0 || which > 3 || (cap > 0 && !out)) return -1;
  const TilePass tp = tile_pass(which);
  int n = 0;
  // variants: the projection passes in both workgroup orders; the
  // single-precision N1 pass with one or two columns per thread
  const int flag = tp.zproj ? fg::kTileKyMajor : (tp.elem == 8 ? fg::kTileColumnPairs : 0);
  for (int variant = 0; variant < (flag ? 2 : 1); ++variant)
    for (int b = 1; b <= 512; b *= 2)
      if (fg::tile_valid(tp.zproj, tile_len(P, which), P->M, tp.elem, b | (variant ? flag : 0))) {
        if (n < cap) out[n] = b | (variant ? flag : 0);
        ++n;
      }
  return n;
}

fg_status fg_plan_set_tiles(fg_plan* P, const int tiles[4]) {
  if (!P || !tiles) return FG_E_ARG;
  for (int w = 0; w < 4; ++w) {
    const TilePass tp = tile_pass(w);
    if (tiles[w] != 0 && !fg::tile_valid(tp.zproj, tile_len(P, w), P->M, tp.elem, tiles[w])) {
      P->err = "tile width " + std::to_string(tiles[w]) + " not valid for pass " + std::to_string(w);
      return FG_E_ARG;
    }
  }
  for (int w = 0; w < 4; ++w) P->tiles[w] = tiles[w];
  P->tiles_gen += 1;
  return FG_OK;
}

fg_status fg_plan_get_tiles(const fg_plan* P, int tiles[4]) {
  if (!P || !tiles) return FG_E_ARG;
  for (int w = 0; w < 4; ++w) {
    const TilePass tp = tile_pass(w);
    const int L = tile_len(P, w);
    const int T = tp.zproj ? fg::zgrad_threads(L, tp.elem) : fg::line_threads(L);
    const int built_in = tp.zproj ? (fg::zgrad_tile(L, P->M, tp.elem) | fg::kTileKyMajor)
                                  : fg::column_tile_t(T, L, P->M, tp.elem);
    tiles[w] = P->tiles[w] > 0 ? P->tiles[w] : built_in;
  }
  return FG_OK;
}

fg_status fg_plan_time_pass(fg_plan* P, int which, int tile, int reps, double* ms) {
  if (!P || which < 0 || which > 3 || reps < 1 || !ms) return FG_E_ARG;
  const TilePass tp = tile_pass(which);
  if (tile != 0 && !fg::tile_valid(tp.zproj, tile_len(P, which), P->M, tp.elem, tile)) return FG_E_ARG;
  if (which >= 2 && P->prec != FG_MIXED) return FG_E_ARG;  // single-precision passes exist in mixed plans only
  return run(P, [&]() {
    if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
    P->lin_open = false;
    if (which < 2)
      time_pass_impl<double>(P, tp.zproj, tile, reps, ms);
    else
      time_pass_impl<float>(P, tp.zproj, tile, reps, ms);
  });
}

}  // extern "C"

// --------------------------------------------- allocation-free projection --
// fg_project_noalloc: the compatibility projection of fg_project without a
// plan or workspace.  Its transform tables and spectral work buffer live in
// `scratch`, a fixed array in the library's code object on every device (held
// until the process ends).  In host code `scratch` names only a host-side
// stand-in: its device address on the current device comes from
// hipGetSymbolAddress, taken once per device and kept in g_scratch_dev[],
// and only that address is ever handed to kernels.
constexpr size_t kScratchTableBytes = 64 * 1024;                // transform and symbol tables
constexpr size_t kScratchWorkBytes = 64ull * 1024 * 1024;       // 9 N doubles of spectrum
static __device__ __align__(256) char scratch[kScratchTableBytes + kScratchWorkBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (nullptr on failure).
void* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

// The tables of host_tables<double>, computed on the device (sincospi in
// double instead of long double rounded once: the entries agree to an ulp,
// with the same exact values at the quarter and half angles).
__global__ void __launch_bounds__(256) k_tables_f64(TablesDev<double> t, int n0, int n1, int n2, double h0, double h1,
                                                    double h2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int M = n2 / 2;
  auto root = [&](int L, cplx<double>* w) {
    if (j >= L) return;
    double sv, cv;
    sincospi(2.0 * (double)j / (double)L, &sv, &cv);
    cplx<double> r{cv, -sv};
    if (4 * j == L) r = cplx<double>{0.0, -1.0};
    if (2 * j == L) r = cplx<double>{-1.0, 0.0};
    if (4 * j == 3 * L) r = cplx<double>{0.0, 1.0};
    if (j == 0) r = cplx<double>{1.0, 0.0};
    w[j] = r;
  };
  root(n0, t.tw0);
  root(n1, t.tw1);
  root(M, t.twM);
  if (j < M) {
    double sv, cv;
    sincospi(2.0 * (double)j / (double)n2, &sv, &cv);
    cplx<double> r{cv, -sv};
    if (j == 0) r = cplx<double>{1.0, 0.0};
    if (4 * j == n2) r = cplx<double>{0.0, -1.0};
    t.post[j] = r;
  }
  auto half = [&](int n, int count, double h, double* c, double* sc, double* sn) {
    if (j >= count) return;
    double sv, cv;
    sincospi((double)j / (double)n, &sv, &cv);
    if (j == 0) sv = 0.0;
    if (2 * j == n) {
      cv = 0.0;
      sv = 1.0;
    }
    c[j] = cv;
    sc[j] = (2.0 / h) * sv;
    sn[j] = sv;
  };
  half(n0, n0, h0, t.cz, t.sz, t.snz);
  half(n1, n1, h1, t.cy, t.sy, t.sny);
  half(n2, M + 1, h2, t.cx, t.sx, t.snx);
}

}  // namespace

extern "C" {

fg_status fg_project_noalloc(const int grid[3], const double spacing[3], const double* x, double* y, void* stream) {
  if (!grid || !spacing || !x || !y) return FG_E_ARG;
  for (int k = 0; k < 3; ++k)
    if (!(spacing[k] > 0.0) || !std::isfinite(spacing[k])) return FG_E_ARG;
  if (!fg::fft_n0_length_supported(grid[0]) || !fg::fft_n1_length_supported(grid[1])) return FG_E_SIZE;
  if (grid[2] % 2 != 0 || grid[2] < 4 || !fg::fft_length_supported(grid[2] / 2)) return FG_E_SIZE;
  const long N = (long)grid[0] * grid[1] * grid[2];
  if ((size_t)N * 9 * sizeof(double) > kScratchWorkBytes) return FG_E_SIZE;
  char* base = (char*)scratch_on_current_device();
  if (!base) return FG_E_HIP;
  try {
    fg_plan P;  // a view of the grid only: no workspace, no pinned memory
    P.n0 = grid[0];
    P.n1 = grid[1];
    P.n2 = grid[2];
    P.M = grid[2] / 2;
    P.N = N;
    for (int k = 0; k < 3; ++k) P.h[k] = spacing[k];
    P.prec = FG_FP64;
    P.stream = (hipStream_t)stream;
    size_t off = 0;
    TablesDev<double>& t = P.t64;
    t.tw0 = carve<cplx<double>>(base, off, P.n0);
    t.tw1 = carve<cplx<double>>(base, off, P.n1);
    t.twM = carve<cplx<double>>(base, off, P.M);
    t.post = carve<cplx<double>>(base, off, P.M);
    t.cz = carve<double>(base, off, P.n0);
    t.sz = carve<double>(base, off, P.n0);
    t.cy = carve<double>(base, off, P.n1);
    t.sy = carve<double>(base, off, P.n1);
    t.cx = carve<double>(base, off, P.M + 1);
    t.sx = carve<double>(base, off, P.M + 1);
    t.snz = carve<double>(base, off, P.n0);
    t.sny = carve<double>(base, off, P.n1);
    t.snx = carve<double>(base, off, P.M + 1);
    if (off > kScratchTableBytes) return FG_E_SIZE;
    P.S64 = (double*)(base + kScratchTableBytes);
    const int nt = std::max(std::max(P.n0, P.n1), P.M + 1);
    hipLaunchKernelGGL(k_tables_f64, dim3((nt + 255) / 256), dim3(256), 0, P.stream, t, P.n0, P.n1, P.n2, P.h[0],
                       P.h[1], P.h[2]);
    C2REpi epi{1.0, nullptr, true, nullptr, Skip{}};
    project9<double>(&P, x, P.S64, y, epi);
    return hipGetLastError() == hipSuccess ? FG_OK : FG_E_HIP;
  } catch (...) {
    return FG_E_HIP;
  }
}

}  // extern "C"
