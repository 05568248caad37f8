// Plan, workspace, tables and the solver drivers behind the C ABI of
// include/fgfft.h.  All device work is issued on the plan's stream; the
// only host synchronisations are the scalar read-backs of convergence tests.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fgfft.h"
#include "fg_launch.hpp"
#include "fg_pointwise.hpp"
#include "fg_scalar.hpp"
#include "fg_cgfront.hpp"
#include "fg_fft3.hpp"

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
    default: return 1;
  }
}

int column_tile_t(int T, int L, int M, int elem_bytes) {
  int B = 1;
  while ((M % (2 * B)) == 0 && T * 2 * B <= 256 && (long)L * 2 * B * elem_bytes <= 65536) B *= 2;
  return B;
}

int column_tile(int L, int M, int elem_bytes) { return column_tile_t(line_threads(L), L, M, elem_bytes); }

int zline_threads(int L) {
  if (L == 256) return Line3<256>::T;
  if (L == 128) return Line3<128>::T;
  return line_threads(L);
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
  SpecTables<R> spec() const { return SpecTables<R>{tw0, tw1, twM, post, cz, sz, cy, sy, cx, sx}; }
};

}  // namespace

struct fg_plan {
  int n0, n1, n2, M;
  long N;
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
  KrylovScalars* ks = nullptr;   // [0] mechanics CG, [1] scalar PCG
  int* flags = nullptr;          // [0] domain
  double* dscal = nullptr;       // small FP64 scalars (norms), 64 entries
  double* part = nullptr;        // partial sums
  double* part2 = nullptr;
  double* Fu = nullptr;          // uniform tensor (9)
  double* S64 = nullptr;         // 9N doubles: stress / FP64 spectra
  void* S = nullptr;             // 9N T (aliases S64 in FP64 plans)
  void* x = nullptr;             // 9N T
  void* r = nullptr;             // 9N T
  void* p = nullptr;             // 9N T
  void* st = nullptr;            // 12N T tangent state
  double* sc = nullptr;          // scalar solver area, 16N doubles
  size_t part_n = 0;

  // material (caller-owned)
  const double *E = nullptr, *nu = nullptr, *Om = nullptr, *D = nullptr, *smax = nullptr;
  double gc = 0, lc = 0, RT = 0, cmax = 1;
  bool have_material = false;
  // state (caller-owned)
  double *F = nullptr, *c = nullptr, *d = nullptr, *H = nullptr;
  double* zeroN = nullptr;  // N zeros (c, d when not given) inside the scalar area

  // optional per-kernel-class timing with HIP events (fg_profile_*)
  bool prof_on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[FG_NPASS];
  size_t prof_used[FG_NPASS] = {};
  long prof_noop[FG_NPASS] = {};

  // pinned host scalars
  KrylovScalars* hks = nullptr;
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
  };
  tabs(P->t64, double());
  tabs(P->t32, float());
  P->ks = carve<KrylovScalars>(base, off, 2);
  P->flags = carve<int>(base, off, 4);
  P->dscal = carve<double>(base, off, 64);
  P->Fu = carve<double>(base, off, 16);
  P->part_n = (size_t)9 * (N / 256 + 2) + 8192;
  P->part = carve<double>(base, off, P->part_n);
  P->part2 = carve<double>(base, off, P->part_n);
  const size_t tb = (P->prec == FG_FP64) ? sizeof(double) : sizeof(float);
  P->S64 = carve<double>(base, off, 9 * N);
  if (P->prec == FG_FP64) {
    P->S = P->S64;
  } else {
    P->S = carve<char>(base, off, 9 * N * tb);
  }
  P->x = carve<char>(base, off, 9 * N * tb);
  P->r = carve<char>(base, off, 9 * N * tb);
  P->p = carve<char>(base, off, 9 * N * tb);
  P->st = carve<char>(base, off, 12 * N * tb);
  P->sc = carve<double>(base, off, 16 * N);
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
  auto half = [&](int n, int count, double h, void* cptr, void* sptr) {
    std::vector<R> cc(count), ss(count);
    for (int m = 0; m < count; ++m) {
      const long double a = PI * (long double)m / (long double)n;
      long double cv = std::cos(a), sv = std::sin(a);
      if (m == 0) sv = 0.0L;
      if (2 * m == n) cv = 0.0L;  // exact zero at q = pi
      cc[m] = (R)cv;
      ss[m] = (R)((2.0L / (long double)h) * sv);
    }
    put(cptr, cc.data(), count * sizeof(R));
    put(sptr, ss.data(), count * sizeof(R));
  };
  half(P->n0, P->n0, P->h[0], dev.cz, dev.sz);
  half(P->n1, P->n1, P->h[1], dev.cy, dev.sy);
  half(P->n2, P->M + 1, P->h[2], dev.cx, dev.sx);
}

// Event pair around one launch of kernel class `pass` (no-op unless on).
struct ProfScope {
  fg_plan* P;
  int pass;
  hipEvent_t stop = nullptr;
  ProfScope(fg_plan* P_, int pass_) : P(P_), pass(pass_) {
    if (!P->prof_on) return;
    auto& v = P->prof_ev[pass];
    size_t& u = P->prof_used[pass];
    if (u == v.size()) {
      hipEvent_t a, b;
      FG_HIP(hipEventCreate(&a));
      FG_HIP(hipEventCreate(&b));
      v.emplace_back(a, b);
    }
    FG_HIP(hipEventRecord(v[u].first, P->stream));
    stop = v[u].second;
    ++u;
  }
  ~ProfScope() {
    if (stop) (void)hipEventRecord(stop, P->stream);
  }
};

inline unsigned blocks_for(long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }
inline unsigned grid_stride_blocks(long n) { return (unsigned)std::min<long>(2048, (n + 255) / 256); }

void check_launch() { FG_HIP(hipGetLastError()); }

void sync_read(fg_plan* P) {
  FG_HIP(hipMemcpyAsync(P->hks, P->ks, 2 * sizeof(KrylovScalars), hipMemcpyDeviceToHost, P->stream));
  FG_HIP(hipMemcpyAsync(P->hd, P->dscal, 64 * sizeof(double), hipMemcpyDeviceToHost, P->stream));
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

// ----------------------------------------------------------------------------
// 3-D transforms on the plan grid.
template <typename R> const TablesDev<R>& tabs(const fg_plan* P);
template <> const TablesDev<double>& tabs<double>(const fg_plan* P) { return P->t64; }
template <> const TablesDev<float>& tabs<float>(const fg_plan* P) { return P->t32; }

// Forward passes 1 and 2 (N2 real-to-complex, N1 complex) of ncomp fields,
// in -> data (in may equal data).
template <typename R>
void fwd_xy(fg_plan* P, const R* in, R* data, int ncomp, const int* skip) {
  const SpecTables<R> tb = tabs<R>(P).spec();
  {
    ProfScope ps(P, FG_PASS_R2C);
    launch_r2c<R>(P->M, in, data, (long)ncomp * P->n0 * P->n1, tb, skip, P->stream);
  }
  ProfScope ps(P, FG_PASS_AXIS);
  launch_axis<R>(P->n1, false, data, P->M, (long)P->n1 * P->M, 0, P->M, ncomp * P->n0, 1, tb.tw1, skip,
                 P->stream);
}

// Inverse passes 2 and 1, data -> out with the C2R epilogue; returns #partials.
template <typename R>
int inv_yx(fg_plan* P, R* data, R* out, int ncomp, const C2REpi& epi) {
  const SpecTables<R> tb = tabs<R>(P).spec();
  {
    ProfScope ps(P, FG_PASS_AXIS);
    launch_axis<R>(P->n1, true, data, P->M, (long)P->n1 * P->M, 0, P->M, ncomp * P->n0, 1, tb.tw1, epi.skip,
                   P->stream);
  }
  ProfScope ps(P, FG_PASS_C2R);
  return launch_c2r<R>(P->M, data, out, (long)ncomp * P->n0 * P->n1, tb, epi, P->stream);
}

// y = G * x for 9-component fields (projection), returns #partials.
template <typename R>
int project9(fg_plan* P, const R* in, R* work, R* out, const C2REpi& epi) {
  fwd_xy<R>(P, in, work, 9, epi.skip);
  {
    ProfScope ps(P, FG_PASS_ZPROJ);
    launch_zproj<R>(P->n0, work, P->n1, P->M, tabs<R>(P).spec(), (R)(1.0 / (double)P->N), epi.skip, P->stream);
  }
  return inv_yx<R>(P, work, out, 9, epi);
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
void constitutive(fg_plan* P, const double* Fu, double* Pout, void* state, double* pparts) {
  ProfScope ps(P, FG_PASS_CONSTITUTIVE);
  const unsigned nb = blocks_for(P->N);
  const double* c = P->c ? P->c : P->zeroN;
  const double* d = P->d ? P->d : P->zeroN;
  if (P->prec == FG_FP64)
    hipLaunchKernelGGL((k_constitutive<double>), dim3(nb), dim3(256), 0, P->stream, P->F, Fu, c, d, P->E, P->nu,
                       P->Om, Pout, (double*)state, pparts, P->flags, P->N);
  else
    hipLaunchKernelGGL((k_constitutive<float>), dim3(nb), dim3(256), 0, P->stream, P->F, Fu, c, d, P->E, P->nu,
                       P->Om, Pout, (float*)state, pparts, P->flags, P->N);
  check_launch();
}

// ||G*P|| of the stress in S64 (in place), into dscal[slot]; G*P stays in S64.
void residual_norm(fg_plan* P, int slot) {
  C2REpi epi{1.0, nullptr, true, P->part, nullptr};
  const int nb = project9<double>(P, P->S64, P->S64, P->S64, epi);
  reduce_to(P, P->part, nb, slot);
}

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
  P->prof_noop[FG_PASS_FRONT] += noop;
  P->prof_noop[FG_PASS_AXIS] += 2 * noop;
  P->prof_noop[FG_PASS_ZPROJ] += noop;
  P->prof_noop[FG_PASS_C2R] += noop;
  P->prof_noop[FG_PASS_FINALIZE] += 2 * noop;
}

template <typename T>
void cg_solve(fg_plan* P, const fg_solver_opts* o, fg_stats* stats) {
  T* S = (T*)P->S;
  T* x = (T*)P->x;
  T* r = (T*)P->r;
  T* p = (T*)P->p;
  const T* st = (const T*)P->st;
  KrylovScalars* ks = P->ks;
  const long n9 = 9 * P->N;
  // ks was initialised (rr0, rr, iter = 0, done) by the residual pass
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, x, T(0), n9);
  check_launch();
  {
    // only tol2 / maxit are host-set; the rest was set on the device
    P->hd[62] = (o->fixed_lin > 0) ? 0.0 : o->tol_lin * o->tol_lin;
    ((int*)(P->hd + 63))[0] = (o->fixed_lin > 0) ? o->fixed_lin : o->max_lin;
    FG_HIP(hipMemcpyAsync(&ks->tol2, P->hd + 62, sizeof(double), hipMemcpyHostToDevice, P->stream));
    FG_HIP(hipMemcpyAsync(&ks->maxit, P->hd + 63, sizeof(int), hipMemcpyHostToDevice, P->stream));
  }
  const SpecTables<T> tb = tabs<T>(P).spec();
  const int* skip = &ks->done;
  int chunk = 8;
  long launched = 0;
  for (int guard = 0; guard < 1000000; ++guard) {
    launched += chunk;
    for (int k = 0; k < chunk; ++k) {
      // x += alpha_{k-1} p_{k-1}; p = r + beta p; Y = K:p; p.Y; N2 pass of Y
      int nbf;
      {
        ProfScope ps(P, FG_PASS_FRONT);
        nbf = launch_cg_front<T>(P->M, S, p, x, r, st, ks, P->part, P->N, (long)P->n0 * P->n1, tb, P->stream);
      }
      {
        ProfScope ps(P, FG_PASS_FINALIZE);  // alpha = r.r / p.Kp
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part, nbf, ks, (double*)nullptr, 0, 0);
      }
      {
        ProfScope ps(P, FG_PASS_AXIS);
        launch_axis<T>(P->n1, false, S, P->M, (long)P->n1 * P->M, 0, P->M, 9 * P->n0, 1, tb.tw1, skip, P->stream);
      }
      {
        ProfScope ps(P, FG_PASS_ZPROJ);
        launch_zproj<T>(P->n0, S, P->n1, P->M, tb, (T)(1.0 / (double)P->N), skip, P->stream);
      }
      {
        ProfScope ps(P, FG_PASS_AXIS);
        launch_axis<T>(P->n1, true, S, P->M, (long)P->n1 * P->M, 0, P->M, 9 * P->n0, 1, tb.tw1, skip, P->stream);
      }
      int nbc;
      {
        // r -= alpha G(K p), r.r
        ProfScope ps(P, FG_PASS_C2R);
        C2REpi epi{1.0, nullptr, true, P->part2, skip, r, ks};
        nbc = launch_c2r<T>(P->M, S, S, 9L * P->n0 * P->n1, tb, epi, P->stream);
      }
      {
        ProfScope ps(P, FG_PASS_FINALIZE);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part2, nbc, ks, (double*)nullptr, 1, 0);
      }
      check_launch();
    }
    sync_read(P);
    if (P->hks[0].done) break;
    chunk = next_chunk(P->hks[0], launched);
  }
  const KrylovScalars& h = P->hks[0];
  note_noop_iterations(P, launched - h.iter);
  // the last deferred solution update
  hipLaunchKernelGGL((k_cg_final_x<T>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, x, p, ks, n9);
  check_launch();
  if (stats) {
    stats->lin_iters_last = h.iter;
    stats->lin_relres = h.rr0 > 0 ? std::sqrt(h.rr / h.rr0) : 0.0;
  }
  // An inexact inner solve in the mixed form (single-precision rounding
  // breaking p.Ap > 0, or the iteration cap) still hands its correction to
  // the double-precision Newton loop, which measures the true residual.
  const bool inexact_ok = (P->prec == FG_MIXED) && h.iter > 0;
  if (h.flag == 1 && !inexact_ok) throw Status(FG_E_BREAKDOWN, "CG breakdown: p.Ap <= 0");
  if (h.flag == 2 && !inexact_ok) throw Status(FG_E_NOCONV, "CG reached max_lin iterations");
}

// Newton loop of Alg. 1 at the current F (increment already applied).
void newton(fg_plan* P, const double Fmacro[9], const fg_solver_opts* o, fg_stats* stats) {
  const long n9 = 9 * P->N;
  // normaliser of eq. (31): ||G*P(Fbar)||, with floors (A8)
  FG_HIP(hipMemcpyAsync(P->Fu, Fmacro, 9 * sizeof(double), hipMemcpyHostToDevice, P->stream));
  const unsigned nbN = blocks_for(P->N);
  constitutive(P, P->Fu, P->S64, nullptr, P->part2);
  reduce_to(P, P->part2, (int)nbN, 0);  // ||P(Fbar)||^2
  residual_norm(P, 1);                  // ||G*P(Fbar)||^2
  sync_read(P);
  check_domain(P);
  const double den = std::max(std::max(std::sqrt(P->hd[1]), 1e-14 * std::sqrt(P->hd[0])), 1e-300);
  int it = 0;
  if (stats) {
    stats->newton_iters = 0;
    stats->lin_iters_total = 0;
    stats->n_history = 0;
  }
  while (true) {
    constitutive(P, nullptr, P->S64, P->st, nullptr);
    residual_norm(P, 2);
    sync_read(P);
    check_domain(P);
    const double err = std::sqrt(P->hd[2]) / den;
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
    // b = -G*(G*P): second projection of the residual (compatible rhs)
    {
      C2REpi epi{-1.0, nullptr, true, P->part, nullptr};
      const int nb = project9<double>(P, P->S64, P->S64, P->S64, epi);
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part, nb, P->ks, (double*)nullptr, 5, 0);
      check_launch();
      if (P->prec == FG_FP64) {
        FG_HIP(hipMemcpyAsync(P->r, P->S64, n9 * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
      } else {
        hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream,
                           (float*)P->r, (const double*)P->S64, n9);
        check_launch();
      }
    }
    if (P->prec == FG_FP64) {
      cg_solve<double>(P, o, stats);
      hipLaunchKernelGGL((k_axpy_into_f64<double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, P->F,
                         (const double*)P->x, n9);
    } else {
      fg_solver_opts om = *o;
      // Inner forcing: the single-precision operator is accurate to a few
      // 1e-7 at 256^3 (FFT rounding), so CG is not asked for more than 1e-5;
      // the double-precision Newton residual refines the rest.
      if (om.fixed_lin <= 0) om.tol_lin = std::max(o->tol_lin, 1e-5);
      cg_solve<float>(P, &om, stats);
      // The correction must be compatible (F~ stays a gradient field): single-
      // precision FFT rounding leaves an incompatible part of a few 1e-7 in x
      // that the equilibrium residual never sees, so x is projected once in
      // double precision before the update, dF = G * x.
      hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, P->S64,
                         (const float*)P->x, n9);
      {
        C2REpi epi{1.0, nullptr, true, nullptr, nullptr};
        project9<double>(P, P->S64, P->S64, P->S64, epi);
      }
      hipLaunchKernelGGL((k_axpy_into_f64<double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, P->F,
                         (const double*)P->S64, n9);
    }
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
// G(K:lam) = -G(K:W) for the compatible, zero-mean lam with the same CG, then
// the per-voxel gradients with respect to log E and Omega.
template <typename T>
void adjoint(fg_plan* P, const double W[9], double* gE, double* gO, const fg_solver_opts* o, fg_stats* stats) {
  const long N = P->N, n9 = 9 * N;
  T* S = (T*)P->S;
  T* pbuf = (T*)P->p;
  constitutive(P, nullptr, nullptr, P->st, nullptr);
  FG_HIP(hipMemcpyAsync(P->Fu, W, 9 * sizeof(double), hipMemcpyHostToDevice, P->stream));
  hipLaunchKernelGGL((k_fill_uniform9<T>), dim3(blocks_for(N)), dim3(256), 0, P->stream, pbuf, (const double*)P->Fu,
                     N);
  hipLaunchKernelGGL((k_contract<T>), dim3(blocks_for(N / 2)), dim3(256), 0, P->stream, S, pbuf, (const T*)nullptr,
                     (const T*)P->st, (const KrylovScalars*)nullptr, N, 0);
  check_launch();
  {
    // b = -G*(G*(K:W)): the second projection keeps the right-hand side
    // compatible to rounding (as for the Newton right-hand side)
    C2REpi e1{1.0, nullptr, true, nullptr, nullptr};
    project9<T>(P, S, S, S, e1);
    C2REpi e2{-1.0, nullptr, true, P->part, nullptr};
    const int nb = project9<T>(P, S, S, S, e2);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part, nb, P->ks, (double*)nullptr, 5, 0);
    FG_HIP(hipMemcpyAsync(P->r, S, n9 * sizeof(T), hipMemcpyDeviceToDevice, P->stream));
    check_launch();
  }
  sync_read(P);
  check_domain(P);
  if (!P->hks[0].done) {
    cg_solve<T>(P, o, stats);
  } else {
    hipLaunchKernelGGL((k_fill<T>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, (T*)P->x, T(0), n9);
  }
  const double* c = P->c ? P->c : P->zeroN;
  const double* d = P->d ? P->d : P->zeroN;
  hipLaunchKernelGGL((k_adjoint_grad<T>), dim3(blocks_for(N)), dim3(256), 0, P->stream, P->F, c, d, P->E, P->nu,
                     P->Om, (const T*)P->x, (const double*)P->Fu, gE, gO, P->flags, N);
  check_launch();
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
  KrylovScalars* ks = P->ks + 1;
  P->hd[60] = (o->fixed_lin > 0) ? 0.0 : o->tol_lin * o->tol_lin;
  ((int*)(P->hd + 61))[0] = (o->fixed_lin > 0) ? o->fixed_lin : o->max_lin;
  FG_HIP(hipMemcpyAsync(&ks->tol2, P->hd + 60, sizeof(double), hipMemcpyHostToDevice, P->stream));
  FG_HIP(hipMemcpyAsync(&ks->maxit, P->hd + 61, sizeof(int), hipMemcpyHostToDevice, P->stream));
  const int* skip = &ks->done;
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
    if (P->hks[1].done) break;
    chunk = next_chunk(P->hks[1], 0);
  }
  const KrylovScalars& h = P->hks[1];
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
                     v.a, v.r, v.x, P->gc, P->lc, P->part, P->part2, P->flags, P->N);
  check_launch();
  reduce_to(P, P->part, (int)nbN, 0);  // sum H
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part2, (int)nbN, P->ks + 1, (double*)nullptr,
                     5, 1);
  check_launch();
  sync_read(P);
  check_domain(P);
  if (stats) stats->lin_iters_total = 0;
  const double Hbar = P->hd[0] / (double)P->N;
  if (!P->hks[1].done) {
    scalar_pcg(P, ScalarOp::PFF, P->gc / P->lc + 2.0 * Hbar, P->gc * P->lc, 0.0, o, stats);
  } else if (stats) {
    stats->lin_iters_last = 0;
    stats->lin_relres = 0.0;
  }
  FG_HIP(hipMemcpyAsync(P->d, v.x, P->N * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
}

void fick(fg_plan* P, double dt, const double* cdot, const fg_solver_opts* o, fg_stats* stats) {
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
                       P->cmax, v.mu, v.w, P->part, P->flags, N);
    check_launch();
    reduce_to(P, P->part, (int)nbN, 2);  // sum 1/w
    hipLaunchKernelGGL(k_fick_residual, dim3(nbN), dim3(256), 0, P->stream, P->c, v.ct, v.mu, v.A6, cdot, dt, g,
                       v.r, v.x, P->part2, N);
    check_launch();
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, P->stream, P->part2, (int)nbN, P->ks + 1,
                       (double*)nullptr, 5, 1);
    check_launch();
    sync_read(P);
    check_domain(P);
    const double winv = P->hd[2] / (double)N;
    if (!P->hks[1].done) scalar_pcg(P, ScalarOp::FICK, winv, dt * abar, dt, o, stats);
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
                     P->N);
  check_launch();
}

}  // namespace

// ------------------------------------------------------------------ C ABI --
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

void need_ready(fg_plan* P, bool need_state) {
  if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
  if (!P->have_material) throw Status(FG_E_STATE, "material not set");
  if (need_state && !P->F) throw Status(FG_E_STATE, "state not set");
}
}  // namespace

extern "C" {

fg_status fg_plan_create(const int grid[3], const double spacing[3], fg_precision prec, void* stream,
                         fg_plan** out) {
  if (!grid || !spacing || !out) return FG_E_ARG;
  *out = nullptr;
  if (prec != FG_FP64 && prec != FG_MIXED) return FG_E_ARG;
  for (int k = 0; k < 3; ++k)
    if (!(spacing[k] > 0.0) || !std::isfinite(spacing[k])) return FG_E_ARG;
  if (!fg::fft_axis_length_supported(grid[0]) || !fg::fft_axis_length_supported(grid[1])) return FG_E_SIZE;
  if (grid[2] % 2 != 0 || !fg::fft_length_supported(grid[2] / 2) || grid[2] < 4) return FG_E_SIZE;
  fg_plan* P = new (std::nothrow) fg_plan();
  if (!P) return FG_E_HIP;
  P->n0 = grid[0];
  P->n1 = grid[1];
  P->n2 = grid[2];
  P->M = grid[2] / 2;
  P->N = (long)grid[0] * grid[1] * grid[2];
  for (int k = 0; k < 3; ++k) P->h[k] = spacing[k];
  P->prec = prec;
  P->stream = (hipStream_t)stream;
  P->need = layout(P, nullptr) + kAlign;
  if (hipHostMalloc((void**)&P->hks, 2 * sizeof(KrylovScalars), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&P->hd, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&P->hflags, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    fg_plan_destroy(P);
    return FG_E_HIP;
  }
  *out = P;
  return FG_OK;
}

size_t fg_plan_workspace_bytes(const fg_plan* P) { return P ? P->need : 0; }

fg_status fg_plan_set_workspace(fg_plan* P, void* dev, size_t bytes) {
  if (!P || !dev) return FG_E_ARG;
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
    FG_HIP(hipMemsetAsync(P->ks, 0, 2 * sizeof(KrylovScalars), P->stream));
    FG_HIP(hipMemsetAsync(P->flags, 0, 4 * sizeof(int), P->stream));
    P->zeroN = P->sc + 15 * P->N;
    FG_HIP(hipMemsetAsync(P->zeroN, 0, P->N * sizeof(double), P->stream));
    FG_HIP(hipStreamSynchronize(P->stream));  // the host blob goes out of scope
  });
}

fg_status fg_set_material(fg_plan* P, const double* E, const double* nu, const double* Omega, const double* D,
                          const double* sigma_max, double gc, double lc, double RT, double c_max) {
  if (!P || !E || !nu || !Omega) return FG_E_ARG;
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
  if (!P || !F) return FG_E_ARG;
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

fg_status fg_adjoint_gradient(fg_plan* P, const double dL_dPavg[9], double* dL_dlogE, double* dL_dOmega,
                              const fg_solver_opts* opts, fg_stats* stats) {
  if (!P || !dL_dPavg || !opts) return FG_E_ARG;
  if (!dL_dlogE && !dL_dOmega) return FG_E_ARG;
  return run(P, [&]() {
    need_ready(P, true);
    if (P->prec != FG_FP64) throw Status(FG_E_ARG, "the adjoint is built for FG_FP64 plans");
    if (stats) std::memset(stats, 0, sizeof(fg_stats));
    adjoint<double>(P, dL_dPavg, dL_dlogE, dL_dOmega, opts, stats);
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
      hipLaunchKernelGGL((k_contract<double>), dim3(blocks_for(P->N / 2)), dim3(256), 0, P->stream, y, (double*)x,
                         (const double*)nullptr,
                         (const double*)P->st, (const KrylovScalars*)nullptr, P->N, 0);
      check_launch();
      C2REpi epi{1.0, nullptr, true, nullptr, nullptr};
      project9<double>(P, y, y, y, epi);
    } else {
      constitutive(P, nullptr, nullptr, P->st, nullptr);
      float* xf = (float*)P->p;
      float* yf = (float*)P->S;
      hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, xf, x,
                         n9);
      hipLaunchKernelGGL((k_contract<float>), dim3(blocks_for(P->N / 2)), dim3(256), 0, P->stream, yf, xf,
                         (const float*)nullptr,
                         (const float*)P->st, (const KrylovScalars*)nullptr, P->N, 0);
      check_launch();
      C2REpi epi{1.0, nullptr, true, nullptr, nullptr};
      project9<float>(P, yf, yf, yf, epi);
      hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_stride_blocks(n9)), dim3(256), 0, P->stream, y,
                         (const float*)yf, n9);
    }
    check_launch();
  });
}

fg_status fg_project(fg_plan* P, const double* x, double* y) {
  if (!P || !x || !y) return FG_E_ARG;
  return run(P, [&]() {
    if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
    C2REpi epi{1.0, nullptr, true, nullptr, nullptr};
    project9<double>(P, x, P->S64, y, epi);
    check_launch();
  });
}

fg_status fg_fft_r2c(fg_plan* P, double* data, int ncomp) {
  if (!P || !data || ncomp <= 0) return FG_E_ARG;
  return run(P, [&]() {
    if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
    const SpecTables<double> tb = P->t64.spec();
    fwd_xy<double>(P, data, data, ncomp, nullptr);
    launch_axis<double>(P->n0, false, data, (long)P->n1 * P->M, P->M, (long)P->n0 * P->n1 * P->M, P->M, P->n1,
                        ncomp, tb.tw0, nullptr, P->stream);
    check_launch();
  });
}

fg_status fg_fft_c2r(fg_plan* P, double* data, int ncomp) {
  if (!P || !data || ncomp <= 0) return FG_E_ARG;
  return run(P, [&]() {
    if (!P->ws) throw Status(FG_E_STATE, "workspace not set");
    const SpecTables<double> tb = P->t64.spec();
    launch_axis<double>(P->n0, true, data, (long)P->n1 * P->M, P->M, (long)P->n0 * P->n1 * P->M, P->M, P->n1,
                        ncomp, tb.tw0, nullptr, P->stream);
    C2REpi epi{1.0 / (double)P->N, nullptr, true, nullptr, nullptr};
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

fg_status fg_profile_begin(fg_plan* P) {
  if (!P) return FG_E_ARG;
  return run(P, [&]() {
    FG_HIP(hipStreamSynchronize(P->stream));
    P->prof_on = true;
    for (int k = 0; k < FG_NPASS; ++k) {
      P->prof_used[k] = 0;
      P->prof_noop[k] = 0;
    }
  });
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
  if (!P) return;
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

}  // extern "C"
