// Device-side control of the batched Newton solve (Alg. 1 for many
// independent items on one grid).  Every item runs its own Newton loop with
// its own CG; the host launches a fixed sequence of "ticks" and each item
// advances by one step per tick:
//   - an item whose CG is running does one CG iteration (masked by the done
//     flag of its Krylov scalars),
//   - an item whose CG has ended does the Newton step: F += dF, P and the
//     tangent, the residual norm and the convergence test of eq. (31), and
//     for the next iteration the right-hand side and a fresh CG.
// The Newton-step kernels are masked by a per-item flag array `idle`, which
// the gate kernel computes at the start of the Newton half of each tick.
#pragma once
#include "fg_fft.hpp"
#include "fg_pointwise.hpp"

namespace fg {

constexpr int FG_NHIST = 32;

// Per-item Newton control block (device memory, one per batch item).
struct NewtonCtl {
  double den;    // normaliser of eq. (31) for the item
  double tol;    // Newton tolerance on err_res
  double err;    // last err_res
  double err_hist[FG_NHIST];
  int max_newton;
  int it;        // Newton iterations done (corrections applied or under way)
  int n_hist;
  int finished;  // 1: converged or failed
  int status;    // fg_status of the item
  int started;   // a CG solve was started and has not been accounted yet
  int mixed;     // an inexact inner solve is accepted (FP32 CG)
  int lin_total, lin_last;
  int lin_hist[FG_NHIST];
};

// idle[b] = 0 for items whose CG has ended and which are not finished (they
// take the Newton step of this tick), 1 otherwise.  Books the iteration count
// of the CG that just ended and fails items whose CG broke down (FP64) or hit
// its cap.  active[0] = number of unfinished items.  One workgroup.
__global__ void __launch_bounds__(1024)
k_newton_gate(const KrylovScalars* __restrict__ ks, NewtonCtl* __restrict__ nc, int* __restrict__ idle,
              int* __restrict__ active, int nitems, int st_breakdown, int st_noconv) {
  __shared__ double red[16];
  double cnt = 0.0;
  for (int b = threadIdx.x; b < nitems; b += blockDim.x) {
    const KrylovScalars& k = ks[b];
    NewtonCtl& c = nc[b];
    int id = 1;
    if (!c.finished && k.done) {
      if (c.started) {
        c.started = 0;
        c.lin_last = k.iter;
        c.lin_total += k.iter;
        if (c.it >= 1 && c.it <= FG_NHIST) c.lin_hist[c.it - 1] = k.iter;
        const bool inexact_ok = c.mixed && k.iter > 0;
        if (k.flag == 1 && !inexact_ok) {
          c.status = st_breakdown;
          c.finished = 1;
        } else if (k.flag == 2 && !inexact_ok) {
          c.status = st_noconv;
          c.finished = 1;
        }
      }
      if (!c.finished) id = 0;
    }
    idle[b] = id;
    cnt += c.finished ? 0.0 : 1.0;
  }
  const double s = block_sum(cnt, red);
  if (threadIdx.x == 0) active[0] = (int)(s + 0.5);
}

// Newton test of one item (one workgroup per item): err = ||G*P|| / den from
// the item's partial sums of (G*P) : (G*P).  Converged items and items out of
// iterations finish; the others count the iteration about to be taken.
__global__ void __launch_bounds__(1024)
k_newton_check(const double* __restrict__ partials, int nparts, NewtonCtl* __restrict__ nc, int* __restrict__ idle,
               int st_noconv) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  if (idle[b]) return;
  const double s = sum_partials(partials + (long)b * nparts, nparts, red);
  if (threadIdx.x != 0) return;
  NewtonCtl& c = nc[b];
  const double err = sqrt(s) / c.den;
  if (c.n_hist < FG_NHIST) c.err_hist[c.n_hist] = err;
  c.n_hist += 1;
  c.err = err;
  if (!(err == err)) {
    c.status = st_noconv;
    c.finished = 1;
  } else if (err <= c.tol) {
    c.finished = 1;
  } else if (c.it >= c.max_newton) {
    c.status = st_noconv;
    c.finished = 1;
  } else {
    c.it += 1;
  }
  if (c.finished) idle[b] = 1;
}

// Start the item's CG on the right-hand side whose partial sums of b.b are
// given (rr0 = rr = b.b, iteration 0; tol2 and maxit stay as set).
__global__ void __launch_bounds__(1024)
k_newton_cg_start(const double* __restrict__ partials, int nparts, KrylovScalars* __restrict__ ks,
                  NewtonCtl* __restrict__ nc, const int* __restrict__ idle) {
  __shared__ double red[16];
  const int b = blockIdx.x;
  if (idle[b]) return;
  const double s = sum_partials(partials + (long)b * nparts, nparts, red);
  if (threadIdx.x != 0) return;
  KrylovScalars& k = ks[b];
  k.rr0 = s;
  k.rr = s;
  k.iter = 0;
  k.flag = 0;
  k.beta = 0.0;
  k.done = (s == 0.0) ? 1 : 0;
  nc[b].started = 1;
}

// Per-item field kernels: grid.y = item, n values per item; masked by idle.
// F += dF (dF in type T).
template <typename T>
__global__ void __launch_bounds__(256)
k_items_axpy(double* __restrict__ F, const T* __restrict__ dF, const int* __restrict__ idle, long n) {
  const int b = blockIdx.y;
  if (idle[b]) return;
  F += (long)b * n;
  dF += (long)b * n;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) F[i] += (double)dF[i];
}

}  // namespace fg
