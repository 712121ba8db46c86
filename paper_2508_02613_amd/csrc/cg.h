// Preconditioned CG control (Saad Alg. 9.1 in the split form used by the
// paper's footnote to eq. prec_lin_system_general) kept on the device:
// single-block kernels (one block per cell of a batch) reduce the per-block
// partial sums in a fixed order (deterministic) and update the scalars alpha,
// beta, the iteration count and the stop flag.  Every loop kernel returns at
// once when its cell's flag is set, so the host may queue (or replay as a
// graph) iterations ahead of the convergence test, and cells of a batch stop
// independently.
#pragma once
#include "jfft_common.h"
#include "stencil.h"

namespace jfft {

constexpr int CTRL_THREADS = 1024;
constexpr int CTRL_WAVES = CTRL_THREADS / 64;

// Fixed-order sum of n partials by one block: thread t sums t, t + T, t + 2T,
// ... (T = CTRL_THREADS) in that order, then a fixed tree.  Eight partials are
// loaded at a time before they are added, so the loads overlap instead of
// forming one dependent chain.  Result valid in thread 0.
__device__ __forceinline__ double fixed_sum(const double *p, long long n, double *sm) {
  double v = 0.0;
  long long i = threadIdx.x;
  for (; i + 7LL * CTRL_THREADS < n; i += 8LL * CTRL_THREADS) {
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = p[i + (long long)k * CTRL_THREADS];
#pragma unroll
    for (int k = 0; k < 8; ++k) v += t[k];
  }
  for (; i < n; i += CTRL_THREADS) v += p[i];
  return block_sum<CTRL_THREADS>(v, sm);
}

// alpha_k = (r.z) / (p.q); breakdown if p.q <= 0 or alpha not finite.
// parity: which of the two search-direction buffers holds p_k.
__global__ void k_cg_alpha(CgState *st, const double *part, long long n, History h, int parity,
                           long long cs) {
  __shared__ double sm[CTRL_WAVES];
  st = cshift(st, blockIdx.x, cs);
  part = cshift(part, blockIdx.x, cs);
  shift_hist(h, blockIdx.x, cs);
  if (st->done) return;
  const double pq = fixed_sum(part, n, sm);
  if (threadIdx.x == 0) cg_alpha_step(st, pq, h, parity);
}

// ||r_{k+1}||^2; count the update of u; stop on tolerance or maxit.
__global__ void k_cg_rr(CgState *st, const double *part, long long n, History h, long long cs) {
  __shared__ double sm[CTRL_WAVES];
  st = cshift(st, blockIdx.x, cs);
  part = cshift(part, blockIdx.x, cs);
  shift_hist(h, blockIdx.x, cs);
  if (st->done) return;
  const double rr = fixed_sum(part, n, sm);
  if (threadIdx.x == 0) cg_rr_step(st, rr, h);
}

// beta_k = (r.z)_new / (r.z)_old.
__global__ void k_cg_beta(CgState *st, const double *part, long long n, History h, long long cs) {
  __shared__ double sm[CTRL_WAVES];
  st = cshift(st, blockIdx.x, cs);
  part = cshift(part, blockIdx.x, cs);
  shift_hist(h, blockIdx.x, cs);
  if (st->done) return;
  const double rz = fixed_sum(part, n, sm);
  if (threadIdx.x == 0) cg_beta_step(st, rz, h);
}

// ||f||^2 and ||f_abs||^2 from partials; the homogeneous-material test.
// The stopping threshold relative to ||f||: tol itself (relative rule), or
// sqrt(tol) / ||f|| for the absolute rule ||r||^2 <= tol of the paper's runs.
__global__ void k_solve_norms(CgState *st, const double *partF, const double *partA, long long n,
                              double tol, int absolute, long long cs) {
  __shared__ double sm[CTRL_WAVES];
  st = cshift(st, blockIdx.x, cs);
  partF = cshift(partF, blockIdx.x, cs);
  partA = cshift(partA, blockIdx.x, cs);
  const double f2 = fixed_sum(partF, n, sm);
  const double a2 = fixed_sum(partA, n, sm);
  if (threadIdx.x == 0) {
    st->fnorm2 = f2;
    st->fabs2 = a2;
    st->homog = (sqrt(f2) <= 1e-13 * sqrt(a2)) ? 1 : 0;
    st->outer_done = st->homog;
    st->outer = 0;
    st->total_iters = 0;
    st->final_status = ST_OK;
    st->rn = sqrt(f2);
    st->tolr = (absolute && f2 > 0.0) ? sqrt(tol / f2) : tol;
  }
}

// Inner PCG set-up.  FP64 solve (mixed = 0): stop at ||r|| <= tol ||f||.
// Mixed inner solve on r / ||r|| (mixed = 1): stop at relative
// max(inner_tol, tol ||f|| / (2 ||r||)), or after inner_cap iterations
// (> 0): an FP32 solve that stalls short of its tolerance then hands its
// progress to the next FP64 refinement sweep instead of running on.  Cells already finished (homogeneous
// material, or refinement converged) start in the stopped state.
__global__ void k_cg_init(CgState *st, double inner_tol, int mixed, int maxit, int hist_cap,
                          int inner_cap, long long cs) {
  st = cshift(st, blockIdx.x, cs);
  if (threadIdx.x != 0) return;
  double t2;
  int mx = maxit;
  if (mixed) {
    const double rel = fmax(inner_tol, 0.5 * st->tolr * sqrt(st->fnorm2) / st->rn);
    t2 = rel * rel;
    mx = maxit - st->total_iters;
    if (mx < 1) mx = 1;
    if (inner_cap > 0 && mx > inner_cap) mx = inner_cap;
  } else {
    t2 = st->tolr * st->tolr * st->fnorm2;
  }
  st->tol2 = t2;
  st->maxit = mx;
  st->hist_cap = hist_cap;
  st->iter = 0;
  st->arrive[0] = st->arrive[1] = st->arrive[2] = 0;
  st->done = st->outer_done;
  st->status = ST_OK;
  st->pending = 0;
  st->first = 1;
  st->parity = 0;
}

// Start of the loop: rr0 and rz0 from partials; stop at once when
// ||r_0||^2 <= tol2 (or maxit == 0).
__global__ void k_cg_start(CgState *st, const double *partRR, long long nRR, const double *partRZ,
                           long long nRZ, long long cs) {
  __shared__ double sm[CTRL_WAVES];
  st = cshift(st, blockIdx.x, cs);
  partRR = cshift(partRR, blockIdx.x, cs);
  partRZ = cshift(partRZ, blockIdx.x, cs);
  const double rr = fixed_sum(partRR, nRR, sm);
  const double rz = fixed_sum(partRZ, nRZ, sm);
  if (threadIdx.x == 0) {
    if (st->done) return;  // finished before this solve
    st->rr = rr;
    st->rr0 = rr;
    st->rz = rz;
    if (rr <= st->tol2) {
      st->done = 1;
    } else if (st->maxit <= 0) {
      st->done = 1;
      st->status = ST_NOT_CONVERGED;
    }
  }
}

// Mixed precision, refinement sweeps after the first: the FP32 CG of the
// previous sweep is continued instead of restarted (a "reliable update":
// the recursive residual is replaced by the true FP64 residual, the search
// direction is kept).  In exact arithmetic the replacement changes nothing,
// so the iterates are those of one uninterrupted CG run; a restart would
// drop the Krylov space built so far and repeat much of its convergence.
// The FP32 vectors of a sweep are scaled by 1 / ||r|| of that sweep, so the
// kept direction is rescaled by s = rn_prev / rn and beta = (r.z)_new /
// (s^2 (r.z)_old).  A cell continues when its previous inner solve formed a
// direction and did not break down; otherwise it restarts.  alpha = 0: the
// previous sweep's last update of the correction was already applied.
__global__ void k_cg_init_continue(CgState *st, double inner_tol, int maxit, int inner_cap,
                                   long long cs) {
  st = cshift(st, blockIdx.x, cs);
  if (threadIdx.x != 0) return;
  const bool cont = st->outer >= 1 && st->iter > 0 && st->status != ST_BREAKDOWN;
  const double rel = fmax(inner_tol, 0.5 * st->tolr * sqrt(st->fnorm2) / st->rn);
  int mx = maxit - st->total_iters;
  if (mx < 1) mx = 1;
  if (inner_cap > 0 && mx > inner_cap) mx = inner_cap;
  st->tol2 = rel * rel;
  st->maxit = mx;
  st->hist_cap = 0;
  st->iter = 0;
  st->arrive[0] = st->arrive[1] = st->arrive[2] = 0;
  st->done = st->outer_done;
  st->status = ST_OK;
  st->pending = 0;
  st->alpha = 0.0;
  st->first = cont ? 0 : 1;
  // parity is kept: k_scale_direction reads the buffer that holds p
}

// The kept direction, rescaled to this sweep's FP32 scale, into p1 (the
// buffer the first iteration of a loop reads p_old from).
template <typename Real>
__global__ void k_scale_direction(const Real *p0, Real *p1, long long n, const CgState *st,
                                  long long cs) {
  const int cell = blockIdx.y;
  st = cshift(st, cell, cs);
  if (st->done || st->first) return;
  const Real *src = cshift(st->parity ? (const Real *)p1 : p0, cell, cs);
  Real *dst = cshift(p1, cell, cs);
  const Real s = (Real)(st->rn_prev / st->rn);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = s * src[i];
}

// k_cg_start for a continued loop: also beta of the kept direction.
__global__ void k_cg_start_continue(CgState *st, const double *partRR, long long nRR,
                                    const double *partRZ, long long nRZ, long long cs) {
  __shared__ double sm[CTRL_WAVES];
  st = cshift(st, blockIdx.x, cs);
  partRR = cshift(partRR, blockIdx.x, cs);
  partRZ = cshift(partRZ, blockIdx.x, cs);
  const double rr = fixed_sum(partRR, nRR, sm);
  const double rz = fixed_sum(partRZ, nRZ, sm);
  if (threadIdx.x == 0) {
    if (st->done) return;
    if (!st->first) {
      const double s = st->rn_prev / st->rn;
      const double beta = rz / (s * s * st->rz);
      if (isfinite(beta)) {
        st->beta = beta;
      } else {
        st->first = 1;  // restart from z
      }
    }
    st->rr = rr;
    st->rr0 = rr;
    st->rz = rz;
    if (rr <= st->tol2) {
      st->done = 1;
    } else if (st->maxit <= 0) {
      st->done = 1;
      st->status = ST_NOT_CONVERGED;
    }
  }
}

// Mixed precision: the FP64 residual ||f - K u|| of this sweep decides
// whether refinement continues.  (The first sweep starts from u = u0.)
__global__ void k_outer_check(CgState *st, const double *part, long long n, int max_outer,
                              int maxit, long long cs) {
  __shared__ double sm[CTRL_WAVES];
  st = cshift(st, blockIdx.x, cs);
  part = cshift(part, blockIdx.x, cs);
  const double rr = fixed_sum(part, n, sm);
  if (threadIdx.x == 0) {
    if (st->outer_done) return;
    const double rn = sqrt(rr);
    st->rn_prev = st->rn;
    st->rn = rn;
    if (rn <= st->tolr * sqrt(st->fnorm2)) {
      st->outer_done = 1;
      st->final_status = ST_OK;
    } else if (st->outer >= max_outer || st->total_iters >= maxit) {
      st->outer_done = 1;
      st->final_status = ST_NOT_CONVERGED;
    }
  }
}

// After an inner solve: count it; a breakdown before any progress ends the
// refinement.
__global__ void k_outer_update(CgState *st, long long cs) {
  st = cshift(st, blockIdx.x, cs);
  if (threadIdx.x != 0 || st->outer_done) return;
  st->outer += 1;
  st->total_iters += st->iter;
  if (st->status == ST_BREAKDOWN && st->iter == 0) {
    st->outer_done = 1;
    st->final_status = ST_BREAKDOWN;
  }
}

// A free slot of a continuously batched group: stopped, so every kernel of
// the captured iterations returns at once for it.
__global__ void k_slot_park(CgState *st, long long cs) {
  st = cshift(st, blockIdx.x, cs);
  if (threadIdx.x != 0) return;
  st->done = 1;
  st->outer_done = 1;
  st->pending = 0;
  st->arrive[0] = st->arrive[1] = st->arrive[2] = 0;
}

// A slot's material check, run after its solve set-up: E with negative or
// non-finite entries (count in small[0], see k_check_E) stops the slot
// before any iteration with the status JFFT_E_INVALID.
__global__ void k_slot_validate(CgState *st, const double *small, long long cs) {
  st = cshift(st, blockIdx.x, cs);
  small = cshift(small, blockIdx.x, cs);
  if (threadIdx.x != 0 || small[0] == 0.0) return;
  st->outer_done = 1;
  st->done = 1;
  st->final_status = ST_INVALID;
}

// FP64 solve: final status from the loop state.
__global__ void k_fp64_final(CgState *st, long long cs) {
  st = cshift(st, blockIdx.x, cs);
  if (threadIdx.x != 0 || st->final_status == ST_INVALID) return;
  st->total_iters = st->iter;
  st->outer = st->homog ? 0 : 1;
  st->final_status = st->homog ? ST_OK : st->status;
}

// Generic fixed-order reduction of `count` groups of n partials each into out[g]
// (one block per cell).
__global__ void k_reduce_groups(const double *part, long long n, int count, double *out,
                                long long cs) {
  __shared__ double sm[CTRL_WAVES];
  part = cshift(part, blockIdx.x, cs);
  out = cshift(out, blockIdx.x, cs);
  for (int g = 0; g < count; ++g) {
    const double s = fixed_sum(part + (long long)g * n, n, sm);
    if (threadIdx.x == 0) out[g] = s;
  }
}

// ------------------------------------------------------ vector kernels ---
// All take the cell from blockIdx.y (blockIdx.z where y is the component).

// u += alpha p_k if an update is pending (after the loop stopped); p_k is
// the buffer recorded in st->parity.
template <typename Real>
__global__ void k_finish_u(Real *u, const Real *p0, const Real *p1, long long n, const CgState *st,
                           long long cs) {
  const int cell = blockIdx.y;
  st = cshift(st, cell, cs);
  if (!st->pending) return;
  u = cshift(u, cell, cs);
  const Real *p = cshift(st->parity ? p1 : p0, cell, cs);
  const Real alpha = (Real)st->alpha;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    u[i] += alpha * p[i];
}

// out = a - b (out may be NULL), with partial sums of (a - b)^2.
template <typename Real>
__global__ void k_sub_norm(const Real *a, const Real *b, Real *out, long long n, double *part,
                           long long cs) {
  __shared__ double red[8];
  const int cell = blockIdx.y;
  a = cshift(a, cell, cs);
  b = cshift(b, cell, cs);
  out = cshift(out, cell, cs);
  part = cshift(part, cell, cs);
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const Real v = a[i] - b[i];
    if (out) out[i] = v;
    acc += (double)v * (double)v;
  }
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Partial sums of x.y (y may equal x).
template <typename Real>
__global__ void k_dot(const Real *x, const Real *y, long long n, double *part, long long cs) {
  __shared__ double red[8];
  const int cell = blockIdx.y;
  x = cshift(x, cell, cs);
  y = cshift(y, cell, cs);
  part = cshift(part, cell, cs);
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc += (double)x[i] * (double)y[i];
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Per-component partial sums of x: part[c * nblk + b] (component blockIdx.y,
// cell blockIdx.z).
template <typename Real>
__global__ void k_comp_sum(const Real *x, long long N, double *part, long long cs) {
  __shared__ double red[8];
  const int c = blockIdx.y;
  x = cshift(x, blockIdx.z, cs);
  part = cshift(part, blockIdx.z, cs);
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    acc += (double)x[c * N + i];
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) part[(long long)c * gridDim.x + blockIdx.x] = s;
}

// x[c] -= sums[c] / N.
template <typename Real>
__global__ void k_sub_mean(Real *x, long long N, const double *sums, long long cs) {
  const int c = blockIdx.y;
  x = cshift(x, blockIdx.z, cs);
  sums = cshift(sums, blockIdx.z, cs);
  const Real m = (Real)(sums[c] / (double)N);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    x[c * N + i] -= m;
}

// b = a between arrays with their own cell strides.
template <typename Real>
__global__ void k_copy(const Real *a, long long as, Real *b, long long bs, long long n) {
  a = cshift(a, blockIdx.y, as);
  b = cshift(b, blockIdx.y, bs);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// b += a (single cell).
template <typename Real>
__global__ void k_add(const Real *a, Real *b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] += a[i];
}

template <typename Real>
__global__ void k_fill(Real *a, Real v, long long n, long long cs) {
  a = cshift(a, blockIdx.y, cs);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    a[i] = v;
}

// u = u0 unless the cell's material is homogeneous (then u = 0).
__global__ void k_start_vector(const double *u0, long long u0s, double *u, long long n,
                               const CgState *st, long long cs) {
  const int cell = blockIdx.y;
  st = cshift(st, cell, cs);
  u = cshift(u, cell, cs);
  if (u0) u0 = cshift(u0, cell, u0s);
  const bool zero = st->homog || !u0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    u[i] = zero ? 0.0 : u0[i];
}

// J^1/2 = diag^-1/2 after the void rule (exact zeros -> void_value).
template <typename Real>
__global__ void k_jhalf(const double *diag, Real *Jh, long long n, double void_value, long long cs) {
  diag = cshift(diag, blockIdx.y, cs);
  Jh = cshift(Jh, blockIdx.y, cs);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double d = diag[i];
    if (d == 0.0) d = void_value;
    Jh[i] = (Real)(1.0 / sqrt(d));
  }
}

// Element moduli: partial counts of bad entries (negative or non-finite).
__global__ void k_check_E(const double *E, long long es, long long n, double *part, long long cs) {
  __shared__ double red[8];
  E = cshift(E, blockIdx.y, es);
  part = cshift(part, blockIdx.y, cs);
  double bad = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double e = E[i];
    if (!(e >= 0.0) || !isfinite(e)) bad += 1.0;
  }
  const double s = block_sum<256>(bad, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// b = a * scale; with st != NULL the scale is 1 / st->rn (mixed refinement).
template <typename A, typename B>
__global__ void k_convert(const A *a, B *b, long long n, double scale, const CgState *st,
                          long long cs) {
  a = cshift(a, blockIdx.y, cs);
  b = cshift(b, blockIdx.y, cs);
  if (st) {
    st = cshift(st, blockIdx.y, cs);
    scale = st->rn > 0.0 ? 1.0 / st->rn : 0.0;
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = (B)((double)a[i] * scale);
}

// u64 += ||r|| c32 (iterative refinement correction) while refining.
__global__ void k_axpy_f32_to_f64(const float *c, double *u, long long n, const CgState *st,
                                  long long cs) {
  st = cshift(st, blockIdx.y, cs);
  if (st->outer_done) return;
  c = cshift(c, blockIdx.y, cs);
  u = cshift(u, blockIdx.y, cs);
  const double scale = st->rn;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    u[i] += scale * (double)c[i];
}

// ------------------------------------------- projected L-BFGS on [0, 1] ----
// A variable held at a bound by its gradient (x = 0 with g > 0, x = 1 with
// g < 0) is frozen for the step.
__device__ __forceinline__ bool topo_free(double x, double g) {
  return !((x <= 0.0 && g > 0.0) || (x >= 1.0 && g < 0.0));
}

// q = g on the free variables, 0 on the frozen ones.
__global__ void k_topo_free(const double *x, const double *g, double *q, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    q[i] = topo_free(x[i], g[i]) ? g[i] : 0.0;
}

// d = -z on the free variables, 0 on the frozen ones.
__global__ void k_topo_dir(const double *x, const double *g, const double *z, double *d,
                           long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    d[i] = topo_free(x[i], g[i]) ? -z[i] : 0.0;
}

// xt = clip(x + alpha d, 0, 1), st = xt - x.
__global__ void k_topo_trial(const double *x, const double *d, double alpha, double *xt,
                             double *st, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = fmin(1.0, fmax(0.0, x[i] + alpha * d[i]));
    xt[i] = v;
    st[i] = v - x[i];
  }
}

// y = a x + b y (a, b host scalars).
__global__ void k_axpby(double a, const double *x, double b, double *y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}

// out = a - b.
__global__ void k_sub(const double *a, const double *b, double *out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

// Per-block maxima of |x|.
__global__ void k_absmax(const double *x, long long n, double *part) {
  __shared__ double sm[4];
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    m = fmax(m, fabs(x[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[wid] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) r = fmax(r, sm[w]);
    part[blockIdx.x] = r;
  }
}


}  // namespace jfft
