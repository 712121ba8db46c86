// Preconditioned CG control (Saad Alg. 9.1 in the split form used by the
// paper's footnote to eq. prec_lin_system_general) kept on the device:
// single-block kernels reduce the per-block partial sums in a fixed order
// (deterministic) and update the scalars alpha, beta, the iteration count and
// the stop flag.  Every loop kernel returns at once when the flag is set, so
// the host may queue iterations ahead of the convergence test.
#pragma once
#include "jfft_common.h"
#include "stencil.h"

namespace jfft {

constexpr int CTRL_THREADS = 256;

// Fixed-order sum of n partials by one block: thread t sums t, t + 256, ...
// sequentially, then a fixed tree.  Result valid in thread 0.
__device__ __forceinline__ double fixed_sum(const double *p, long long n, double *sm) {
  double v = 0.0;
  for (long long i = threadIdx.x; i < n; i += CTRL_THREADS) v += p[i];
  return block_sum<CTRL_THREADS>(v, sm);
}

enum StatusCode { ST_OK = 0, ST_NOT_CONVERGED = 4, ST_BREAKDOWN = 5 };

struct History {
  double *alpha, *beta, *res;
};

// alpha_k = (r.z) / (p.q); breakdown if p.q <= 0 or alpha not finite.
__global__ void k_cg_alpha(CgState *st, const double *part, long long n, History h) {
  __shared__ double sm[8];
  if (st->done) return;
  const double pq = fixed_sum(part, n, sm);
  if (threadIdx.x == 0) {
    st->pq = pq;
    const double alpha = st->rz / pq;
    if (!(pq > 0.0) || !isfinite(alpha)) {
      st->done = 1;
      st->status = ST_BREAKDOWN;
      st->pending = 0;
    } else {
      st->alpha = alpha;
      st->pending = 1;
      if (h.alpha && st->iter < st->hist_cap) h.alpha[st->iter] = alpha;
    }
  }
}

// ||r_{k+1}||^2; count the update of u; stop on tolerance or maxit.
__global__ void k_cg_rr(CgState *st, const double *part, long long n, History h) {
  __shared__ double sm[8];
  if (st->done) return;
  const double rr = fixed_sum(part, n, sm);
  if (threadIdx.x == 0) {
    st->rr = rr;
    st->iter += 1;
    if (h.res && st->iter - 1 < st->hist_cap) h.res[st->iter - 1] = sqrt(rr);
    if (rr <= st->tol2) {
      st->done = 1;
      st->status = ST_OK;
    } else if (st->iter >= st->maxit) {
      st->done = 1;
      st->status = ST_NOT_CONVERGED;
    }
  }
}

// beta_k = (r.z)_new / (r.z)_old.
__global__ void k_cg_beta(CgState *st, const double *part, long long n, History h) {
  __shared__ double sm[8];
  if (st->done) return;
  const double rz = fixed_sum(part, n, sm);
  if (threadIdx.x == 0) {
    const double beta = rz / st->rz;
    if (!isfinite(beta)) {
      st->done = 1;
      st->status = ST_BREAKDOWN;
    } else {
      st->beta = beta;
      st->rz = rz;
      st->first = 0;
      if (h.beta && st->iter - 1 < st->hist_cap) h.beta[st->iter - 1] = beta;
    }
  }
}

// Start of the loop: rr0 and rz0 from partials; stop at once when
// ||r_0||^2 <= tol2 (or maxit == 0).
__global__ void k_cg_start(CgState *st, const double *partRR, long long nRR, const double *partRZ,
                           long long nRZ) {
  __shared__ double sm[8];
  const double rr = fixed_sum(partRR, nRR, sm);
  const double rz = fixed_sum(partRZ, nRZ, sm);
  if (threadIdx.x == 0) {
    st->rr = rr;
    st->rz = rz;
    st->first = 1;
    st->pending = 0;
    st->iter = 0;
    st->beta = 0.0;
    st->alpha = 0.0;
    st->done = 0;
    st->status = ST_OK;
    if (rr <= st->tol2) {
      st->done = 1;
    } else if (st->maxit <= 0) {
      st->done = 1;
      st->status = ST_NOT_CONVERGED;
    }
  }
}

// Generic fixed-order reduction of `count` groups of n partials each into out[g].
__global__ void k_reduce_groups(const double *part, long long n, int count, double *out) {
  __shared__ double sm[8];
  for (int g = 0; g < count; ++g) {
    const double s = fixed_sum(part + (long long)g * n, n, sm);
    if (threadIdx.x == 0) out[g] = s;
  }
}

// ------------------------------------------------------ vector kernels ---
// u += alpha p if an update is pending (after the loop stopped).
template <typename Real>
__global__ void k_finish_u(Real *u, const Real *p, long long n, const CgState *st) {
  if (!st->pending) return;
  const Real alpha = (Real)st->alpha;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    u[i] += alpha * p[i];
}

// out = a - b, with partial sums of out.out.
template <typename Real>
__global__ void k_sub_norm(const Real *a, const Real *b, Real *out, long long n, double *part) {
  __shared__ double red[8];
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
__global__ void k_dot(const Real *x, const Real *y, long long n, double *part) {
  __shared__ double red[8];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc += (double)x[i] * (double)y[i];
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Per-component partial sums of x: part[c * nblk + b].
template <typename Real>
__global__ void k_comp_sum(const Real *x, long long N, double *part) {
  __shared__ double red[8];
  const int c = blockIdx.y;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    acc += (double)x[c * N + i];
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) part[(long long)c * gridDim.x + blockIdx.x] = s;
}

// x[c] -= sums[c] / N.
template <typename Real>
__global__ void k_sub_mean(Real *x, long long N, const double *sums) {
  const int c = blockIdx.y;
  const Real m = (Real)(sums[c] / (double)N);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    x[c * N + i] -= m;
}

template <typename Real>
__global__ void k_copy(const Real *a, Real *b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

template <typename Real>
__global__ void k_fill(Real *a, Real v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    a[i] = v;
}

// J^1/2 = diag^-1/2 after the void rule (exact zeros -> void_value).
template <typename Real>
__global__ void k_jhalf(const double *diag, Real *Jh, long long n, double void_value) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double d = diag[i];
    if (d == 0.0) d = void_value;
    Jh[i] = (Real)(1.0 / sqrt(d));
  }
}

// Element moduli: validity check (finite, >= 0) by partial counts of bad entries.
__global__ void k_check_E(const double *E, long long n, double *part) {
  __shared__ double red[8];
  double bad = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double e = E[i];
    if (!(e >= 0.0) || !isfinite(e)) bad += 1.0;
  }
  const double s = block_sum<256>(bad, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Conversions for the mixed-precision path.
template <typename A, typename B>
__global__ void k_convert(const A *a, B *b, long long n, double scale) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = (B)((double)a[i] * scale);
}

// u64 += scale * c32 (iterative refinement correction).
__global__ void k_axpy_f32_to_f64(const float *c, double *u, long long n, double scale) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    u[i] += scale * (double)c[i];
}

}  // namespace jfft
