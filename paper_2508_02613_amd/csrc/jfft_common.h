// Internal declarations shared by the HIP translation units of libjfft.
// Device code targets gfx950 (CDNA4, 64-wide wavefronts) only.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace jfft {

template <typename Real>
struct CxT;
template <>
struct CxT<double> {
  using T = double2;
  using R2 = double2;
};
template <>
struct CxT<float> {
  using T = float2;
  using R2 = float2;
};

// Batches: a group of B cells of identical shape shares one workspace laid
// out as B equal slices of `cs` bytes.  Kernels take the pointers of cell 0
// and shift them to their cell (found from a grid dimension); read-only
// tables shared by all cells are not shifted.
// The shift is byte-pointer arithmetic, not an integer round trip, and
// kernels keep the shifted pointers in local variables rather than writing
// them back into their by-value argument structs: either way the compiler
// loses track of the global address space and falls back to flat accesses,
// which share the LDS wait counter, so that every LDS wait also waits for the
// outstanding HBM loads.
// Streaming (non-temporal) store of one value: for the large per-iteration
// outputs that the next kernel reads once.  Measured on the 256^3 solve:
// with plain stores the dirty lines of one pass are written back while the
// next pass streams its own inputs, which slows the next pass by 5-15 %.
template <typename T>
__device__ __forceinline__ void st_stream(T *p, T v) {
  __builtin_nontemporal_store(v, p);
}
template <>
__device__ __forceinline__ void st_stream<float2>(float2 *p, float2 v) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  f2v w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<f2v *>(p));
}
template <>
__device__ __forceinline__ void st_stream<double2>(double2 *p, double2 v) {
  typedef double d2v __attribute__((ext_vector_type(2)));
  d2v w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<d2v *>(p));
}

template <typename T>
__device__ __forceinline__ T *cshift(T *p, int cell, long long cs) {
  using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  const long long off = p ? (long long)cell * cs : 0;  // NULL stays NULL
  return reinterpret_cast<T *>(reinterpret_cast<Byte *>(p) + off);
}

enum StatusCode { ST_OK = 0, ST_INVALID = 1, ST_NOT_CONVERGED = 4, ST_BREAKDOWN = 5 };

// Per-iteration CG history (alpha_k, beta_k, ||r_k||) of a cell, or NULLs.
struct History {
  double *alpha, *beta, *res;
};

__device__ __forceinline__ void shift_hist(History &h, int cell, long long cs) {
  h.alpha = cshift(h.alpha, cell, cs);
  h.beta = cshift(h.beta, cell, cs);
  h.res = cshift(h.res, cell, cs);
}

// CG scalars kept on the device so that the whole loop runs without host
// round trips; written by the single-block control kernels and by the last
// block of a kernel that runs a fused control step.
struct CgState {
  double rz;        // r_k . z_k
  double pq;        // p_k . K p_k
  double alpha;     // alpha_k (also the pending u update factor)
  double beta;      // beta_k
  double rr;        // ||r_k||^2
  double tol2;      // stopping threshold on ||r_k||^2
  double rr0;       // ||r_0||^2 of the current loop (host-side stop prediction)
  double tolr;      // stopping threshold as a fraction of ||f|| (either rule)
  int iter;         // completed updates of u
  int maxit;
  int done;         // 1 once stopped (later kernels of the loop return at once)
  int status;       // jfft_status value at stop
  int first;        // 1 until the first search direction exists
  int pending;      // 1 while alpha * p is owed to u
  int hist_cap;     // history capacity (0 = off)
  int parity;       // parity of the loop iteration that wrote the latest p
  // solve-level state (one per cell of a batch)
  double fnorm2;    // ||f||^2
  double fabs2;     // ||f_abs||^2 (scale of the homogeneous-material test)
  double rn;        // ||r||, FP64 refinement residual of the current sweep
  double rn_prev;   // ||r|| of the previous sweep (the scale of its FP32 vectors)
  int homog;        // 1 if f vanishes to rounding: u = 0 after zero iterations
  int outer_done;   // refinement finished (mixed precision)
  int outer;        // refinement sweeps taken
  int total_iters;  // inner iterations over all sweeps
  int final_status; // jfft_status of the whole solve
  int arrive[3];    // arrival counters of the fused control steps (alpha, ||r||^2, beta); 0 between launches
};

// Fourier tables of one axis for the Green symbol of K_ref (Q1 elements,
// exact 2-point Gauss integration): a = (2 - 2 cos t)/h = 4 sin^2(t/2)/h,
// b = h (2 + cos t)/3, s = sin t, t = 2 pi k / n.
struct AxisTables {
  const double *a, *b, *s;
};

// Division by a run-time constant d >= 1 through a multiply and a shift
// (Granlund and Montgomery's method for invariant divisors): with
// l = ceil(log2 d) and M = floor(2^32 (2^l - d) / d) + 1,
// floor(n / d) = (umulhi(n, M) + n) >> l for 0 <= n < 2^31.  Integer division
// by a run-time value is a long instruction sequence on the GPU; the FFT
// index math divides by stage lengths, sub-transform sizes and row lengths.
struct FastDiv {
  unsigned mul;
  int shift;
  int d;
  __host__ __device__ FastDiv() : mul(1), shift(0), d(1) {}
  __host__ explicit FastDiv(int divisor) : d(divisor) {
    shift = 0;
    while ((1LL << shift) < divisor) ++shift;
    mul = (unsigned)(((1ULL << 32) * ((1ULL << shift) - (unsigned long long)divisor)) /
                         (unsigned long long)divisor +
                     1ULL);
  }
  __device__ __forceinline__ int div(int n) const {
    return (int)((__umulhi((unsigned)n, mul) + (unsigned)n) >> shift);
  }
  __device__ __forceinline__ int mod(int n) const { return n - div(n) * d; }
};

constexpr int kMaxStages = 12;
struct FftPlan {
  int L;      // transform length
  int nst;    // number of Stockham stages
  int radix[kMaxStages];
  FastDiv mdiv[kMaxStages];  // L / radix of each stage
  FastDiv pdiv[kMaxStages];  // product of the earlier radices
};

// Geometry and constants passed by value to kernels.
struct GridDev {
  int dim;
  int nx, ny, nz;     // nz = 1 in 2D
  long long N;        // nodes = elements
  int mx;             // nx / 2 + 1 half-spectrum entries per x row
  double ihx, ihy, ihz;  // 1 / h
  double w;           // Gauss weight = element volume / 2^d
  double vol;         // |Y|
};

// Kernel identifiers for timing.
enum KernelId {
  KID_STIFF_CG = 0,
  KID_STIFF_APPLY,
  KID_STIFF_COMB,
  KID_XFWD,
  KID_YFWD,
  KID_GREEN,
  KID_YINV,
  KID_XINV,
  KID_DIAGPC,
  KID_CTRL,
  KID_RHS,
  KID_VEC,
  KID_REDUCE,
  KID_STRESS,
  KID_SETUP,
  KID_COUNT
};
extern const char *const kKernelNames[KID_COUNT];

}  // namespace jfft
