// FFT passes of the Green-Jacobi preconditioner
//     z = J^1/2 F^-1 G^ F J^1/2 r      (Sec. 3.3, eq. prec_lin_systemJG_2)
// on the half spectrum of the real fields (x is the real-to-complex axis).
//
// Every pass keeps a tile of lines in LDS and runs a self-sorting
// mixed-radix Stockham FFT (radices 2, 3, 4, 5, 8) on it:
//   x pass   : real rows of n points -> complex rows of n/2 points (two real
//              samples per complex value), Stockham FFT, then the split into
//              the n/2 + 1 half-spectrum bins.  Fused: r <- r - alpha q,
//              ||r||^2, the J^1/2 scaling.  The inverse x pass undoes it and
//              fuses the outer J^1/2 scaling and the r.z partial sums.
//   y pass   : strided C2C along y on tiles of W consecutive x bins.
//   last axis: C2C along z (3D) or y (2D), the d x d Green multiply at every
//              frequency of the tile (held in registers for all components),
//              and the inverse C2C, in one kernel (one spectrum round trip
//              instead of three).
// The transforms are unnormalised; 1/N is folded into G^.
#pragma once
#include "jfft_common.h"
#include "stencil.h"

namespace jfft {

constexpr int FFT_THREADS = 256;
// max complex points per thread in one tile (2048 per 256-thread block)
template <typename Real>
struct MaxPt {
  static constexpr int value = 8;
};

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b) {
  C r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C>
__device__ __forceinline__ C mul_mi(C a) {
  C r;
  if (INV) {
    r.x = -a.y;
    r.y = a.x;
  } else {
    r.x = a.y;
    r.y = -a.x;
  }
  return r;
}

// In-register DFT of R points, forward (exp(-2 pi i jk/R)) or inverse (+).
template <typename Real, int R, bool INV>
struct Dft;

template <typename Real, bool INV>
struct Dft<Real, 2, INV> {
  using C = typename CxT<Real>::T;
  __device__ __forceinline__ static void run(C *v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename Real, bool INV>
struct Dft<Real, 4, INV> {
  using C = typename CxT<Real>::T;
  __device__ __forceinline__ static void run(C *v) {
    C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    C s13 = cadd(v[1], v[3]), d13 = mul_mi<INV>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  }
};

template <typename Real, bool INV>
struct Dft<Real, 8, INV> {
  using C = typename CxT<Real>::T;
  __device__ __forceinline__ static void run(C *v) {
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Dft<Real, 4, INV>::run(e);
    Dft<Real, 4, INV>::run(o);
    const Real r = (Real)0.70710678118654752440084436210485;
    // o[k] *= w8^k, w8 = exp(-+ 2 pi i / 8)
    C t1, t3;
    if (!INV) {
      t1.x = r * (o[1].x + o[1].y);
      t1.y = r * (o[1].y - o[1].x);
      t3.x = r * (o[3].y - o[3].x);
      t3.y = -r * (o[3].x + o[3].y);
    } else {
      t1.x = r * (o[1].x - o[1].y);
      t1.y = r * (o[1].y + o[1].x);
      t3.x = -r * (o[3].x + o[3].y);
      t3.y = r * (o[3].x - o[3].y);
    }
    C t2 = mul_mi<INV>(o[2]);
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], t1);
    v[5] = csub(e[1], t1);
    v[2] = cadd(e[2], t2);
    v[6] = csub(e[2], t2);
    v[3] = cadd(e[3], t3);
    v[7] = csub(e[3], t3);
  }
};

template <typename Real, bool INV>
struct Dft<Real, 3, INV> {
  using C = typename CxT<Real>::T;
  __device__ __forceinline__ static void run(C *v) {
    const Real h = (Real)0.5, s = (Real)0.86602540378443864676372317075294;
    C t1 = cadd(v[1], v[2]);
    C t2 = csub(v[1], v[2]);
    C m;
    m.x = v[0].x - h * t1.x;
    m.y = v[0].y - h * t1.y;
    C j = mul_mi<INV>(t2);  // -+ i (v1 - v2)
    j.x *= s;
    j.y *= s;
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, j);
    v[2] = csub(m, j);
  }
};

template <typename Real, bool INV>
struct Dft<Real, 5, INV> {
  using C = typename CxT<Real>::T;
  __device__ __forceinline__ static void run(C *v) {
    const Real c1 = (Real)0.30901699437494742410229341718282;   // cos 2pi/5
    const Real c2 = (Real)-0.80901699437494742410229341718282;  // cos 4pi/5
    const Real s1 = (Real)0.95105651629515357211643933337938;   // sin 2pi/5
    const Real s2 = (Real)0.58778525229247312916870595463907;   // sin 4pi/5
    C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    C t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    C a1, a2, b1, b2;
    a1.x = v[0].x + c1 * t1.x + c2 * t2.x;
    a1.y = v[0].y + c1 * t1.y + c2 * t2.y;
    a2.x = v[0].x + c2 * t1.x + c1 * t2.x;
    a2.y = v[0].y + c2 * t1.y + c1 * t2.y;
    C u1, u2;
    u1.x = s1 * t3.x + s2 * t4.x;
    u1.y = s1 * t3.y + s2 * t4.y;
    u2.x = s2 * t3.x - s1 * t4.x;
    u2.y = s2 * t3.y - s1 * t4.y;
    b1 = mul_mi<INV>(u1);
    b2 = mul_mi<INV>(u2);
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};

// One Stockham stage of radix R on T lines of length L held in LDS:
// element (point p, line c) at buf[p * sp + c * sc].  Stage input stride
// L / R, current sub-transform length p (product of earlier radices).
// tw[j * tws] = exp(-2 pi i j / L).  All threads read their butterflies,
// synchronise, then write, so one buffer suffices.
// NPT bounds the points per thread (L * W <= NPT * NT, NT = threads).  mdv
// and pdv divide by m = L / R and by p; the divisions by W (tile lines, a
// constant where the caller's W is one) stay plain.
template <typename Real, int R, bool INV, int NPT, int NT>
__device__ __forceinline__ void stockham_stage(typename CxT<Real>::T *buf, int L, int W, int p,
                                               int sp, int sc, const typename CxT<Real>::T *tw,
                                               int tws, bool i_fastest, const FastDiv &mdv,
                                               const FastDiv &pdv) {
  using C = typename CxT<Real>::T;
  constexpr int MB = (NPT + R - 1) / R;
  const int m = mdv.d;
  const int nb = m * W;
  const int step = L / (p * R);
  C v[MB][R];
  int iv[MB], cv[MB];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int f = threadIdx.x + b * NT;
    int i, c;
    if (i_fastest) {
      c = mdv.div(f);
      i = f - c * m;
    } else {
      i = f / W;
      c = f - i * W;
    }
    iv[b] = i;
    cv[b] = c;
    if (f < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[(i + r * m) * sp + c * sc];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int f = threadIdx.x + b * NT;
    if (f < nb) {
      const int i = iv[b], c = cv[b];
      const int ip = pdv.div(i);
      const int k = i - ip * p;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C t = tw[(r * k * step) * tws];
        if (INV) t.y = -t.y;
        v[b][r] = cmul(v[b][r], t);
      }
      Dft<Real, R, INV>::run(v[b]);
      const int j = ip * p * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(j + r * p) * sp + c * sc] = v[b][r];
    }
  }
  __syncthreads();
}

template <typename Real, bool INV, int NPT = MaxPt<Real>::value, int NT = FFT_THREADS>
__device__ void lds_fft(typename CxT<Real>::T *buf, const FftPlan &pl, int W, int sp, int sc,
                        const typename CxT<Real>::T *tw, int tws, bool i_fastest) {
  int p = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.radix[s];
    switch (R) {
      case 8: stockham_stage<Real, 8, INV, NPT, NT>(buf, pl.L, W, p, sp, sc, tw, tws, i_fastest, pl.mdiv[s], pl.pdiv[s]); break;
      case 4: stockham_stage<Real, 4, INV, NPT, NT>(buf, pl.L, W, p, sp, sc, tw, tws, i_fastest, pl.mdiv[s], pl.pdiv[s]); break;
      case 2: stockham_stage<Real, 2, INV, NPT, NT>(buf, pl.L, W, p, sp, sc, tw, tws, i_fastest, pl.mdiv[s], pl.pdiv[s]); break;
      case 3: stockham_stage<Real, 3, INV, NPT, NT>(buf, pl.L, W, p, sp, sc, tw, tws, i_fastest, pl.mdiv[s], pl.pdiv[s]); break;
      case 5: stockham_stage<Real, 5, INV, NPT, NT>(buf, pl.L, W, p, sp, sc, tw, tws, i_fastest, pl.mdiv[s], pl.pdiv[s]); break;
      default: break;
    }
    p *= R;
  }
}

// The same transform with the length L and the line count W known at compile
// time, for W lines held as buf[p * W + c] (the y and last-axis passes).
// The radices are those factor_plan picks (8 first, then 4, 2, 3, 5), so the
// arithmetic, and the result, are those of lds_fft; what changes is that
// the index math (divisions by W, p and L / R, the twiddle strides) reduces
// to shifts and constants, the stage loop and its radix switch unroll, and
// the first stage skips its unit twiddles.
constexpr int ct_radix(int rem) {
  return rem % 8 == 0 ? 8 : (rem % 4 == 0 ? 4 : (rem % 2 == 0 ? 2 : (rem % 3 == 0 ? 3 : 5)));
}

template <typename Real, int R, bool INV, int NT, int L, int P, int W>
__device__ __forceinline__ void stockham_stage_ct(typename CxT<Real>::T *buf,
                                                  const typename CxT<Real>::T *tw) {
  using C = typename CxT<Real>::T;
  constexpr int M = L / R;
  constexpr int NB = M * W;                 // butterflies of the stage
  constexpr int MB = (NB + NT - 1) / NT;    // per thread
  constexpr int STEP = L / (P * R);
  C v[MB][R];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int f = (int)threadIdx.x + b * NT;
    const int i = f / W, c = f % W;
    if (NB % NT == 0 || f < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[(i + r * M) * W + c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int f = (int)threadIdx.x + b * NT;
    if (NB % NT == 0 || f < NB) {
      const int i = f / W, c = f % W;
      const int ip = i / P, k = i % P;
      if (P > 1) {  // the first stage's twiddles are all exp(0) = 1
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C t = tw[r * k * STEP];
          if (INV) t.y = -t.y;
          v[b][r] = cmul(v[b][r], t);
        }
      }
      Dft<Real, R, INV>::run(v[b]);
      const int j = ip * P * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(j + r * P) * W + c] = v[b][r];
    }
  }
  __syncthreads();
}

template <typename Real, bool INV, int NT, int L, int W, int P = 1>
__device__ __forceinline__ void lds_fft_ct(typename CxT<Real>::T *buf,
                                           const typename CxT<Real>::T *tw) {
  if constexpr (P < L) {
    constexpr int R = ct_radix(L / P);
    stockham_stage_ct<Real, R, INV, NT, L, P, W>(buf, tw);
    lds_fft_ct<Real, INV, NT, L, W, P * R>(buf, tw);
  }
}

// W lines of length L at buf[p * W + c]: the compile-time transform for the
// common lengths, else the plan's.
template <typename Real, bool INV, int NPT, int NT, int W>
__device__ __forceinline__ void lds_fft_lines(typename CxT<Real>::T *buf, const FftPlan &pl,
                                              const typename CxT<Real>::T *tw) {
  if (pl.L == 256 && 256 * W <= NPT * NT)
    lds_fft_ct<Real, INV, NT, 256, W>(buf, tw);
  else if (pl.L == 128 && 128 * W <= NPT * NT)
    lds_fft_ct<Real, INV, NT, 128, W>(buf, tw);
  else if (pl.L == 512 && 512 * W <= NPT * NT)
    lds_fft_ct<Real, INV, NT, 512, W>(buf, tw);
  else
    lds_fft<Real, INV, NPT, NT>(buf, pl, W, W, 1, tw, 1, false);
}

// The x passes' layout: W rows (a run-time count) of a compile-time length
// L, row c at buf[c * (L + 1) + i], twiddles of the 2L-point table at
// stride 2.  Same stages and arithmetic as lds_fft with i_fastest.
template <typename Real, int R, bool INV, int NPT, int NT, int L, int P>
__device__ __forceinline__ void stockham_stage_rows_ct(typename CxT<Real>::T *buf, int W,
                                                       const typename CxT<Real>::T *tw) {
  using C = typename CxT<Real>::T;
  constexpr int M = L / R;
  constexpr int SC = L + 1;
  constexpr int MB = (NPT + R - 1) / R;
  constexpr int STEP = L / (P * R);
  const int nb = M * W;
  C v[MB][R];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int f = (int)threadIdx.x + b * NT;
    const int c = f / M, i = f % M;
    if (f < nb) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[i + r * M + c * SC];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int f = (int)threadIdx.x + b * NT;
    if (f < nb) {
      const int c = f / M, i = f % M;
      const int ip = i / P, k = i % P;
      if (P > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C t = tw[(r * k * STEP) * 2];
          if (INV) t.y = -t.y;
          v[b][r] = cmul(v[b][r], t);
        }
      }
      Dft<Real, R, INV>::run(v[b]);
      const int j = ip * P * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[j + r * P + c * SC] = v[b][r];
    }
  }
  __syncthreads();
}

template <typename Real, bool INV, int NPT, int NT, int L, int P = 1>
__device__ __forceinline__ void lds_fft_rows_ct(typename CxT<Real>::T *buf, int W,
                                                const typename CxT<Real>::T *tw) {
  if constexpr (P < L) {
    constexpr int R = ct_radix(L / P);
    stockham_stage_rows_ct<Real, R, INV, NPT, NT, L, P>(buf, W, tw);
    lds_fft_rows_ct<Real, INV, NPT, NT, L, P * R>(buf, W, tw);
  }
}

// W rows of the x passes: the compile-time transform for the common half
// lengths, else the plan's.
template <typename Real, bool INV, int NPT = MaxPt<Real>::value, int NT = FFT_THREADS>
__device__ __forceinline__ void lds_fft_rows(typename CxT<Real>::T *buf, const FftPlan &pl,
                                             int W, const typename CxT<Real>::T *tw) {
  if (pl.L == 128)
    lds_fft_rows_ct<Real, INV, NPT, NT, 128>(buf, W, tw);
  else if (pl.L == 256)
    lds_fft_rows_ct<Real, INV, NPT, NT, 256>(buf, W, tw);
  else if (pl.L == 64)
    lds_fft_rows_ct<Real, INV, NPT, NT, 64>(buf, W, tw);
  else
    lds_fft<Real, INV, NPT, NT>(buf, pl, W, 1, pl.L + 1, tw, 2, true);
}

// Half-spectrum layout, tile-major: [d][nz][ntx][ny][TW] complex, where the
// mx = nx/2 + 1 bins of an x row are cut into ntx tiles of TW = 8 bins.  A
// y-pass tile (component, z, x-tile) is then one contiguous block, the x
// passes read and write contiguous (rows x TW) chunks, and the z pass reads
// whole 128-byte lines: one ky row of a tile in FP64, two adjacent ones in
// FP32 (ZRows).  The bins past mx in the last tile are zero.
template <typename Real>
struct TileW {
  static constexpr int value = 8;  // the x-pass index math below shifts by 3
};
template <typename Real>
struct ZRows {
  static constexpr int value = 128 / (TileW<Real>::value * (int)sizeof(typename CxT<Real>::T));
};

template <typename Real>
__device__ __forceinline__ void load_twiddles(typename CxT<Real>::T *sm, const double2 *g, int n) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    typename CxT<Real>::T t;
    t.x = (Real)g[j].x;
    t.y = (Real)g[j].y;
    sm[j] = t;
  }
}

// ------------------------------------------------------------ x passes ---
template <typename Real>
struct XArgs {
  Real *r;             // residual (updated in place when UPDATE)
  const Real *q;       // K p (UPDATE)
  const Real *Jh;      // J^1/2 [d][N] (USE_J)
  Real *out;           // inverse pass: z
  typename CxT<Real>::T *spec;  // half spectrum, tile-major (see TileW)
  double *partA;       // ||r||^2 partials (forward), r.z partials (inverse)
  const CgState *st;
  CgState *ctl;        // forward pass in the loop: the same state when the ||r||^2 step is fused
  History h;
  const double2 *tw;   // exp(-2 pi i j / nx), j < nx
  FftPlan plan;        // length nx / 2
  int nx, mx, ntx, ny;
  long long nrows;     // d * ny * nz rows per cell
  int rows_per_block;  // RB, a power of two
  int log2_rb;
  FastDiv dm;          // m = nx / 2
  FastDiv dhalf;       // m / 2 + 1 slot pairs per row
  int check_done;
  long long cs;        // bytes between the cells of a batch (cell = blockIdx.y)
};

// Tile-major addressing of the RB consecutive x rows of one block, rows
// row0 + row = plane * ny + y: one 64-bit division per block, then 32-bit
// steps (a block's rows may run into the next planes when ny < RB).
template <int TW>
struct RowTiles {
  long long pl0;
  int y0, ny, ntx;
  __device__ __forceinline__ RowTiles(long long row0, int ny_, int ntx_) : ny(ny_), ntx(ntx_) {
    pl0 = row0 / ny;
    y0 = (int)(row0 - pl0 * ny);
  }
  __device__ __forceinline__ long long offset(int row, int kt, int w) const {
    int y = y0 + row;
    int dp = 0;
    if (y >= ny) {
      dp = y / ny;
      y -= dp * ny;
    }
    return (((pl0 + dp) * ntx + kt) * ny + y) * TW + w;
  }
};

// Forward: r <- r - alpha q (UPDATE), s = J^1/2 r (USE_J), X = rfft(s) per row.
template <typename Real, bool UPDATE, bool USE_J>
__global__ void __launch_bounds__(FFT_THREADS) k_xfwd(XArgs<Real> a) {
  using C = typename CxT<Real>::T;
  using R2 = typename CxT<Real>::R2;
  // cell pointers as locals (see cshift)
  const int cell = blockIdx.y;
  Real *const r = cshift(a.r, cell, a.cs);
  const Real *const q = cshift(a.q, cell, a.cs);
  const Real *const Jh = cshift(a.Jh, cell, a.cs);
  Real *const out = cshift(a.out, cell, a.cs);
  C *const spec = cshift(a.spec, cell, a.cs);
  double *const partA = cshift(a.partA, cell, a.cs);
  const CgState *const st = cshift(a.st, cell, a.cs);
  (void)q;
  (void)out;
  if (a.check_done && st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *buf = tw + a.nx;
  __shared__ double red[8];
  const int m = a.nx / 2;
  const int RB = a.rows_per_block;
  const int sc = m + 1;  // LDS row stride
  const long long row0 = (long long)blockIdx.x * RB;
  load_twiddles<Real>(tw, a.tw, a.nx);
  Real alpha = 0;
  if (UPDATE) alpha = (Real)st->alpha;
  double rr = 0.0;
  // The block's RB rows are one contiguous run of RB * m pairs.  All loads
  // are issued before any is used (fixed, unrolled slots), so that a thread
  // has its whole share in flight at once.
  constexpr int XP = MaxPt<Real>::value;  // RB * m <= XP * FFT_THREADS
  const int tot = RB * m;
  const long long base = row0 * m;
  const long long lim = a.nrows * (long long)m;
  // Loads are unconditional at clamped (valid) offsets: a predicated load
  // makes the compiler wait for it at once.
  R2 rv[XP], qv[XP], jv[XP];
#pragma unroll
  for (int j = 0; j < XP; ++j) {
    const int f = threadIdx.x + j * FFT_THREADS;
    const long long off = min(base + min(f, tot - 1), lim - 1);
    rv[j] = reinterpret_cast<const R2 *>(r)[off];
    if (UPDATE) qv[j] = reinterpret_cast<const R2 *>(q)[off];
    if (USE_J) jv[j] = reinterpret_cast<const R2 *>(Jh)[off];
  }
#pragma unroll
  for (int j = 0; j < XP; ++j) {
    const int f = threadIdx.x + j * FFT_THREADS;
    if (f >= tot) continue;
    const long long off = base + f;
    C z;
    z.x = 0;
    z.y = 0;
    if (off < lim) {
      R2 v = rv[j];
      if (UPDATE) {
        v.x -= alpha * qv[j].x;
        v.y -= alpha * qv[j].y;
        st_stream(reinterpret_cast<R2 *>(r) + off, v);
      }
      rr += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
      if (USE_J) {
        v.x *= jv[j].x;
        v.y *= jv[j].y;
      }
      z.x = v.x;
      z.y = v.y;
    }
    const int fr = a.dm.div(f);
    buf[fr * sc + (f - fr * m)] = z;
  }
  __syncthreads();
  lds_fft_rows<Real, false>(buf, a.plan, RB, tw);
  // split X[k] = (Z[k] + conj Z[m-k])/2 - i w^k (Z[k] - conj Z[m-k])/2 (Z
  // indices mod m; k = m is the Nyquist bin), evaluated bin by bin in the
  // order of the tile-major stores: a run of RB x TW consecutive complex
  // values per x-tile; bins past mx are written as zero
  {
    constexpr int TW = TileW<Real>::value;
    static_assert(TW == 8, "tile-major x-pass addressing assumes 8 bins per tile");
    constexpr int SP = XP + 2;  // RB * ntx * TW <= RB * (m + TW) <= SP * FFT_THREADS
    const RowTiles<TW> rt(row0, a.ny, a.ntx);
    // bin kx of a row: Z slots kx mod m and (m - kx) mod m (kx <= m)
    auto split = [&](const C *zrow, int kx) {
      C X;
      X.x = 0;
      X.y = 0;
      if (kx < a.mx) {
        const C zk = zrow[kx == m ? 0 : kx], zm = zrow[kx == 0 ? 0 : m - kx];
        C sm, d;
        sm.x = (Real)0.5 * (zk.x + zm.x);
        sm.y = (Real)0.5 * (zk.y - zm.y);
        d.x = (Real)0.5 * (zk.x - zm.x);
        d.y = (Real)0.5 * (zk.y + zm.y);
        const C wd = cmul(tw[kx], d);  // -i w^k d
        X.x = sm.x + wd.y;
        X.y = sm.y - wd.x;
      }
      return X;
    };
    if (a.log2_rb <= 5) {
      // RB <= 32: a thread keeps its row and bin lane in every slot, and the
      // x-tile steps by 32 / RB, so the address is one increment per slot
      const int w = threadIdx.x & (TW - 1);
      const int row = (threadIdx.x >> 3) & (RB - 1);
      const int kt0 = threadIdx.x >> (3 + a.log2_rb), dkt = 32 >> a.log2_rb;
      if (row0 + row < a.nrows) {
        C *dst = spec + rt.offset(row, kt0, w);
        const long long step = (long long)dkt * a.ny * TW;
        const C *zrow = buf + row * sc;
#pragma unroll
        for (int j = 0; j < SP; ++j) {
          const int kt = kt0 + j * dkt;
          if (kt < a.ntx) st_stream(dst + j * step, split(zrow, kt * TW + w));
        }
      }
    } else {
      const int tot = (a.ntx * TW) << a.log2_rb;
#pragma unroll
      for (int j = 0; j < SP; ++j) {
        const int f = threadIdx.x + j * FFT_THREADS;
        const int w = f & (TW - 1), row = (f >> 3) & (RB - 1), kt = f >> (3 + a.log2_rb);
        if (f >= tot || row0 + row >= a.nrows) continue;
        st_stream(spec + rt.offset(row, kt, w), split(buf + row * sc, kt * TW + w));
      }
    }
  }
  const double s = block_sum<FFT_THREADS>(rr, red);
  if (threadIdx.x == 0 && partA) partA[blockIdx.x] = s;
  if (a.ctl)
    fused_ctrl<FFT_THREADS, CTRL_RR>(cshift(a.ctl, cell, a.cs), partA, gridDim.x, a.h, cell,
                                     a.cs, 0, red);
}

// Inverse: t = irfft(X) (unnormalised), z = J^1/2 t (USE_J).  (r.z is
// formed in the Green pass, so r is not read here.)
template <typename Real, bool USE_J>
__global__ void __launch_bounds__(FFT_THREADS) k_xinv(XArgs<Real> a) {
  using C = typename CxT<Real>::T;
  using R2 = typename CxT<Real>::R2;
  // cell pointers as locals (see cshift)
  const int cell = blockIdx.y;
  const Real *const Jh = cshift(a.Jh, cell, a.cs);
  Real *const out = cshift(a.out, cell, a.cs);
  C *const spec = cshift(a.spec, cell, a.cs);
  const CgState *const st = cshift(a.st, cell, a.cs);
  if (a.check_done && st->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  C *buf = tw + a.nx;
  const int m = a.nx / 2;
  const int RB = a.rows_per_block;
  const int sc = m + 1;
  const long long row0 = (long long)blockIdx.x * RB;
  load_twiddles<Real>(tw, a.tw, a.nx);
  // spectrum chunks (RB x TW per x-tile): all loads in flight at once (fixed,
  // unrolled slots at clamped, valid positions)
  constexpr int XP = MaxPt<Real>::value;  // RB * m <= XP * FFT_THREADS
  constexpr int TW = TileW<Real>::value;
  static_assert(TW == 8, "tile-major x-pass addressing assumes 8 bins per tile");
  constexpr int SP = XP + 2;              // RB * ntx * TW <= RB * (m + TW) <= SP * FFT_THREADS
  {
    const RowTiles<TW> rt(row0, a.ny, a.ntx);
    const int last_row = (int)min((long long)RB - 1, a.nrows - 1 - row0);
    C sv[SP];
    if (a.log2_rb <= 5) {
      // RB <= 32: fixed row and bin lane per thread, x-tile step 32 / RB
      const int w = threadIdx.x & (TW - 1);
      const int row = (threadIdx.x >> 3) & (RB - 1);
      const int kt0 = threadIdx.x >> (3 + a.log2_rb), dkt = 32 >> a.log2_rb;
      const C *src = spec + rt.offset(min(row, last_row), 0, w);
      const long long tstep = (long long)a.ny * TW;
#pragma unroll
      for (int j = 0; j < SP; ++j)  // unconditional loads at clamped (valid) tiles
        sv[j] = src[min(kt0 + j * dkt, a.ntx - 1) * tstep];
      const bool rowok = row0 + row < a.nrows;
#pragma unroll
      for (int j = 0; j < SP; ++j) {
        const int kt = kt0 + j * dkt, kx = kt * TW + w;
        if (kt < a.ntx && kx <= m) {
          C v = sv[j];
          if (!rowok) v.x = v.y = 0;
          buf[row * sc + kx] = v;
        }
      }
    } else {
      const int tot = (a.ntx * TW) << a.log2_rb;
#pragma unroll
      for (int j = 0; j < SP; ++j) {
        const int f = min((int)threadIdx.x + j * FFT_THREADS, tot - 1);
        const int w = f & (TW - 1), row = min((f >> 3) & (RB - 1), last_row), kt = f >> (3 + a.log2_rb);
        sv[j] = spec[rt.offset(row, kt, w)];
      }
#pragma unroll
      for (int j = 0; j < SP; ++j) {
        const int f = threadIdx.x + j * FFT_THREADS;
        const int w = f & (TW - 1), row = (f >> 3) & (RB - 1), kt = f >> (3 + a.log2_rb);
        const int kx = kt * TW + w;
        if (f < tot && kx <= m) {
          C v = sv[j];
          if (row0 + row >= a.nrows) v.x = v.y = 0;
          buf[row * sc + kx] = v;
        }
      }
    }
  }
  // J^1/2 for the epilogue: in flight during the transform
  const int tot = RB * m;
  const long long base = row0 * m;
  const long long lim = a.nrows * (long long)m;
  R2 jv[XP];
#pragma unroll
  for (int j = 0; j < XP; ++j) {  // unconditional loads at clamped (valid) offsets
    const int f = threadIdx.x + j * FFT_THREADS;
    const long long off = min(base + min(f, tot - 1), lim - 1);
    if (USE_J) jv[j] = reinterpret_cast<const R2 *>(Jh)[off];
  }
  __syncthreads();
  // Z[k] = (X[k] + conj X[m-k]) + i conj(w^k) (X[k] - conj X[m-k]), k < m.
  // A thread owns the pair (k, m - k) of one row: it reads and writes only
  // those two slots, so no barrier is needed inside the loop.
  // (Straight-line code: a small array indexed by a run-time count would be
  // placed in per-lane scratch memory.)
  const int half = m / 2 + 1;
  auto unsplit = [&](C xk, C xm, int q) {
    C e, d;
    e.x = xk.x + xm.x;
    e.y = xk.y - xm.y;
    d.x = xk.x - xm.x;
    d.y = xk.y + xm.y;
    C wc = tw[q];
    wc.y = -wc.y;
    const C o = cmul(wc, d);
    C z;
    z.x = e.x - o.y;  // e + i o
    z.y = e.y + o.x;
    return z;
  };
  for (int f = threadIdx.x; f < RB * half; f += FFT_THREADS) {
    const int row = a.dhalf.div(f), k = f - row * half;
    const C xa = buf[row * sc + k];
    const C xb = buf[row * sc + (m - k)];
    const C z0 = unsplit(xa, xb, k);
    // the partner slot m - k, unless it is k itself or k = 0 (no Z[m])
    const bool two = k != 0 && 2 * k != m;
    C z1 = z0;
    if (two) z1 = unsplit(xb, xa, m - k);
    buf[row * sc + k] = z0;
    if (two) buf[row * sc + (m - k)] = z1;
  }
  __syncthreads();
  lds_fft_rows<Real, true>(buf, a.plan, RB, tw);
#pragma unroll
  for (int j = 0; j < XP; ++j) {
    const int f = threadIdx.x + j * FFT_THREADS;
    const long long off = base + f;
    if (f >= tot || off >= lim) continue;
    const int fr = a.dm.div(f);
    const C z = buf[fr * sc + (f - fr * m)];
    R2 t;
    t.x = z.x;
    t.y = z.y;
    if (USE_J) {
      t.x *= jv[j].x;
      t.y *= jv[j].y;
    }
    st_stream(reinterpret_cast<R2 *>(out) + off, t);
  }
}

// ------------------------------------------------- strided C2C passes ----
template <typename Real>
struct YArgs {
  typename CxT<Real>::T *spec;
  const CgState *st;
  const double2 *tw;  // exp(-2 pi i j / L)
  FftPlan plan;
  int ntx, ny, nz;
  int check_done;
  long long cs;  // bytes between the cells of a batch (cell = blockIdx.z)
};

// C2C along y on tiles (component, z, x-tile) of ny points x TW bins, each one
// contiguous block of the tile-major spectrum.  Blocks are persistent over
// tiles; the next tile's loads are in flight in registers while the current
// tile is transformed in LDS.  ny * TW <= MaxPt * NT.
template <typename Real, bool INV, int NT>
__global__ void __launch_bounds__(NT) k_ypass(YArgs<Real> a) {
  using C = typename CxT<Real>::T;
  constexpr int PPT = MaxPt<Real>::value;
  constexpr int TW = TileW<Real>::value;
  C *const spec = cshift(a.spec, blockIdx.z, a.cs);  // a local (see cshift)
  if (a.check_done && cshift(a.st, blockIdx.z, a.cs)->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  const int L = a.ny;
  C *buf = tw + L;
  load_twiddles<Real>(tw, a.tw, L);
  const int npts = L * TW;
  const long long per_comp = (long long)a.nz * a.ntx;  // gridDim.y = components
  C *const comp_base = spec + (long long)blockIdx.y * per_comp * npts;
  // The prefetch is held as separate real and imaginary arrays: an array of
  // double-complex values here is placed in per-lane scratch memory by the
  // compiler, which doubles the pass's memory traffic.
  Real pre_re[PPT], pre_im[PPT];
  auto load = [&](long long t) {  // unconditional loads at clamped positions
    const C *base = comp_base + t * npts;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const C v = base[min((int)threadIdx.x + j * NT, npts - 1)];
      pre_re[j] = v.x;
      pre_im[j] = v.y;
    }
  };
  long long t = blockIdx.x;
  if (t < per_comp) load(t);
  for (; t < per_comp; t += gridDim.x) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int f = threadIdx.x + j * NT;
      if (f < npts) {
        C v;
        v.x = pre_re[j];
        v.y = pre_im[j];
        buf[f] = v;
      }
    }
    __syncthreads();
    if (t + gridDim.x < per_comp) load(t + gridDim.x);
    lds_fft_lines<Real, INV, PPT, NT, TW>(buf, a.plan, tw);
    C *base = comp_base + t * npts;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int f = threadIdx.x + j * NT;
      if (f < npts) {
        // the forward pass's output is read next by the Green pass and stays
        // cached; the inverse pass's output streams out (measured: the other
        // choices slow the consumer by 3-5 %)
        if (INV) st_stream(base + f, buf[f]);
        else base[f] = buf[f];
      }
    }
    __syncthreads();
  }
}

template <typename Real>
struct GArgs {
  typename CxT<Real>::T *spec;
  const CgState *st;
  CgState *ctl;       // in the loop: the same state when the beta step is fused (else NULL)
  History h;
  const double2 *tw;  // exp(-2 pi i j / L), L = length of the last axis
  FftPlan plan;
  AxisTables tx, ty, tz;  // Fourier tables of K_ref
  double lam, mu;         // reference Lame constants
  double invN;            // 1 / N (normalisation of the unnormalised transforms)
  int dim, mx, ntx, ny, nz;
  int check_done;
  long long cs;           // bytes between the cells of a batch (cell = blockIdx.z)
  double *partB;          // per-block partials of r.z (Parseval, see k_green_axis)
  // 2D linear triangles (tri != 0): K^_ref from its 3 x 3 stencil (see
  // green2_tri)
  int tri;
  double tS[9][3];
  double hx, hy;  // node spacings (the triangles' symbol reads cos - 1 off the a tables)
};

// Green multiply at one frequency: zh = G^(k) sh with G^ = K^_ref(k)^-1 / N,
// G^(0) = 0 (Alg. 1 step 3).  K^_ref of Q1 elements with exact Gauss
// integration is real symmetric:
//   K_ii = (lam + 2 mu) a_i prod_{j != i} b_j + mu sum_{j != i} a_j prod_{l != j} b_l
//   K_ij = (lam + mu) s_i s_j prod_{l != i, j} b_l
// (a = 4 sin^2(theta / 2) / h, b = h (2 + cos theta) / 3, s = sin theta per
// axis; the caller forms the entries).  The symbol is evaluated in the
// precision of the pass (T: float in the mixed path, whose spectrum is FP32;
// double otherwise).  K^_ref(k) is SPD for k != 0 with a condition number
// bounded by the Lame ratio and the symbol's anisotropy, so its cofactor
// inverse loses only a few bits.  In FP32 the reciprocal of the determinant
// is the hardware's (1 ulp), a relative change of G^ per frequency far below
// the FP32 path's own rounding.

// s / d: exact division in FP64, s times the hardware reciprocal in FP32
template <typename T>
__device__ __forceinline__ T scaled_recip(T s, T d) {
  if constexpr (sizeof(T) == 4) {
    return s * __builtin_amdgcn_rcpf(d);
  } else {
    return s / d;
  }
}

template <typename T, typename C>
__device__ __forceinline__ void green3_apply(T k00, T k11, T k22, T k01, T k02, T k12, T invN,
                                             bool zero, C (&v)[3]) {
  if (zero) {
    for (int i = 0; i < 3; ++i) v[i].x = v[i].y = 0;
    return;
  }
  // symmetric inverse by cofactors
  const T c00 = k11 * k22 - k12 * k12;
  const T c01 = k02 * k12 - k01 * k22;
  const T c02 = k01 * k12 - k02 * k11;
  const T c11 = k00 * k22 - k02 * k02;
  const T c12 = k01 * k02 - k00 * k12;
  const T c22 = k00 * k11 - k01 * k01;
  const T det = k00 * c00 + k01 * c01 + k02 * c02;
  const T sc = scaled_recip(invN, det);
  const T g00 = c00 * sc, g01 = c01 * sc, g02 = c02 * sc;
  const T g11 = c11 * sc, g12 = c12 * sc, g22 = c22 * sc;
  const T x0 = v[0].x, x1 = v[1].x, x2 = v[2].x;
  const T y0 = v[0].y, y1 = v[1].y, y2 = v[2].y;
  v[0].x = g00 * x0 + g01 * x1 + g02 * x2;
  v[0].y = g00 * y0 + g01 * y1 + g02 * y2;
  v[1].x = g01 * x0 + g11 * x1 + g12 * x2;
  v[1].y = g01 * y0 + g11 * y1 + g12 * y2;
  v[2].x = g02 * x0 + g12 * x1 + g22 * x2;
  v[2].y = g02 * y0 + g12 * y1 + g22 * y2;
}

template <typename T, typename C>
__device__ __forceinline__ void green2_apply(T k00, T k11, T k01, T invN, bool zero, C (&v)[2]) {
  if (zero) {
    for (int i = 0; i < 2; ++i) v[i].x = v[i].y = 0;
    return;
  }
  const T sc = scaled_recip(invN, k00 * k11 - k01 * k01);
  const T g00 = k11 * sc, g11 = k00 * sc, g01 = -k01 * sc;
  const T x0 = v[0].x, x1 = v[1].x, y0 = v[0].y, y1 = v[1].y;
  v[0].x = g00 * x0 + g01 * x1;
  v[0].y = g00 * y0 + g01 * y1;
  v[1].x = g01 * x0 + g11 * x1;
  v[1].y = g01 * y0 + g11 * y1;
}

// Green multiply for the 2D linear-triangle discretisation.  K_ref is the
// 3 x 3 stencil (K u)(x) = sum_d S_d u(x + d), d in {-1, 0, 1}^2, so
// K^(k) = sum_d S_d exp(i theta . d), theta = 2 pi (kx / nx, ky / ny).  The
// split of every pixel into two triangles is symmetric under the point
// reflection x -> -x, so S_-d = S_d and K^ = sum_d S_d cos(theta . d) is real
// symmetric (it is not of the separable quadrilateral form: the split is not
// symmetric under the reflection of one axis).  S[d] = (S_00, S_11, S_01) of
// offset d = (dx, dy), index (dy + 1) * 3 + dx + 1.
// Rigid translations lie in the kernel of K_ref, so sum_d S_d = 0 and
// K^ = sum_d S_d (cos(theta . d) - 1).  That form is evaluated from
// cm = cos(theta) - 1 and s = sin(theta) per axis (cm from the accurate
// 4 sin^2(theta / 2) table): every term is O(theta^2), where the plain cosine
// sum would cancel O(1) terms down to O(theta^2) and lose the low
// frequencies' accuracy (in FP32 about 1e-3 relative at the lowest
// frequency of a 512-point axis).
template <typename T, typename C>
__device__ __forceinline__ void green2_tri(T cmx, T sx, T cmy, T sy, const double (&S)[9][3],
                                           T invN, bool zero, C (&v)[2]) {
  if (zero) {
    for (int i = 0; i < 2; ++i) v[i].x = v[i].y = 0;
    return;
  }
  T k00 = 0, k11 = 0, k01 = 0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      if (dx == 0 && dy == 0) continue;  // cos(0) - 1 = 0
      // cos(theta_x dx + theta_y dy) - 1
      //   = cmx' cmy' + cmx' + cmy' - sx' sy',  cm' = cm (d != 0) or 0, s' = d s
      const T cxd = dx ? cmx : (T)0, sxd = (T)dx * sx;
      const T cyd = dy ? cmy : (T)0, syd = (T)dy * sy;
      const T cd = cxd * cyd + cxd + cyd - sxd * syd;
      const int o = (dy + 1) * 3 + dx + 1;
      k00 += (T)S[o][0] * cd;
      k11 += (T)S[o][1] * cd;
      k01 += (T)S[o][2] * cd;
    }
  green2_apply<T>(k00, k11, k01, invN, false, v);
}

// Last axis: forward C2C, Green multiply, inverse C2C for every component of
// one tile: an x-tile (TW bins) at KY adjacent ky rows along z (3D; the KY *
// TW complex values at one z are one contiguous 128-byte line for KY = 2), or
// an x-tile along y (2D, KY = 1).  The transformed components stay in
// registers for the Green multiply; the next component's loads are in flight
// while the current one is transformed.  L * KY * TW <= MaxPt * NT.
// FP32: at most 128 VGPRs (four waves per SIMD, two 512-thread blocks per
// CU); the unrolled transforms would otherwise take more and cut the
// resident blocks, which costs this pass more than the leaner index math
// saves (measured at 256^3: 174 us unbounded, 122 us bounded, 146 us with
// the run-time plan).  Not for the one-row 3D tiles of 512-point axes, which
// would spill.
template <typename Real, int DIM, int KY, int NT>
__global__ void __launch_bounds__(NT, (sizeof(Real) == 4 && !(DIM == 3 && KY == 1)) ? 4 : 1)
    k_green_axis(GArgs<Real> a) {
  using C = typename CxT<Real>::T;
  constexpr int PPT = MaxPt<Real>::value;
  constexpr int TW = TileW<Real>::value;
  constexpr int LN = KY * TW;  // lines of the tile
  C *const spec = cshift(a.spec, blockIdx.z, a.cs);  // a local (see cshift)
  if (a.check_done && cshift(a.st, blockIdx.z, a.cs)->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *tw = reinterpret_cast<C *>(smem_raw);
  const int L = DIM == 3 ? a.nz : a.ny;
  C *buf = tw + L;  // [L][LN]
  Real *tab = reinterpret_cast<Real *>(buf + L * LN);  // [L][3]: a, b, s of the transform axis
  load_twiddles<Real>(tw, a.tw, L);
  {
    const AxisTables &ta = DIM == 3 ? a.tz : a.ty;
    for (int j = threadIdx.x; j < L; j += NT) {
      tab[3 * j] = (Real)ta.a[j];
      tab[3 * j + 1] = (Real)ta.b[j];
      tab[3 * j + 2] = (Real)ta.s[j];
    }
  }
  const int kt = blockIdx.x % a.ntx;
  const int ky0 = DIM == 3 ? (int)(blockIdx.x / a.ntx) * KY : 0;
  // element (position t along the axis, line l) of component c:
  //   base[c * comp_stride + t * axis_stride + l]
  const long long comp_stride = (long long)a.nz * a.ntx * a.ny * TW;
  const long long axis_stride = DIM == 3 ? (long long)a.ntx * a.ny * TW : TW;
  C *const base = spec + (DIM == 3 ? ((long long)kt * a.ny + ky0) * TW : (long long)kt * a.ny * TW);
  const int npts = L * LN;
  // prefetch as separate real and imaginary arrays (see k_ypass)
  Real pre_re[PPT], pre_im[PPT];
  auto load = [&](int c) {  // unconditional loads at clamped positions
    const C *bc = base + c * comp_stride;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int f = min((int)threadIdx.x + j * NT, npts - 1);
      const C v = bc[(long long)(f / LN) * axis_stride + f % LN];
      pre_re[j] = v.x;
      pre_im[j] = v.y;
    }
  };
  C stash[DIM][PPT];
  load(0);
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int f = threadIdx.x + j * NT;
      if (f < npts) {
        C v;
        v.x = pre_re[j];
        v.y = pre_im[j];
        buf[f] = v;
      }
    }
    __syncthreads();
    if (c + 1 < DIM) load(c + 1);
    lds_fft_lines<Real, false, PPT, NT, LN>(buf, a.plan, tw);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int f = threadIdx.x + j * NT;
      if (f < npts) stash[c][j] = buf[f];
    }
    __syncthreads();
  }
  // Green multiply on the points this thread holds, and r.z by Parseval:
  // with s = J^1/2 r, t = F^-1 (G^ F s) and z = J^1/2 t, r.z = s.t =
  // sum over the full spectrum of conj(s^) (G^ s^) (1/N is folded into G^);
  // on the half spectrum the bins 0 < kx < nx/2 stand for their conjugate
  // partners too (weight 2), kx = 0 and kx = nx/2 for themselves (weight 1).
  // NT is a multiple of LN, so a thread's points share their line l (one kx,
  // ky) and differ only in the position t along the axis: the symbol's
  // factors of the other axes are formed once per thread, and per point only
  // the transform axis' a, b, s (staged in LDS) enter.
  static_assert(NT % LN == 0, "a thread's points must share their tile line");
  double rz = 0.0;
  const int l = threadIdx.x % LN;
  const int kxu = kt * TW + l % TW;
  const double wk = kxu >= a.mx ? 0.0 : (kxu == 0 || kxu == a.mx - 1 ? 1.0 : 2.0);
  const int kx = min(kxu, a.mx - 1);
  const Real lam = (Real)a.lam, mu = (Real)a.mu, invN = (Real)a.invN;
  const Real l2m = lam + (Real)2 * mu, lm = lam + mu;
  if constexpr (DIM == 3) {
    const int ky = ky0 + l / TW;
    const Real A0 = (Real)a.tx.a[kx], B0 = (Real)a.tx.b[kx], S0 = (Real)a.tx.s[kx];
    const Real A1 = (Real)a.ty.a[ky], B1 = (Real)a.ty.b[ky], S1 = (Real)a.ty.s[ky];
    // K^_ij as affine functions of the z factors (a2, b2, s2):
    //   k00 = c00a b2 + c00b a2, k11 = c11a b2 + c00b a2, k22 = c22a a2 + c22b b2,
    //   k01 = c01 b2, k02 = c02 s2, k12 = c12 s2
    const Real c00a = l2m * A0 * B1 + mu * B0 * A1, c00b = mu * B0 * B1;
    const Real c11a = l2m * B0 * A1 + mu * A0 * B1;
    const Real c22a = l2m * B0 * B1, c22b = mu * (A0 * B1 + B0 * A1);
    const Real c01 = lm * S0 * S1, c02 = lm * S0 * B1, c12 = lm * B0 * S1;
    const bool kxy0 = kx == 0 && ky == 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int f = threadIdx.x + j * NT;
      if (f < npts) {
        const int t = f / LN;
        const Real A2 = tab[3 * t], B2 = tab[3 * t + 1], S2 = tab[3 * t + 2];
        const Real k00 = c00a * B2 + c00b * A2, k11 = c11a * B2 + c00b * A2;
        const Real k22 = c22a * A2 + c22b * B2;
        const Real k01 = c01 * B2, k02 = c02 * S2, k12 = c12 * S2;
        C v[3] = {stash[0][j], stash[1][j], stash[2][j]};
        green3_apply<Real>(k00, k11, k22, k01, k02, k12, invN, kxy0 && t == 0, v);
        double e = 0.0;
        for (int c = 0; c < 3; ++c) {
          e += (double)stash[c][j].x * (double)v[c].x + (double)stash[c][j].y * (double)v[c].y;
          stash[c][j] = v[c];
        }
        rz += wk * e;
      }
    }
  } else {
    const Real A0 = (Real)a.tx.a[kx], B0 = (Real)a.tx.b[kx], S0 = (Real)a.tx.s[kx];
    // quadrilaterals: k00 = mu b0 a1 + l2m a0 b1, k11 = l2m b0 a1 + mu a0 b1, k01 = lm s0 s1
    const Real q00a = mu * B0, q00b = l2m * A0, q11a = l2m * B0, q11b = mu * A0, q01 = lm * S0;
    // triangles: cos(theta_x) - 1 = -a0 h / 2
    const Real cmx = (Real)(-0.5 * a.tx.a[kx] * a.hx);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int f = threadIdx.x + j * NT;
      if (f < npts) {
        const int t = f / LN;
        const Real A1 = tab[3 * t], B1 = tab[3 * t + 1], S1 = tab[3 * t + 2];
        C v[2] = {stash[0][j], stash[1][j]};
        if (a.tri) {
          const Real cmy = (Real)-0.5 * A1 * (Real)a.hy;
          green2_tri<Real>(cmx, S0, cmy, S1, a.tS, invN, kx == 0 && t == 0, v);
        } else {
          green2_apply<Real>(q00a * A1 + q00b * B1, q11a * A1 + q11b * B1, q01 * S1, invN,
                             kx == 0 && t == 0, v);
        }
        double e = 0.0;
        for (int c = 0; c < 2; ++c) {
          e += (double)stash[c][j].x * (double)v[c].x + (double)stash[c][j].y * (double)v[c].y;
          stash[c][j] = v[c];
        }
        rz += wk * e;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int f = threadIdx.x + j * NT;
      if (f < npts) buf[f] = stash[c][j];
    }
    __syncthreads();
    lds_fft_lines<Real, true, PPT, NT, LN>(buf, a.plan, tw);
    C *bc = base + c * comp_stride;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int f = threadIdx.x + j * NT;
      if (f < npts) bc[(long long)(f / LN) * axis_stride + f % LN] = buf[f];  // read next by the y pass: keep it cached
    }
    __syncthreads();
  }
  __shared__ double red[NT / 64];
  const double srz = block_sum<NT>(rz, red);
  if (threadIdx.x == 0 && a.partB) cshift(a.partB, blockIdx.z, a.cs)[blockIdx.x] = srz;
  if (a.ctl)
    fused_ctrl<NT, CTRL_BETA>(cshift(a.ctl, blockIdx.z, a.cs), cshift(a.partB, blockIdx.z, a.cs),
                              gridDim.x, a.h, blockIdx.z, a.cs, 0, red);
}

// ------------------------------------- diagonal / identity preconditioner -
// r <- r - alpha q (UPDATE), z = Jinv r (JACOBI) or z = r (NONE); partials of
// ||r||^2 (partA) and r.z (partB).
template <typename Real, bool UPDATE, bool JACOBI>
__global__ void __launch_bounds__(256) k_diag_pc(Real *r, const Real *q, const Real *Jh, Real *z,
                                                 long long n, const CgState *st, int check_done,
                                                 double *partA, double *partB, long long cs) {
  const int cell = blockIdx.y;
  r = cshift(r, cell, cs);
  q = cshift(q, cell, cs);
  Jh = cshift(Jh, cell, cs);
  z = cshift(z, cell, cs);
  st = cshift(st, cell, cs);
  partA = cshift(partA, cell, cs);
  partB = cshift(partB, cell, cs);
  if (check_done && st->done) return;
  __shared__ double red[8];
  Real alpha = 0;
  if (UPDATE) alpha = (Real)st->alpha;
  double rr = 0.0, rz = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    Real rv = r[i];
    if (UPDATE) {
      rv -= alpha * q[i];
      r[i] = rv;
    }
    Real zv = rv;
    if (JACOBI) {
      const Real j = Jh[i];
      zv = rv * j * j;
    }
    z[i] = zv;
    rr += (double)rv * (double)rv;
    rz += (double)rv * (double)zv;
  }
  const double s1 = block_sum<256>(rr, red);
  const double s2 = block_sum<256>(rz, red);
  if (threadIdx.x == 0) {
    if (partA) partA[blockIdx.x] = s1;
    if (partB) partB[blockIdx.x] = s2;
  }
}

}  // namespace jfft
