// Host driver and C ABI of the MI355X J-FFT solver (see include/jfft.h).
//
// One cell = one periodic grid on one stream.  set_material copies E, runs
// Algorithm 2 (d 2^d stiffness applications to unit combs, Sec. 3.2) on the
// device and forms J^1/2.  solve assembles f, runs the PCG loop entirely on
// the device (CG scalars live in device memory; the host only polls the stop
// flag every few iterations), then removes the mean of u (Sec. 5), recomputes
// the true residual and evaluates the stresses and sigma_bar.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "jfft.h"
#include "cg.h"
#include "fft.h"
#include "jfft_common.h"
#include "stencil.h"

namespace jfft {
const char *const kKernelNames[KID_COUNT] = {
    "stiffness_cg",  "stiffness_apply", "stiffness_comb", "fft_x_forward", "fft_y_forward",
    "fft_green_axis", "fft_y_inverse",  "fft_x_inverse",  "diag_precond",  "cg_control",
    "rhs",            "vector",         "reduce",         "stress",        "setup"};
}

using namespace jfft;

static thread_local std::string g_last_error;

static jfft_status fail(jfft_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(JFFT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));           \
  } while (0)

namespace {

constexpr int kHistMax = 4096;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool factor_plan(int L, FftPlan &pl) {
  pl.L = L;
  pl.nst = 0;
  int r = L;
  const int pref[5] = {8, 4, 2, 3, 5};
  while (r > 1) {
    bool ok = false;
    for (int k = 0; k < 5; ++k) {
      if (r % pref[k] == 0) {
        if (pl.nst >= kMaxStages) return false;
        pl.radix[pl.nst++] = pref[k];
        r /= pref[k];
        ok = true;
        break;
      }
    }
    if (!ok) return false;
  }
  return true;
}

template <typename Real>
struct PcgBufs {
  Real *u, *r, *z, *q, *p[2];
  const Real *E, *Jh;
  typename CxT<Real>::T *spec;
};

}  // namespace

struct jfft_cell_s {
  int dim = 0;
  int n[3] = {1, 1, 1};
  double len[3] = {1, 1, 1};
  jfft_precision prec = JFFT_FP64;
  jfft_precond pc = JFFT_PC_GREEN_JACOBI;
  hipStream_t stream = nullptr;
  int device = 0;
  GridDev g{};
  FftPlan plan_x{}, plan_y{}, plan_z{};
  int tz = 32;

  // workspace
  unsigned char *ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  bool ready = false;

  // FP64 buffers
  double *E = nullptr, *Jh = nullptr, *diag = nullptr, *f = nullptr, *r = nullptr, *z = nullptr,
         *q = nullptr, *p[2] = {nullptr, nullptr};
  double2 *spec = nullptr;
  // FP32 buffers (MIXED)
  float *E32 = nullptr, *Jh32 = nullptr, *r32 = nullptr, *z32 = nullptr, *q32 = nullptr,
        *p32[2] = {nullptr, nullptr}, *c32 = nullptr;
  float2 *spec32 = nullptr;
  // tables
  double2 *tw[3] = {nullptr, nullptr, nullptr};
  double *ftab[3][3] = {};
  double *F = nullptr, *macro = nullptr;
  CgState *st = nullptr;
  double *partA = nullptr, *partB = nullptr;
  long long npart = 0;
  double *small = nullptr;
  double *hist[3] = {nullptr, nullptr, nullptr};
  int hist_cap = 0;  // entries recorded per solve (<= kHistMax)

  // host pinned mirrors
  CgState *st_h = nullptr;
  double *small_h = nullptr;

  bool has_material = false;
  double lam = 0, mu = 0;
  double void_value = 1.0;
  double inner_tol = 1e-5;
  int max_outer = 30;

  // timing
  bool timing = false;
  struct Pending {
    int kid;
    hipEvent_t a, b;
  };
  std::vector<Pending> pend;
  std::vector<hipEvent_t> pool;
  double ktime[KID_COUNT] = {};
  long kcount[KID_COUNT] = {};

  hipEvent_t phase_ev[4] = {nullptr, nullptr, nullptr, nullptr};

  ~jfft_cell_s() {
    flush_timing();
    for (auto &e : pool) (void)hipEventDestroy(e);
    for (auto &e : phase_ev)
      if (e) (void)hipEventDestroy(e);
    if (ws_owned && ws) (void)hipFree(ws);
    if (st_h) (void)hipHostFree(st_h);
    if (small_h) (void)hipHostFree(small_h);
  }

  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void flush_timing() {
    if (pend.empty()) return;
    (void)hipStreamSynchronize(stream);
    for (auto &pd : pend) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess) {
        ktime[pd.kid] += ms;
        kcount[pd.kid] += 1;
      }
      pool.push_back(pd.a);
      pool.push_back(pd.b);
    }
    pend.clear();
  }
  hipEvent_t tb(int) {
    if (!timing) return nullptr;
    hipEvent_t a = get_event();
    (void)hipEventRecord(a, stream);
    return a;
  }
  void te(int kid, hipEvent_t a) {
    if (!timing || !a) return;
    hipEvent_t b = get_event();
    (void)hipEventRecord(b, stream);
    pend.push_back({kid, a, b});
    if (pend.size() >= 8192) flush_timing();
  }
};

#define LAUNCH(cell, kid, ...)                                                   \
  do {                                                                           \
    hipEvent_t _tb = (cell)->tb(kid);                                            \
    __VA_ARGS__;                                                                 \
    (cell)->te(kid, _tb);                                                        \
    hipError_t _e = hipGetLastError();                                           \
    if (_e != hipSuccess)                                                        \
      return fail(JFFT_E_HIP, std::string("launch ") + kKernelNames[kid] + ": " + \
                                  hipGetErrorString(_e));                        \
  } while (0)

namespace {

int vec_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (int)std::max<long long>(1, std::min<long long>(b, 1024));
}

struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  }
};

template <typename Real>
int x_rows_per_block(int m) {
  return std::max(1, std::min(64, MaxPt<Real>::value * FFT_THREADS / std::max(1, m)));
}

// x bins per tile of a strided pass over an axis of length L: 128-byte row
// segments (8 double or 16 float complex bins), fewer for long axes
template <typename Real>
int tile_width(int L) {
  const int w = 128 / (int)sizeof(typename CxT<Real>::T);
  return std::max(1, std::min(w, MaxPt<Real>::value * FFT_THREADS / L));
}

// Compute (or apply) the workspace layout.  When base == nullptr only the size
// is computed.
size_t layout_workspace(jfft_cell_s *c, unsigned char *base) {
  const long long N = c->g.N;
  const int d = c->dim;
  const long long nd = (long long)d * N;
  const long long nspec = (long long)d * c->g.nz * c->g.ny * c->g.mxp;
  Layout L;
  auto put = [&](auto *&ptr, size_t bytes) {
    size_t o = L.take(bytes);
    if (base) ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(base + o);
  };
  put(c->E, sizeof(double) * N);
  put(c->f, sizeof(double) * nd);
  put(c->r, sizeof(double) * nd);
  put(c->z, sizeof(double) * nd);
  put(c->q, sizeof(double) * nd);
  put(c->p[0], sizeof(double) * nd);
  put(c->p[1], sizeof(double) * nd);
  const bool useJ = c->pc == JFFT_PC_JACOBI || c->pc == JFFT_PC_GREEN_JACOBI;
  const bool useG = c->pc == JFFT_PC_GREEN || c->pc == JFFT_PC_GREEN_JACOBI;
  put(c->diag, sizeof(double) * nd);
  if (useJ) put(c->Jh, sizeof(double) * nd);
  if (useG) put(c->spec, sizeof(double2) * nspec);
  if (c->prec == JFFT_MIXED) {
    put(c->E32, sizeof(float) * N);
    if (useJ) put(c->Jh32, sizeof(float) * nd);
    put(c->r32, sizeof(float) * nd);
    put(c->z32, sizeof(float) * nd);
    put(c->q32, sizeof(float) * nd);
    put(c->p32[0], sizeof(float) * nd);
    put(c->p32[1], sizeof(float) * nd);
    put(c->c32, sizeof(float) * nd);
    if (useG) put(c->spec32, sizeof(float2) * nspec);
  }
  for (int a = 0; a < 3; ++a) {
    const int n = a == 0 ? c->g.nx : (a == 1 ? c->g.ny : c->g.nz);
    put(c->tw[a], sizeof(double2) * n);
    for (int t = 0; t < 3; ++t) put(c->ftab[a][t], sizeof(double) * n);
  }
  put(c->F, sizeof(double) * 24);
  put(c->macro, sizeof(double) * 8);
  put(c->st, sizeof(CgState));
  put(c->partA, sizeof(double) * c->npart);
  put(c->partB, sizeof(double) * c->npart);
  put(c->small, sizeof(double) * 64);
  for (int t = 0; t < 3; ++t) put(c->hist[t], sizeof(double) * kHistMax);
  return L.off;
}

long long max_partials(jfft_cell_s *c) {
  const GridDev &g = c->g;
  long long mx = 4 * 1024;  // vector kernels, stress blocks (<= 1024 per group, up to 6 groups)
  const long long tiles = (long long)((g.nx + TILE - 1) / TILE) * ((g.ny + TILE - 1) / TILE);
  mx = std::max(mx, tiles * ((g.nz + c->tz - 1) / c->tz));
  const int m = g.nx / 2;
  const long long rows = (long long)c->dim * g.ny * g.nz;
  mx = std::max(mx, (rows + x_rows_per_block<double>(m) - 1) / x_rows_per_block<double>(m));
  mx = std::max(mx, (g.N + 255) / 256 * 6);  // stress partials [ds][blocks]
  return mx;
}

jfft_status upload_tables(jfft_cell_s *c) {
  const int ns[3] = {c->g.nx, c->g.ny, c->g.nz};
  const double hs[3] = {c->len[0] / ns[0], c->len[1] / ns[1], c->dim == 3 ? c->len[2] / ns[2] : 1.0};
  for (int a = 0; a < 3; ++a) {
    const int n = ns[a];
    std::vector<double2> tw(n);
    std::vector<double> A(n), B(n), S(n);
    for (int j = 0; j < n; ++j) {
      const double t = 2.0 * M_PI * (double)j / (double)n;
      const double cs = std::cos(t), sn = std::sin(t);
      tw[j].x = cs;
      tw[j].y = -sn;
      A[j] = (2.0 - 2.0 * cs) / hs[a];
      B[j] = hs[a] * (2.0 + cs) / 3.0;
      S[j] = sn;
    }
    HIP_TRY(hipMemcpyAsync(c->tw[a], tw.data(), sizeof(double2) * n, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->ftab[a][0], A.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->ftab[a][1], B.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->ftab[a][2], S.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                           c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));  // host vectors go out of scope
  return JFFT_OK;
}

jfft_status ensure_ready(jfft_cell_s *c) {
  if (c->ready) return JFFT_OK;
  const size_t need = layout_workspace(c, nullptr);
  if (!c->ws) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) return fail(JFFT_E_OOM, std::string("hipMalloc workspace: ") + hipGetErrorString(e));
    c->ws = static_cast<unsigned char *>(p);
    c->ws_bytes = need;
    c->ws_owned = true;
  } else if (c->ws_bytes < need) {
    return fail(JFFT_E_OOM, "bound workspace smaller than jfft_workspace_bytes");
  }
  layout_workspace(c, c->ws);
  jfft_status s = upload_tables(c);
  if (s) return s;
  c->ready = true;
  return JFFT_OK;
}

// ---------------------------------------------------------------- launches
template <typename Real>
StencilArgs<Real> stencil_args(jfft_cell_s *c, const Real *E) {
  StencilArgs<Real> a{};
  a.E = E;
  a.lam = (Real)(c->lam * c->g.w);
  a.mu = (Real)(c->mu * c->g.w);
  a.ihx = (Real)c->g.ihx;
  a.ihy = (Real)c->g.ihy;
  a.ihz = (Real)c->g.ihz;
  a.nx = c->g.nx;
  a.ny = c->g.ny;
  a.nz = c->g.nz;
  a.N = c->g.N;
  a.tz = c->tz;
  a.st = c->st;
  return a;
}

dim3 stencil_grid(jfft_cell_s *c) {
  const GridDev &g = c->g;
  if (c->dim == 3)
    return dim3((g.nx + TILE - 1) / TILE, (g.ny + TILE - 1) / TILE, (g.nz + c->tz - 1) / c->tz);
  return dim3((g.nx + TILE - 1) / TILE, (g.ny + TILE - 1) / TILE, 1);
}

long long stencil_blocks(jfft_cell_s *c) {
  dim3 gr = stencil_grid(c);
  return (long long)gr.x * gr.y * gr.z;
}

template <typename Real, int MODE>
jfft_status launch_stiffness(jfft_cell_s *c, const StencilArgs<Real> &a) {
  const int kid = MODE == SM_CG ? KID_STIFF_CG : (MODE == SM_APPLY ? KID_STIFF_APPLY : KID_STIFF_COMB);
  dim3 gr = stencil_grid(c);
  if (c->dim == 3) {
    LAUNCH(c, kid, k_stiffness3d<Real, MODE><<<gr, STENCIL3_THREADS, 0, c->stream>>>(a));
  } else {
    LAUNCH(c, kid, k_stiffness2d<Real, MODE><<<gr, STENCIL_THREADS, 0, c->stream>>>(a));
  }
  return JFFT_OK;
}

template <typename Real>
jfft_status apply_K(jfft_cell_s *c, const Real *E, const Real *in, Real *out) {
  StencilArgs<Real> a = stencil_args<Real>(c, E);
  a.in = in;
  a.out = out;
  return launch_stiffness<Real, SM_APPLY>(c, a);
}

template <typename K>
void set_smem(K kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Forward x pass: spec = rfft_x(J^1/2 (r - alpha q)), partA = ||r||^2 partials.
template <typename Real>
jfft_status launch_xfwd(jfft_cell_s *c, Real *r, const Real *q, const Real *Jh,
                        typename CxT<Real>::T *spec, double *partA, bool update, bool check_done,
                        long long *nblk) {
  using C = typename CxT<Real>::T;
  XArgs<Real> a{};
  a.r = r;
  a.q = q;
  a.Jh = Jh;
  a.spec = spec;
  a.partA = partA;
  a.st = c->st;
  a.tw = c->tw[0];
  a.plan = c->plan_x;
  a.nx = c->g.nx;
  a.mx = c->g.mx;
  a.mxp = c->g.mxp;
  a.nrows = (long long)c->dim * c->g.ny * c->g.nz;
  const int m = c->g.nx / 2;
  a.rows_per_block = x_rows_per_block<Real>(m);
  a.check_done = check_done ? 1 : 0;
  const long long nb = (a.nrows + a.rows_per_block - 1) / a.rows_per_block;
  const size_t smem = sizeof(C) * (c->g.nx + (size_t)a.rows_per_block * (m + 1));
  *nblk = nb;
  const bool useJ = Jh != nullptr;
  if (update) {
    if (useJ) {
      set_smem(k_xfwd<Real, true, true>, smem);
      LAUNCH(c, KID_XFWD, k_xfwd<Real, true, true><<<(unsigned)nb, FFT_THREADS, smem, c->stream>>>(a));
    } else {
      set_smem(k_xfwd<Real, true, false>, smem);
      LAUNCH(c, KID_XFWD, k_xfwd<Real, true, false><<<(unsigned)nb, FFT_THREADS, smem, c->stream>>>(a));
    }
  } else {
    if (useJ) {
      set_smem(k_xfwd<Real, false, true>, smem);
      LAUNCH(c, KID_XFWD, k_xfwd<Real, false, true><<<(unsigned)nb, FFT_THREADS, smem, c->stream>>>(a));
    } else {
      set_smem(k_xfwd<Real, false, false>, smem);
      LAUNCH(c, KID_XFWD, k_xfwd<Real, false, false><<<(unsigned)nb, FFT_THREADS, smem, c->stream>>>(a));
    }
  }
  return JFFT_OK;
}

template <typename Real>
jfft_status launch_xinv(jfft_cell_s *c, const Real *r, const Real *Jh,
                        typename CxT<Real>::T *spec, Real *out, double *partB, bool check_done,
                        long long *nblk) {
  using C = typename CxT<Real>::T;
  XArgs<Real> a{};
  a.r = const_cast<Real *>(r);
  a.Jh = Jh;
  a.out = out;
  a.spec = spec;
  a.partA = partB;
  a.st = c->st;
  a.tw = c->tw[0];
  a.plan = c->plan_x;
  a.nx = c->g.nx;
  a.mx = c->g.mx;
  a.mxp = c->g.mxp;
  a.nrows = (long long)c->dim * c->g.ny * c->g.nz;
  const int m = c->g.nx / 2;
  a.rows_per_block = x_rows_per_block<Real>(m);
  a.check_done = check_done ? 1 : 0;
  const long long nb = (a.nrows + a.rows_per_block - 1) / a.rows_per_block;
  const size_t smem = sizeof(C) * (c->g.nx + (size_t)a.rows_per_block * (m + 1));
  *nblk = nb;
  if (Jh) {
    set_smem(k_xinv<Real, true>, smem);
    LAUNCH(c, KID_XINV, k_xinv<Real, true><<<(unsigned)nb, FFT_THREADS, smem, c->stream>>>(a));
  } else {
    set_smem(k_xinv<Real, false>, smem);
    LAUNCH(c, KID_XINV, k_xinv<Real, false><<<(unsigned)nb, FFT_THREADS, smem, c->stream>>>(a));
  }
  return JFFT_OK;
}

template <typename Real>
jfft_status launch_ypass(jfft_cell_s *c, typename CxT<Real>::T *spec, bool inv, bool check_done) {
  using C = typename CxT<Real>::T;
  YArgs<Real> a{};
  a.spec = spec;
  a.st = c->st;
  a.tw = c->tw[1];
  a.plan = c->plan_y;
  a.mx = c->g.mx;
  a.mxp = c->g.mxp;
  a.ny = c->g.ny;
  a.nz = c->g.nz;
  a.check_done = check_done ? 1 : 0;
  a.W = tile_width<Real>(c->g.ny);
  // persistent blocks: a few per CU, each walking tiles of one component
  const long long per_comp = (long long)((c->g.mx + a.W - 1) / a.W) * c->g.nz;
  const long long want = std::max<long long>(1, 2048 / c->dim);
  dim3 gr((unsigned)std::min(per_comp, want), c->dim, 1);
  const size_t smem = sizeof(C) * ((size_t)c->g.ny + (size_t)c->g.ny * a.W);
  if (inv) {
    set_smem(k_ypass<Real, true>, smem);
    LAUNCH(c, KID_YINV, k_ypass<Real, true><<<gr, FFT_THREADS, smem, c->stream>>>(a));
  } else {
    set_smem(k_ypass<Real, false>, smem);
    LAUNCH(c, KID_YFWD, k_ypass<Real, false><<<gr, FFT_THREADS, smem, c->stream>>>(a));
  }
  return JFFT_OK;
}

template <typename Real>
jfft_status launch_green(jfft_cell_s *c, typename CxT<Real>::T *spec, bool check_done) {
  using C = typename CxT<Real>::T;
  GArgs<Real> a{};
  a.spec = spec;
  a.st = c->st;
  const int La = c->dim == 3 ? 2 : 1;
  a.tw = c->tw[La];
  a.plan = c->dim == 3 ? c->plan_z : c->plan_y;
  a.tx = {c->ftab[0][0], c->ftab[0][1], c->ftab[0][2]};
  a.ty = {c->ftab[1][0], c->ftab[1][1], c->ftab[1][2]};
  a.tz = {c->ftab[2][0], c->ftab[2][1], c->ftab[2][2]};
  a.lam = c->lam;
  a.mu = c->mu;
  a.invN = 1.0 / (double)c->g.N;
  a.dim = c->dim;
  a.mx = c->g.mx;
  a.mxp = c->g.mxp;
  a.ny = c->g.ny;
  a.nz = c->g.nz;
  a.check_done = check_done ? 1 : 0;
  const int L = c->dim == 3 ? c->g.nz : c->g.ny;
  a.W = tile_width<Real>(L);
  dim3 gr((c->g.mx + a.W - 1) / a.W, c->dim == 3 ? c->g.ny : 1, 1);
  const size_t smem = sizeof(C) * ((size_t)L + (size_t)L * a.W);
  if (c->dim == 3) {
    set_smem(k_green_axis<Real, 3>, smem);
    LAUNCH(c, KID_GREEN, k_green_axis<Real, 3><<<gr, FFT_THREADS, smem, c->stream>>>(a));
  } else {
    set_smem(k_green_axis<Real, 2>, smem);
    LAUNCH(c, KID_GREEN, k_green_axis<Real, 2><<<gr, FFT_THREADS, smem, c->stream>>>(a));
  }
  return JFFT_OK;
}

// z = M^-1 r.  update: r <- r - alpha q first.  Partials: partA = ||r||^2,
// partB = r.z.  With ctrl, the CG control kernels run between the pieces.
template <typename Real>
jfft_status precond(jfft_cell_s *c, Real *r, const Real *q, const Real *Jh, Real *z,
                    typename CxT<Real>::T *spec, bool update, bool in_loop, long long *nA,
                    long long *nB, History h) {
  const bool useG = c->pc == JFFT_PC_GREEN || c->pc == JFFT_PC_GREEN_JACOBI;
  const bool useJ = c->pc == JFFT_PC_JACOBI || c->pc == JFFT_PC_GREEN_JACOBI;
  if (!useG) {
    const long long n = (long long)c->dim * c->g.N;
    const int nb = vec_blocks(n);
    *nA = *nB = nb;
    const int cd = in_loop ? 1 : 0;
    if (update) {
      if (useJ)
        LAUNCH(c, KID_DIAGPC, k_diag_pc<Real, true, true><<<nb, 256, 0, c->stream>>>(r, q, Jh, z, n, c->st, cd, c->partA, c->partB));
      else
        LAUNCH(c, KID_DIAGPC, k_diag_pc<Real, true, false><<<nb, 256, 0, c->stream>>>(r, q, Jh, z, n, c->st, cd, c->partA, c->partB));
    } else {
      if (useJ)
        LAUNCH(c, KID_DIAGPC, k_diag_pc<Real, false, true><<<nb, 256, 0, c->stream>>>(r, q, Jh, z, n, c->st, cd, c->partA, c->partB));
      else
        LAUNCH(c, KID_DIAGPC, k_diag_pc<Real, false, false><<<nb, 256, 0, c->stream>>>(r, q, Jh, z, n, c->st, cd, c->partA, c->partB));
    }
    if (in_loop) {
      LAUNCH(c, KID_CTRL, k_cg_rr<<<1, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, *nA, h));
      LAUNCH(c, KID_CTRL, k_cg_beta<<<1, CTRL_THREADS, 0, c->stream>>>(c->st, c->partB, *nB, h));
    }
    return JFFT_OK;
  }
  const Real *J = useJ ? Jh : nullptr;
  jfft_status s = launch_xfwd<Real>(c, r, q, J, spec, c->partA, update, in_loop, nA);
  if (s) return s;
  if (in_loop) LAUNCH(c, KID_CTRL, k_cg_rr<<<1, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, *nA, h));
  if (c->dim == 3) {
    if ((s = launch_ypass<Real>(c, spec, false, in_loop))) return s;
    if ((s = launch_green<Real>(c, spec, in_loop))) return s;
    if ((s = launch_ypass<Real>(c, spec, true, in_loop))) return s;
  } else {
    if ((s = launch_green<Real>(c, spec, in_loop))) return s;
  }
  s = launch_xinv<Real>(c, r, J, spec, z, c->partB, in_loop, nB);
  if (s) return s;
  if (in_loop) LAUNCH(c, KID_CTRL, k_cg_beta<<<1, CTRL_THREADS, 0, c->stream>>>(c->st, c->partB, *nB, h));
  return JFFT_OK;
}

__global__ void k_cg_init(CgState *st, double tol2, int maxit, int hist_cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->tol2 = tol2;
    st->maxit = maxit;
    st->hist_cap = hist_cap;
    st->iter = 0;
    st->done = 0;
    st->status = 0;
    st->pending = 0;
    st->first = 1;
  }
}

// PCG loop on prepared buffers: u holds the start vector, r = f - K u.
// Returns after the device flag is set; the final state is in c->st_h.
template <typename Real>
jfft_status run_pcg(jfft_cell_s *c, const PcgBufs<Real> &b, double tol2, int maxit, bool record) {
  History h{nullptr, nullptr, nullptr};
  if (record && c->hist_cap > 0) h = {c->hist[0], c->hist[1], c->hist[2]};
  long long nA = 0, nB = 0;
  LAUNCH(c, KID_CTRL, k_cg_init<<<1, 1, 0, c->stream>>>(c->st, tol2, maxit, record ? c->hist_cap : 0));
  jfft_status s = precond<Real>(c, b.r, nullptr, b.Jh, b.z, b.spec, false, false, &nA, &nB, h);
  if (s) return s;
  LAUNCH(c, KID_CTRL, k_cg_start<<<1, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, nA, c->partB, nB));
  const long long nK = stencil_blocks(c);
  int it = 0;
  int chunk = 2;
  for (;;) {
    for (int k = 0; k < chunk; ++k) {
      ++it;
      StencilArgs<Real> a = stencil_args<Real>(c, b.E);
      a.in = b.p[it & 1];
      a.zin = b.z;
      a.pout = b.p[(it + 1) & 1];
      a.u = b.u;
      a.out = b.q;
      a.partial = c->partA;
      if ((s = launch_stiffness<Real, SM_CG>(c, a))) return s;
      LAUNCH(c, KID_CTRL, k_cg_alpha<<<1, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, nK, h));
      if ((s = precond<Real>(c, b.r, b.q, b.Jh, b.z, b.spec, true, true, &nA, &nB, h))) return s;
    }
    HIP_TRY(hipMemcpyAsync(c->st_h, c->st, sizeof(CgState), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->st_h->done) break;
    chunk = std::min(chunk * 2, 32);
  }
  // apply the owed update u += alpha p_k (p_k written by iteration iter)
  const long long n = (long long)c->dim * c->g.N;
  const Real *plast = b.p[(c->st_h->iter + 1) & 1];
  LAUNCH(c, KID_VEC, k_finish_u<Real><<<vec_blocks(n), 256, 0, c->stream>>>(b.u, plast, n, c->st));
  return JFFT_OK;
}

// Sum of n partials (one group) into small[slot]; no host sync.
jfft_status reduce_to(jfft_cell_s *c, const double *part, long long n, int groups, int slot) {
  LAUNCH(c, KID_REDUCE, k_reduce_groups<<<1, CTRL_THREADS, 0, c->stream>>>(part, n, groups, c->small + slot));
  return JFFT_OK;
}

jfft_status fetch_small(jfft_cell_s *c, int count) {
  HIP_TRY(hipMemcpyAsync(c->small_h, c->small, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return JFFT_OK;
}

jfft_status assemble_rhs(jfft_cell_s *c, const double *macro_h, double *f, double *fabs_out) {
  const int ds = c->dim * (c->dim + 1) / 2;
  HIP_TRY(hipMemcpyAsync(c->macro, macro_h, sizeof(double) * ds, hipMemcpyHostToDevice, c->stream));
  LAUNCH(c, KID_RHS, k_unit_force<<<1, 1, 0, c->stream>>>(c->F, c->macro, c->dim, c->lam * c->g.w, c->mu * c->g.w, c->g.ihx, c->g.ihy, c->g.ihz));
  const long long N = c->g.N;
  LAUNCH(c, KID_RHS, k_rhs<double><<<(unsigned)((N + 255) / 256), 256, 0, c->stream>>>(c->E, c->F, f, fabs_out, c->dim, c->g.nx, c->g.ny, c->g.nz, N));
  return JFFT_OK;
}

jfft_status run_alg2(jfft_cell_s *c, double *diag_out) {
  StencilArgs<double> a = stencil_args<double>(c, c->E);
  a.diag = diag_out;
  const int nloc = 1 << c->dim;
  for (int comp = 0; comp < c->dim; ++comp)
    for (int off = 0; off < nloc; ++off) {
      a.comb_comp = comp;
      a.comb_off = off;
      jfft_status s = launch_stiffness<double, SM_COMB>(c, a);
      if (s) return s;
    }
  return JFFT_OK;
}

jfft_status set_material_impl(jfft_cell_s *c, const double *E_dev, double lam, double mu) {
  if (!E_dev) return fail(JFFT_E_INVALID, "E_dev is NULL");
  if (!(mu > 0.0) || !(lam + 2.0 * mu / c->dim > 0.0) || !std::isfinite(lam) || !std::isfinite(mu))
    return fail(JFFT_E_INVALID, "Lame constants must satisfy mu > 0 and lambda + 2 mu / d > 0");
  jfft_status s = ensure_ready(c);
  if (s) return s;
  c->lam = lam;
  c->mu = mu;
  const long long N = c->g.N;
  const int nb = vec_blocks(N);
  LAUNCH(c, KID_SETUP, k_check_E<<<nb, 256, 0, c->stream>>>(E_dev, N, c->partA));
  if ((s = reduce_to(c, c->partA, nb, 1, 0))) return s;
  if ((s = fetch_small(c, 1))) return s;
  if (c->small_h[0] != 0.0) return fail(JFFT_E_INVALID, "E contains negative or non-finite entries");
  LAUNCH(c, KID_SETUP, k_copy<double><<<nb, 256, 0, c->stream>>>(E_dev, c->E, N));
  const long long nd = (long long)c->dim * N;
  const bool useJ = c->pc == JFFT_PC_JACOBI || c->pc == JFFT_PC_GREEN_JACOBI;
  if (useJ) {
    if ((s = run_alg2(c, c->diag))) return s;
    LAUNCH(c, KID_SETUP, k_jhalf<double><<<vec_blocks(nd), 256, 0, c->stream>>>(c->diag, c->Jh, nd, c->void_value));
  }
  if (c->prec == JFFT_MIXED) {
    LAUNCH(c, KID_SETUP, (k_convert<double, float><<<nb, 256, 0, c->stream>>>(c->E, c->E32, N, 1.0)));
    if (useJ)
      LAUNCH(c, KID_SETUP, k_jhalf<float><<<vec_blocks(nd), 256, 0, c->stream>>>(c->diag, c->Jh32, nd, c->void_value));
  }
  c->has_material = true;
  return JFFT_OK;
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return ms;
}

jfft_status post_process(jfft_cell_s *c, const double *macro_h, double *u, double *sigma_dev,
                         double *sigma_bar, double fnorm, jfft_report *rep) {
  const long long N = c->g.N;
  const int d = c->dim;
  const long long nd = (long long)d * N;
  const int ds = d * (d + 1) / 2;
  jfft_status s;
  // true residual with the FP64 stiffness
  if ((s = apply_K<double>(c, c->E, u, c->q))) return s;
  const int nb = vec_blocks(nd);
  LAUNCH(c, KID_VEC, k_sub_norm<double><<<nb, 256, 0, c->stream>>>(c->f, c->q, nullptr, nd, c->partA));
  if ((s = reduce_to(c, c->partA, nb, 1, 0))) return s;
  // mean removal (Sec. 5)
  const int nbN = vec_blocks(N);
  LAUNCH(c, KID_VEC, k_comp_sum<double><<<dim3(nbN, d), 256, 0, c->stream>>>(u, N, c->partB));
  if ((s = reduce_to(c, c->partB, nbN, d, 8))) return s;
  LAUNCH(c, KID_VEC, k_sub_mean<double><<<dim3(nbN, d), 256, 0, c->stream>>>(u, N, c->small + 8));
  // stresses and sigma_bar
  HIP_TRY(hipMemcpyAsync(c->macro, macro_h, sizeof(double) * ds, hipMemcpyHostToDevice, c->stream));
  const unsigned nbs = (unsigned)((N + 255) / 256);
  LAUNCH(c, KID_STRESS, k_stress<double><<<nbs, 256, 0, c->stream>>>(u, c->E, c->macro, c->lam, c->mu, c->g.w, c->g.ihx, c->g.ihy, c->g.ihz, d, c->g.nx, c->g.ny, c->g.nz, N, sigma_dev, c->partB));
  if ((s = reduce_to(c, c->partB, nbs, ds, 16))) return s;
  if ((s = fetch_small(c, 32))) return s;
  if (rep) rep->rel_res_true = fnorm > 0 ? std::sqrt(c->small_h[0]) / fnorm : 0.0;
  for (int r = 0; r < ds; ++r) sigma_bar[r] = c->small_h[16 + r] / c->g.vol;
  return JFFT_OK;
}

jfft_status solve_impl(jfft_cell_s *c, const double *macro_h, double tol, int maxit,
                       const double *u0, double *u, double *sigma_dev, double *sigma_bar,
                       jfft_report *rep) {
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  if (!macro_h || !u || !sigma_bar) return fail(JFFT_E_INVALID, "NULL macro_strain, u_dev or sigma_bar");
  if (!(tol > 0.0) || maxit < 0) return fail(JFFT_E_INVALID, "tol must be > 0 and maxit >= 0");
  jfft_report lrep{};
  jfft_report *R = rep ? rep : &lrep;
  *R = jfft_report{};
  const long long N = c->g.N;
  const int d = c->dim;
  const long long nd = (long long)d * N;
  jfft_status s;
  for (auto &e : c->phase_ev)
    if (!e) HIP_TRY(hipEventCreate(&e));
  HIP_TRY(hipEventRecord(c->phase_ev[0], c->stream));
  // f and |f|
  if ((s = assemble_rhs(c, macro_h, c->f, c->q))) return s;
  const int nb = vec_blocks(nd);
  LAUNCH(c, KID_VEC, k_dot<double><<<nb, 256, 0, c->stream>>>(c->f, c->f, nd, c->partA));
  LAUNCH(c, KID_VEC, k_dot<double><<<nb, 256, 0, c->stream>>>(c->q, c->q, nd, c->partB));
  if ((s = reduce_to(c, c->partA, nb, 1, 0))) return s;
  if ((s = reduce_to(c, c->partB, nb, 1, 1))) return s;
  if ((s = fetch_small(c, 2))) return s;
  const double fnorm = std::sqrt(c->small_h[0]);
  const double fabsnorm = std::sqrt(c->small_h[1]);
  const bool homogeneous = fnorm <= 1e-13 * fabsnorm;
  // start vector
  if (u0 && !homogeneous) {
    LAUNCH(c, KID_VEC, k_copy<double><<<nb, 256, 0, c->stream>>>(u0, u, nd));
  } else {
    LAUNCH(c, KID_VEC, k_fill<double><<<nb, 256, 0, c->stream>>>(u, 0.0, nd));
  }
  HIP_TRY(hipEventRecord(c->phase_ev[1], c->stream));
  int status = JFFT_OK;
  if (homogeneous) {
    R->iters = 0;
    R->outer = 0;
    R->rel_res = 0.0;
  } else if (c->prec == JFFT_FP64) {
    if (u0) {
      if ((s = apply_K<double>(c, c->E, u, c->q))) return s;
      LAUNCH(c, KID_VEC, k_sub_norm<double><<<nb, 256, 0, c->stream>>>(c->f, c->q, c->r, nd, c->partA));
    } else {
      LAUNCH(c, KID_VEC, k_copy<double><<<nb, 256, 0, c->stream>>>(c->f, c->r, nd));
    }
    PcgBufs<double> b{u, c->r, c->z, c->q, {c->p[0], c->p[1]}, c->E, c->Jh, c->spec};
    if ((s = run_pcg<double>(c, b, tol * tol * fnorm * fnorm, maxit, true))) return s;
    R->iters = c->st_h->iter;
    R->outer = 1;
    R->rel_res = fnorm > 0 ? std::sqrt(c->st_h->rr) / fnorm : 0.0;
    status = c->st_h->status;
  } else {
    // mixed precision: FP64 residual and iterate, FP32 inner PCG
    int total = 0, outer = 0;
    status = JFFT_E_NOT_CONVERGED;
    double rel = 0.0;
    for (;;) {
      if ((s = apply_K<double>(c, c->E, u, c->q))) return s;
      LAUNCH(c, KID_VEC, k_sub_norm<double><<<nb, 256, 0, c->stream>>>(c->f, c->q, c->r, nd, c->partA));
      if ((s = reduce_to(c, c->partA, nb, 1, 0))) return s;
      if ((s = fetch_small(c, 1))) return s;
      const double rn = std::sqrt(c->small_h[0]);
      rel = fnorm > 0 ? rn / fnorm : 0.0;
      if (rn <= tol * fnorm) {
        status = JFFT_OK;
        break;
      }
      if (outer >= c->max_outer || total >= maxit) break;
      const double scale = 1.0 / rn;
      LAUNCH(c, KID_VEC, (k_convert<double, float><<<nb, 256, 0, c->stream>>>(c->r, c->r32, nd, scale)));
      LAUNCH(c, KID_VEC, k_fill<float><<<nb, 256, 0, c->stream>>>(c->c32, 0.0f, nd));
      PcgBufs<float> b{c->c32, c->r32, c->z32, c->q32, {c->p32[0], c->p32[1]}, c->E32, c->Jh32, c->spec32};
      const double itol = std::max(c->inner_tol, 0.5 * tol * fnorm / rn);
      if ((s = run_pcg<float>(c, b, itol * itol, std::max(1, maxit - total), false))) return s;
      total += c->st_h->iter;
      ++outer;
      LAUNCH(c, KID_VEC, k_axpy_f32_to_f64<<<nb, 256, 0, c->stream>>>(c->c32, u, nd, rn));
      if (c->st_h->status == JFFT_E_BREAKDOWN && c->st_h->iter == 0) {
        status = JFFT_E_BREAKDOWN;
        break;
      }
    }
    R->iters = total;
    R->outer = outer;
    R->rel_res = rel;
  }
  HIP_TRY(hipEventRecord(c->phase_ev[2], c->stream));
  if ((s = post_process(c, macro_h, u, sigma_dev, sigma_bar, fnorm, R))) return s;
  if (homogeneous) R->rel_res_true = 0.0;
  HIP_TRY(hipEventRecord(c->phase_ev[3], c->stream));
  HIP_TRY(hipEventSynchronize(c->phase_ev[3]));
  R->setup_ms = elapsed_ms(c->phase_ev[0], c->phase_ev[1]);
  R->loop_ms = elapsed_ms(c->phase_ev[1], c->phase_ev[2]);
  R->post_ms = elapsed_ms(c->phase_ev[2], c->phase_ev[3]);
  R->status = status;
  if (status == JFFT_E_NOT_CONVERGED) g_last_error = "PCG reached maxit";
  if (status == JFFT_E_BREAKDOWN) g_last_error = "PCG breakdown (p.q <= 0 or non-finite scalar)";
  return (jfft_status)status;
}

bool supported_length(int n) {
  if (n < 2 || n > 512 || n % 2) return false;
  FftPlan p;
  return factor_plan(n, p) && factor_plan(n / 2, p);
}

}  // namespace

// ============================================================== C ABI ====
extern "C" {

jfft_status jfft_create_cell(int dim, const int n[3], const double len[3], jfft_precision prec,
                             jfft_precond pc, void *hip_stream, jfft_cell_t *out) {
  if (!out || !n) return fail(JFFT_E_INVALID, "NULL argument");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(JFFT_E_INVALID, "dim must be 2 or 3");
  if (prec != JFFT_FP64 && prec != JFFT_MIXED) return fail(JFFT_E_INVALID, "unknown precision");
  if (pc < JFFT_PC_NONE || pc > JFFT_PC_GREEN_JACOBI) return fail(JFFT_E_INVALID, "unknown preconditioner");
  for (int a = 0; a < dim; ++a) {
    if (n[a] % 2 != 0 && n[a] >= 2) return fail(JFFT_E_ODD_GRID, "node counts must be even");
    if (!supported_length(n[a]))
      return fail(JFFT_E_INVALID, "node counts must be even, in [2, 512] and products of 2, 3, 5");
    if (len && !(len[a] > 0.0 && std::isfinite(len[a]))) return fail(JFFT_E_INVALID, "lengths must be positive");
  }
  jfft_cell_s *c = new (std::nothrow) jfft_cell_s();
  if (!c) return fail(JFFT_E_OOM, "host allocation");
  c->dim = dim;
  c->prec = prec;
  c->pc = pc;
  c->stream = static_cast<hipStream_t>(hip_stream);
  for (int a = 0; a < 3; ++a) {
    c->n[a] = a < dim ? n[a] : 1;
    c->len[a] = (a < dim && len) ? len[a] : 1.0;
  }
  GridDev &g = c->g;
  g.dim = dim;
  g.nx = c->n[0];
  g.ny = c->n[1];
  g.nz = c->n[2];
  g.N = (long long)g.nx * g.ny * g.nz;
  g.mx = g.nx / 2 + 1;
  g.mxp = (g.mx + 15) / 16 * 16;  // rows of the half spectrum start on 128/256-byte boundaries
  double evol = 1.0;
  g.vol = 1.0;
  double hs[3];
  for (int a = 0; a < 3; ++a) {
    hs[a] = c->len[a] / c->n[a];
    if (a < dim) {
      evol *= hs[a];
      g.vol *= c->len[a];
    }
  }
  g.ihx = 1.0 / hs[0];
  g.ihy = 1.0 / hs[1];
  g.ihz = dim == 3 ? 1.0 / hs[2] : 0.0;
  g.w = evol / (1 << dim);
  factor_plan(g.nx / 2, c->plan_x);
  factor_plan(g.ny, c->plan_y);
  factor_plan(g.nz, c->plan_z);
  // z planes per stiffness block: enough blocks to fill 256 CUs several times
  if (dim == 3) {
    const long long tiles = (long long)((g.nx + TILE - 1) / TILE) * ((g.ny + TILE - 1) / TILE);
    int tz = 32;
    while (tz > 4 && tiles * ((g.nz + tz - 1) / tz) < 2048) tz /= 2;
    c->tz = std::min(tz, g.nz);
  } else {
    c->tz = 1;
  }
  c->npart = max_partials(c);
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&c->st_h), sizeof(CgState), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&c->small_h), sizeof(double) * 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return fail(JFFT_E_HIP, std::string("create: ") + hipGetErrorString(e));
  }
  *out = c;
  return JFFT_OK;
}

jfft_status jfft_workspace_bytes(jfft_cell_t c, size_t *bytes) {
  if (!c || !bytes) return fail(JFFT_E_INVALID, "NULL argument");
  *bytes = layout_workspace(c, nullptr);
  return JFFT_OK;
}

jfft_status jfft_bind_workspace(jfft_cell_t c, void *dev_ptr, size_t bytes) {
  if (!c || !dev_ptr) return fail(JFFT_E_INVALID, "NULL argument");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) return fail(JFFT_E_INVALID, "workspace must be 256-byte aligned");
  const size_t need = layout_workspace(c, nullptr);
  if (bytes < need) return fail(JFFT_E_OOM, "workspace smaller than jfft_workspace_bytes");
  if (c->ws_owned && c->ws) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->ws);
  }
  c->ws = static_cast<unsigned char *>(dev_ptr);
  c->ws_bytes = bytes;
  c->ws_owned = false;
  c->ready = false;
  c->has_material = false;
  return ensure_ready(c);
}

jfft_status jfft_set_material(jfft_cell_t c, const double *E_dev, double nu) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  if (!(nu > -1.0 && nu < 0.5)) return fail(JFFT_E_INVALID, "nu must lie in (-1, 0.5)");
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  return set_material_impl(c, E_dev, lam, mu);
}

jfft_status jfft_set_material_lame(jfft_cell_t c, const double *E_dev, double lambda, double mu) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  return set_material_impl(c, E_dev, lambda, mu);
}

jfft_status jfft_solve(jfft_cell_t c, const double *macro_strain, double tol, int maxit,
                       const double *u0_dev, double *u_dev, double *sigma_dev, double *sigma_bar,
                       jfft_report *report) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  return solve_impl(c, macro_strain, tol, maxit, u0_dev, u_dev, sigma_dev, sigma_bar, report);
}

jfft_status jfft_apply_stiffness(jfft_cell_t c, const double *in_dev, double *out_dev) {
  if (!c || !in_dev || !out_dev) return fail(JFFT_E_INVALID, "NULL argument");
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  return apply_K<double>(c, c->E, in_dev, out_dev);
}

jfft_status jfft_apply_precond(jfft_cell_t c, const double *in_dev, double *out_dev) {
  if (!c || !in_dev || !out_dev) return fail(JFFT_E_INVALID, "NULL argument");
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  const long long nd = (long long)c->dim * c->g.N;
  LAUNCH(c, KID_VEC, k_copy<double><<<vec_blocks(nd), 256, 0, c->stream>>>(in_dev, c->r, nd));
  long long nA, nB;
  History h{nullptr, nullptr, nullptr};
  return precond<double>(c, c->r, nullptr, c->Jh, out_dev, c->spec, false, false, &nA, &nB, h);
}

jfft_status jfft_assemble_rhs(jfft_cell_t c, const double *macro_strain, double *f_dev) {
  if (!c || !macro_strain || !f_dev) return fail(JFFT_E_INVALID, "NULL argument");
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  jfft_status s = assemble_rhs(c, macro_strain, f_dev, nullptr);
  if (s) return s;
  HIP_TRY(hipStreamSynchronize(c->stream));  // macro_strain is a host pointer
  return JFFT_OK;
}

jfft_status jfft_jacobi_diag(jfft_cell_t c, double *diag_dev) {
  if (!c || !diag_dev) return fail(JFFT_E_INVALID, "NULL argument");
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  return run_alg2(c, diag_dev);
}

jfft_status jfft_enable_history(jfft_cell_t c, int cap) {
  if (!c || cap < 0 || cap > kHistMax) return fail(JFFT_E_INVALID, "history capacity must lie in [0, 4096]");
  c->hist_cap = cap;
  return JFFT_OK;
}

jfft_status jfft_get_history(jfft_cell_t c, double *alpha, double *beta, double *res, int cap,
                             int *count) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  const int k = std::min(std::min(cap, c->hist_cap), c->st_h ? c->st_h->iter : 0);
  if (count) *count = k;
  if (k <= 0) return JFFT_OK;
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (alpha) HIP_TRY(hipMemcpy(alpha, c->hist[0], sizeof(double) * k, hipMemcpyDeviceToHost));
  if (beta) HIP_TRY(hipMemcpy(beta, c->hist[1], sizeof(double) * k, hipMemcpyDeviceToHost));
  if (res) HIP_TRY(hipMemcpy(res, c->hist[2], sizeof(double) * k, hipMemcpyDeviceToHost));
  return JFFT_OK;
}

jfft_status jfft_enable_timing(jfft_cell_t c, int on) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  c->flush_timing();
  c->timing = on != 0;
  return JFFT_OK;
}

jfft_status jfft_reset_timing(jfft_cell_t c) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  c->flush_timing();
  for (int i = 0; i < KID_COUNT; ++i) {
    c->ktime[i] = 0.0;
    c->kcount[i] = 0;
  }
  return JFFT_OK;
}

jfft_status jfft_kernel_stats(jfft_cell_t c, int i, const char **name, long *launches,
                              double *total_ms, int *count) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  c->flush_timing();
  if (count) *count = KID_COUNT;
  if (i < 0 || i >= KID_COUNT) return JFFT_OK;
  if (name) *name = kKernelNames[i];
  if (launches) *launches = c->kcount[i];
  if (total_ms) *total_ms = c->ktime[i];
  return JFFT_OK;
}

jfft_status jfft_set_void_value(jfft_cell_t c, double value) {
  if (!c || !(value > 0.0) || !std::isfinite(value)) return fail(JFFT_E_INVALID, "void value must be positive");
  c->void_value = value;
  return JFFT_OK;
}

jfft_status jfft_set_mixed_params(jfft_cell_t c, double inner_tol, int max_outer) {
  if (!c || !(inner_tol > 0.0 && inner_tol < 1.0) || max_outer < 1)
    return fail(JFFT_E_INVALID, "inner_tol must lie in (0, 1) and max_outer >= 1");
  c->inner_tol = inner_tol;
  c->max_outer = max_outer;
  return JFFT_OK;
}

void jfft_destroy_cell(jfft_cell_t c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char *jfft_last_error(void) { return g_last_error.c_str(); }

const char *jfft_version(void) { return "jfft-mi355x 0.1 (gfx950)"; }

}  // extern "C"
