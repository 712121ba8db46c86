// Host driver and C ABI of the MI355X J-FFT solver (see include/jfft.h).
//
// A handle holds a group of B periodic cells of identical shape (B = 1 for
// the single-cell entry points) on one stream.  Their workspace is one device
// buffer of B equal slices plus a shared region of read-only tables; kernels
// find their cell from a grid dimension and shift their pointers by the slice
// stride, so one launch serves the whole group and every cell keeps its own
// CG state and stops on its own.
//
// set_material copies E, runs Algorithm 2 (d 2^d stiffness applications to
// unit combs, Sec. 3.2) and forms J^1/2.  solve assembles f, runs the PCG
// loop entirely on the device (CG scalars in device memory; the host only
// polls the stop flags every few iterations, optionally replaying the
// iterations as a captured HIP graph), then removes the mean of u (Sec. 5),
// recomputes the true residual with the FP64 stiffness and evaluates the
// stresses and sigma_bar.  The mixed mode runs FP32 inner solves inside an
// FP64 iterative-refinement loop whose decisions are also taken on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cg.h"
#include "fft.h"
#include "jfft.h"
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

#define TRY(expr)                 \
  do {                            \
    jfft_status _s = (expr);      \
    if (_s != JFFT_OK) return _s; \
  } while (0)

namespace {

constexpr int kHistMax = 4096;
constexpr int kSmall = 64;  // doubles of per-cell reduction results

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
  int p = 1;
  for (int s = 0; s < pl.nst; ++s) {
    pl.mdiv[s] = FastDiv(L / pl.radix[s]);
    pl.pdiv[s] = FastDiv(p);
    p *= pl.radix[s];
  }
  return true;
}

// Pointers of cell 0 for one precision.
template <typename Real>
struct PcgBufs {
  Real *u, *r, *z, *q, *p[2];
  const Real *E, *Jh;
  typename CxT<Real>::T *spec;
};

struct Tunables {
  int tz = 32;          // z planes per stiffness block (3D)
  int ygrid = 2048;     // persistent blocks of the y pass (all components and cells)
  int graph_iters = 0;  // iterations per captured graph (0: launch kernels directly)
  int tiles2d = 0;      // 2D stiffness block shape (1..4, see jfft_tunables; 0: by precision)
  int tiles3d = 0;      // 3D stiffness block shape of the FP32 kernels (1..2; 0: the default)
  int xrows = 0;        // rows per block of the x passes (power of two; 0: the most that fit)
  int fused_control = 0;  // CG scalar steps in the last block of their producers (0: own launches)
  bool tz_auto = true;    // tz follows the material kind and block shape (until set explicitly)
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
  int B = 1;  // cells in the group
  GridDev g{};
  FftPlan plan_x{}, plan_y{}, plan_z{};
  Tunables tun;

  // workspace: B slices of `cs` bytes, then the shared tables
  unsigned char *ws = nullptr;
  size_t ws_bytes = 0;
  long long cs = 0;
  bool ws_owned = false;
  bool ready = false;

  // per-cell buffers (pointers of cell 0)
  double *E = nullptr, *Jh = nullptr, *diag = nullptr, *f = nullptr, *r = nullptr, *z = nullptr,
         *q = nullptr, *p[2] = {nullptr, nullptr}, *u = nullptr;
  double2 *spec = nullptr;
  float *E32 = nullptr, *Jh32 = nullptr, *r32 = nullptr, *z32 = nullptr, *q32 = nullptr,
        *p32[2] = {nullptr, nullptr}, *c32 = nullptr;
  float2 *spec32 = nullptr;
  double *F = nullptr, *macro = nullptr;
  CgState *st = nullptr;
  double *partA = nullptr, *partB = nullptr;
  long long npart = 0;
  double *small = nullptr;
  double *hist[3] = {nullptr, nullptr, nullptr};
  int hist_cap = 0;
  // shared tables
  double2 *tw[3] = {nullptr, nullptr, nullptr};
  double *ftab[3][3] = {};

  // host pinned mirrors (B entries)
  CgState *st_h = nullptr;
  double *small_h = nullptr;

  bool has_material = false;
  double lam = 0, mu = 0;
  double void_value = 1.0;
  double inner_tol = 1e-6;
  int max_outer = 30;
  int inner_cap = 2000;  // iterations of one FP32 inner solve (0: no cap)
  bool mixed_continue = true;  // refinement sweeps continue the FP32 CG (reliable updates)
  double update_tol = 1e-2;    // continued sweeps: residual reduction between reliable updates
  bool stop_abs = false;  // stopping rule ||r||^2 <= tol instead of ||r|| <= tol ||f||
  int diag_method = JFFT_DIAG_CLOSED_FORM;  // how J^1/2 is formed (Algorithm 2 or its closed form)
  int elem = JFFT_ELEM_QUAD;  // 2D element: bilinear quadrilateral or two linear triangles
  double tS[9][3] = {};       // triangles: stencil of K_ref (see green2_tri)

  // power-law material (nonlinear example): E holds the phase, lam and mu the
  // Green reference (the inclusion); uk is the Newton iterate, allocated on
  // first use and owned by the handle
  bool nl = false;
  PowerLawArgs pl{};
  double *uk = nullptr;
  float *uk32 = nullptr;  // FP32 copy of uk for the inner solves of a mixed-precision cell

  // topology optimisation (three-cell 2D triangle groups): L-BFGS vectors,
  // allocated on first use and owned by the handle
  double *topo = nullptr;
  int topo_m = 0;

  // continuous batching: per-cell slot state (empty until the first admission)
  std::vector<int> slot_state, slot_maxit, slot_sweep;
  std::vector<std::chrono::steady_clock::time_point> slot_t0;
  std::vector<double> slot_ms;
  bool in_view = false;  // per-cell pointers moved to one slot (CellView)

  // captured iteration chunks
  // one per (precision, cells launched, depth): the whole group, or a
  // prefix of its slots (continuous batching)
  struct Graph {
    int fp64, cells, iters;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  bool capturing = false;

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

  void drop_graphs() {
    for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }

  ~jfft_cell_s() {
    flush_timing();
    drop_graphs();
    for (auto &e : pool) (void)hipEventDestroy(e);
    for (auto &e : phase_ev)
      if (e) (void)hipEventDestroy(e);
    if (ws_owned && ws) (void)hipFree(ws);
    if (uk) (void)hipFree(uk);
    if (uk32) (void)hipFree(uk32);
    if (topo) (void)hipFree(topo);
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
    if (!timing || capturing) return nullptr;
    hipEvent_t a = get_event();
    (void)hipEventRecord(a, stream);
    return a;
  }
  void te(int kid, hipEvent_t a) {
    if (!timing || capturing || !a) return;
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

// Blocks per cell of the grid-stride vector kernels.  Like every other
// reduction layout of the library it depends on the cell shape only, so a
// cell gives bitwise the same results alone and inside any group.
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

// The most rows an x-pass block holds; the xrows tunable may lower it to
// any power of two down to 1 (more, smaller blocks for small grids).
template <typename Real>
int x_rows_per_block(int m) {  // a power of two (tile-major index math uses shifts)
  const int cap = std::max(1, std::min(64, MaxPt<Real>::value * FFT_THREADS / std::max(1, m)));
  int rb = 1;
  while (rb * 2 <= cap) rb *= 2;
  return rb;
}

// x-tiles per half-spectrum row and complex values per padded row
template <typename Real>
int ntx_of(const jfft_cell_s *c) {
  return (c->g.mx + TileW<Real>::value - 1) / TileW<Real>::value;
}
template <typename Real>
long long spec_row(const jfft_cell_s *c) {
  return (long long)ntx_of<Real>(c) * TileW<Real>::value;
}

bool useJ(const jfft_cell_s *c) { return c->pc == JFFT_PC_JACOBI || c->pc == JFFT_PC_GREEN_JACOBI; }
bool useG(const jfft_cell_s *c) { return c->pc == JFFT_PC_GREEN || c->pc == JFFT_PC_GREEN_JACOBI; }

// Slice layout (one cell) and the shared tables.  With base == nullptr only
// sizes are computed; returns the total bytes.
size_t layout_workspace(jfft_cell_s *c, unsigned char *base) {
  const long long N = c->g.N;
  const int d = c->dim;
  const long long nd = (long long)d * N;
  // tile-major half spectra: d * nz * ny * ntx * TW complex per precision
  const long long nspec64 = (long long)d * c->g.nz * c->g.ny * spec_row<double>(c);
  const long long nspec32 = (long long)d * c->g.nz * c->g.ny * spec_row<float>(c);
  Layout L;
  auto put = [&](auto *&ptr, size_t bytes) {
    size_t o = L.take(bytes);
    if (base) ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(base + o);
  };
  put(c->E, sizeof(double) * N);
  put(c->f, sizeof(double) * nd);
  put(c->u, sizeof(double) * nd);
  put(c->r, sizeof(double) * nd);
  put(c->z, sizeof(double) * nd);
  put(c->q, sizeof(double) * nd);
  put(c->p[0], sizeof(double) * nd);
  put(c->p[1], sizeof(double) * nd);
  put(c->diag, sizeof(double) * nd);
  if (useJ(c)) put(c->Jh, sizeof(double) * nd);
  if (useG(c)) put(c->spec, sizeof(double2) * nspec64);
  if (c->prec == JFFT_MIXED) {
    put(c->E32, sizeof(float) * N);
    if (useJ(c)) put(c->Jh32, sizeof(float) * nd);
    put(c->r32, sizeof(float) * nd);
    put(c->z32, sizeof(float) * nd);
    put(c->q32, sizeof(float) * nd);
    put(c->p32[0], sizeof(float) * nd);
    put(c->p32[1], sizeof(float) * nd);
    put(c->c32, sizeof(float) * nd);
    if (useG(c)) put(c->spec32, sizeof(float2) * nspec32);
  }
  put(c->F, sizeof(double) * 24);
  put(c->macro, sizeof(double) * 8);
  put(c->st, sizeof(CgState));
  put(c->partA, sizeof(double) * c->npart);
  put(c->partB, sizeof(double) * c->npart);
  put(c->small, sizeof(double) * kSmall);
  for (int t = 0; t < 3; ++t) put(c->hist[t], sizeof(double) * kHistMax);
  const size_t slice = align_up(L.off, 256);
  if (base) c->cs = (long long)slice;
  Layout T;
  T.off = slice * (size_t)c->B;
  for (int a = 0; a < 3; ++a) {
    const int n = a == 0 ? c->g.nx : (a == 1 ? c->g.ny : c->g.nz);
    size_t o = T.take(sizeof(double2) * n);
    if (base) c->tw[a] = reinterpret_cast<double2 *>(base + o);
    for (int t = 0; t < 3; ++t) {
      o = T.take(sizeof(double) * n);
      if (base) c->ftab[a][t] = reinterpret_cast<double *>(base + o);
    }
  }
  return T.off;
}

// Output-node tile of the stiffness kernels (x and y edge) and the tile count of a grid.
// 2D block shapes (the tiles2d tunable): 1 = 16 x 16 nodes, 2 = 16 wide x 32,
// 3 = 32 wide x 16, 4 = 32 x 32.  3D block shapes (the tiles3d tunable): 1 =
// 16 x 14, 2 = 32 x 6.  Code 0 stands for the precision's
// default (measured best on the 512^2 groups and the 256^3 cell).
int resolve_tiles(int dim, bool fp64, int code) {
  if (code) return code;
  if (dim == 3) return fp64 ? default_tiles3d<double>() : default_tiles3d<float>();
  return fp64 ? default_tiles2d<double>() : default_tiles2d<float>();
}
int stencil_tile_x(int dim, bool fp64, int code = 0) {
  const int t = resolve_tiles(dim, fp64, code);
  if (dim == 3) return t == 2 ? Geo3<2>::TX : Geo3<1>::TX;
  return t >= 3 ? 2 * TILE : TILE;
}
int stencil_tile_y(int dim, bool fp64, int code = 0) {
  const int t = resolve_tiles(dim, fp64, code);
  if (dim == 3) return t == 2 ? Geo3<2>::TY : Geo3<1>::TY;
  return (t == 2 || t == 4) ? 2 * TILE : TILE;
}
long long stencil_tiles(int dim, int nx, int ny, bool fp64, int code = 0) {
  const int tx = stencil_tile_x(dim, fp64, code), ty = stencil_tile_y(dim, fp64, code);
  return (long long)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty);
}
// the most tiles any block shape of the dimension gives
long long stencil_tiles_max(int dim, int nx, int ny) {
  long long m = 0;
  for (int code = 1; code <= (dim == 3 ? 2 : 4); ++code)
    m = std::max(m, stencil_tiles(dim, nx, ny, false, code));
  return m;
}

long long max_partials(jfft_cell_s *c) {
  const GridDev &g = c->g;
  long long mx = 4 * 1024;  // vector kernels
  const long long tiles = stencil_tiles_max(c->dim, g.nx, g.ny);
  mx = std::max(mx, tiles * ((g.nz + 2 - 1) / 2));  // smallest z chunk allowed (tz >= 2)
  const long long rows = (long long)c->dim * g.ny * g.nz;
  mx = std::max(mx, rows);  // x passes at one row per block (the smallest xrows)
  mx = std::max(mx, (g.N + 255) / 256 * 6);  // stress partials [ds][blocks]
  mx = std::max(mx, (long long)((g.mx + 7) / 8) * (c->dim == 3 ? g.ny : 1));  // Green-pass r.z partials
  return mx;
}

jfft_status upload_tables(jfft_cell_s *c) {
  const int ns[3] = {c->g.nx, c->g.ny, c->g.nz};
  const double hs[3] = {c->len[0] / ns[0], c->len[1] / ns[1], c->dim == 3 ? c->len[2] / ns[2] : 1.0};
  for (int a = 0; a < 3; ++a) {
    const int n = ns[a];
    std::vector<double2> tw(n);
    std::vector<double> A(n), Bt(n), S(n);
    for (int j = 0; j < n; ++j) {
      const double t = 2.0 * M_PI * (double)j / (double)n;
      const double cs = std::cos(t), sn = std::sin(t);
      tw[j].x = cs;
      tw[j].y = -sn;
      // 2 - 2 cos(t) = 4 sin^2(t / 2), without the cancellation at small t
      const double sh = std::sin(M_PI * (double)j / (double)n);
      A[j] = 4.0 * sh * sh / hs[a];
      Bt[j] = hs[a] * (2.0 + cs) / 3.0;
      S[j] = sn;
    }
    HIP_TRY(hipMemcpyAsync(c->tw[a], tw.data(), sizeof(double2) * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ftab[a][0], A.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ftab[a][1], Bt.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->ftab[a][2], S.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));  // host vectors go out of scope
  return JFFT_OK;
}

// Kernels that may need more than 64 KiB of dynamic LDS (512-point axes in
// FP64): allow the 160 KiB of a CU, less the kernel's static LDS.
template <typename K>
hipError_t allow_big_lds(K *kernel) {
  hipFuncAttributes fa{};
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kernel));
  if (e != hipSuccess) return e;
  const int dyn = 160 * 1024 - (int)fa.sharedSizeBytes;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

template <typename Real>
hipError_t allow_big_lds_all() {
  hipError_t e = hipSuccess;
  auto keep = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  keep(allow_big_lds(k_ypass<Real, false, 256>));
  keep(allow_big_lds(k_ypass<Real, true, 256>));
  keep(allow_big_lds(k_ypass<Real, false, 512>));
  keep(allow_big_lds(k_ypass<Real, true, 512>));
  keep(allow_big_lds(k_green_axis<Real, 3, 2, 256>));
  keep(allow_big_lds(k_green_axis<Real, 3, 2, 512>));
  keep(allow_big_lds(k_green_axis<Real, 3, 1, 256>));
  keep(allow_big_lds(k_green_axis<Real, 3, 1, 512>));
  keep(allow_big_lds(k_green_axis<Real, 2, 1, 256>));
  keep(allow_big_lds(k_green_axis<Real, 2, 1, 512>));
  return e;
}

// Once per process; the result of the first call is kept.
hipError_t set_smem_attributes() {
  static std::once_flag once;
  static hipError_t status = hipSuccess;
  std::call_once(once, [] {
    status = allow_big_lds_all<double>();
    const hipError_t e2 = allow_big_lds_all<float>();
    if (status == hipSuccess) status = e2;
  });
  return status;
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
  TRY(upload_tables(c));
  c->drop_graphs();
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
  // cubic elements: half of lam, mu times k_c^2 = ih^2 / 3^c (mode class c)
  for (int k = 0; k < 3; ++k) {
    const double kc2 = c->g.ihx * c->g.ihx / (k == 0 ? 1.0 : (k == 1 ? 3.0 : 9.0));
    a.clam[k] = (Real)(0.5 * c->lam * c->g.w * kc2);
    a.cmu[k] = (Real)(0.5 * c->mu * c->g.w * kc2);
  }
  a.nx = c->g.nx;
  a.ny = c->g.ny;
  a.nz = c->g.nz;
  a.N = c->g.N;
  a.tz = c->dim == 3 ? std::min(c->tun.tz, c->g.nz) : 1;
  a.nbz = c->dim == 3 ? (c->g.nz + a.tz - 1) / a.tz : 1;
  a.cs = c->cs;
  a.st = c->st;
  if (c->nl) {
    if constexpr (std::is_same<Real, double>::value)
      a.uk = c->uk;
    else
      a.uk = c->uk32;
    a.pl = c->pl;
    a.w = (Real)c->g.w;
  }
  return a;
}

// 3D cells with equal element edges use the cubic form of the element kernel.
bool cubic_cells(const jfft_cell_s *c) {
  return c->dim == 3 && c->g.ihx == c->g.ihy && c->g.ihx == c->g.ihz;
}

// The 3D CG stiffness kernel of a precision, element form (cubic), material
// kind (mat: the power-law tangent) and block shape.
template <typename Real>
const void *stiffness_cg_kernel(bool cubic, bool mat, int shape) {
  if (mat)
    return shape == 2 ? reinterpret_cast<const void *>(k_stiffness3d<Real, SM_CG, false, 1, 2>)
                      : reinterpret_cast<const void *>(k_stiffness3d<Real, SM_CG, false, 1>);
  if (shape == 2)
    return cubic ? reinterpret_cast<const void *>(k_stiffness3d<Real, SM_CG, true, 0, 2>)
                 : reinterpret_cast<const void *>(k_stiffness3d<Real, SM_CG, false, 0, 2>);
  return cubic ? reinterpret_cast<const void *>(k_stiffness3d<Real, SM_CG, true>)
               : reinterpret_cast<const void *>(k_stiffness3d<Real, SM_CG, false>);
}

// Blocks of a 3D CG stiffness kernel that the device runs at once, and per CU.
hipError_t stiffness_slots(int device, const void *k, int *slots, int *per_cu_out) {
  int cus = 0, per_cu = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, STENCIL3_THREADS, 0);
  *slots = std::max(1, cus * per_cu);
  *per_cu_out = std::max(1, per_cu);
  return e;
}

// z planes per block of the 3D stiffness kernel.  The choice depends on the
// cell shape, the precision and the device only, never on the group size, so
// reduction layouts (and results) do not either.
// * One block per CU (FP64): the launch runs in rounds of co-resident blocks
//   and a block marches tz + 1 element layers, so the time is modelled as
//   rounds * (tz + 1), minimised over 4 <= tz <= 64 (ties: the larger tz,
//   which re-reads fewer halo planes).
// * Several blocks per CU: blocks that start together stay in step over a
//   long march and contend for the same units at the same time.  Measured
//   on 256^3 (FP32, ms per launch): 16 x 14 blocks 0.469 (tz 6), 0.460 (8
//   and 12), 0.448 (16), slower from 32 on; 32 x 6 blocks, which hold fewer
//   rows and re-read the two halo planes relatively more, 0.383 (8), 0.346
//   (16), 0.341 (20), 0.338 (32), 0.347 (64).  So 16 or 32 planes by the
//   block shape, shortened while the launch would leave slots empty.  (The
//   power-law tangent, two blocks per CU: 0.52 ms at 16 x 14 and 16 planes,
//   0.59 at 32 planes, 0.61 and 0.67 with 32 x 6 blocks; 200^3, FP32.)
int pick_tz(const GridDev &g, bool fp64, int shape, int slots, int per_cu) {
  const long long tiles = stencil_tiles(3, g.nx, g.ny, fp64, shape);
  const int lo = std::min(4, g.nz);
  auto blocks = [&](int tz) { return tiles * ((g.nz + tz - 1) / tz); };
  if (per_cu > 1) {
    int tz = std::min(shape == 2 ? 32 : 16, g.nz);
    while (tz > lo && blocks(tz) < slots) --tz;
    return tz;
  }
  const int hi = std::min(64, g.nz);
  int best = lo;
  long long best_cost = -1;
  for (int tz = lo; tz <= hi; ++tz) {
    const long long cost = (blocks(tz) + slots - 1) / slots * (tz + 1);
    if (best_cost < 0 || cost <= best_cost) {
      best_cost = cost;
      best = tz;
    }
  }
  return best;
}

// The tile-shape tunables apply to the kernels of the PCG loop's precision
// (FP32 in a mixed-precision cell); a mixed cell's FP64 kernels (residuals,
// post-processing) keep their defaults.
bool loop_precision(const jfft_cell_s *c, bool fp64) { return fp64 == (c->prec == JFFT_FP64); }

int tiles2d_of(const jfft_cell_s *c, bool fp64) {
  if (c->tun.tiles2d && loop_precision(c, fp64)) return c->tun.tiles2d;
  return fp64 ? default_tiles2d<double>() : default_tiles2d<float>();
}

// The power-law tangent keeps 16 x 14 blocks unless told otherwise (its two
// gradient sets leave two blocks per CU, where the wider block loses).
int tiles3d_of(const jfft_cell_s *c, bool fp64) {
  if (c->tun.tiles3d && loop_precision(c, fp64)) return c->tun.tiles3d;
  if (c->nl) return 1;
  return fp64 ? default_tiles3d<double>() : default_tiles3d<float>();
}

// z planes per block for the cell's material kind and block shape (see
// pick_tz), or 0 on a HIP error.
int auto_tz(const jfft_cell_s *c, hipError_t *err) {
  const bool fp64 = c->prec == JFFT_FP64;
  const int shape = tiles3d_of(c, fp64);
  const bool cubic = cubic_cells(c);
  const void *k = fp64 ? stiffness_cg_kernel<double>(cubic, c->nl, shape)
                       : stiffness_cg_kernel<float>(cubic, c->nl, shape);
  int slots = 0, per_cu = 0;
  *err = stiffness_slots(c->device, k, &slots, &per_cu);
  return *err == hipSuccess ? pick_tz(c->g, fp64, shape, slots, per_cu) : 0;
}

// Re-picks tz after a change of material kind (or when the automatic choice
// is restored), unless tz was set explicitly (and unless the group would
// exceed the grid's z-dimension).
jfft_status refresh_tz(jfft_cell_s *c) {
  if (c->dim != 3 || !c->tun.tz_auto) return JFFT_OK;
  hipError_t e = hipSuccess;
  const int tz = auto_tz(c, &e);
  if (e != hipSuccess) return fail(JFFT_E_HIP, std::string("occupancy query: ") + hipGetErrorString(e));
  if (tz != c->tun.tz && (long long)((c->g.nz + tz - 1) / tz) * c->B <= 65535) {
    c->tun.tz = tz;
    c->drop_graphs();
  }
  return JFFT_OK;
}

// The resolved block shape of the stiffness kernels of a precision.
int tiles_of(const jfft_cell_s *c, bool fp64) {
  return c->dim == 3 ? tiles3d_of(c, fp64) : tiles2d_of(c, fp64);
}

long long stencil_blocks_per_cell(jfft_cell_s *c, bool fp64) {
  const GridDev &g = c->g;
  const int tz = c->dim == 3 ? std::min(c->tun.tz, g.nz) : 1;
  const int nbz = c->dim == 3 ? (g.nz + tz - 1) / tz : 1;
  return stencil_tiles(c->dim, g.nx, g.ny, fp64, tiles_of(c, fp64)) * nbz;
}

template <typename Real, int MODE>
jfft_status launch_stiffness(jfft_cell_s *c, const StencilArgs<Real> &a, int cells) {
  const int kid = MODE == SM_CG ? KID_STIFF_CG : (MODE == SM_APPLY ? KID_STIFF_APPLY : KID_STIFF_COMB);
  const GridDev &g = c->g;
  const int tt = tiles_of(c, sizeof(Real) == 8);
  const int tx = stencil_tile_x(c->dim, sizeof(Real) == 8, tt),
            ty = stencil_tile_y(c->dim, sizeof(Real) == 8, tt);
  dim3 gr((g.nx + tx - 1) / tx, (g.ny + ty - 1) / ty, a.nbz * cells);
  if (c->nl) {
    // the power-law tangent (3D cells, checked when the material is set);
    // Algorithm 2's combs run in FP64 only
    if constexpr (std::is_same<Real, double>::value || MODE != SM_COMB) {
      if (tt == 2)
        LAUNCH(c, kid, (k_stiffness3d<Real, MODE, false, 1, 2><<<gr, STENCIL3_THREADS, 0, c->stream>>>(a)));
      else
        LAUNCH(c, kid, (k_stiffness3d<Real, MODE, false, 1><<<gr, STENCIL3_THREADS, 0, c->stream>>>(a)));
      return JFFT_OK;
    }
    return fail(JFFT_E_INVALID, "the power-law combs run in FP64 only");
  }
  if (c->dim == 3) {
    const bool cubic = cubic_cells(c);
    if (tt == 2) {
      if (cubic)
        LAUNCH(c, kid, (k_stiffness3d<Real, MODE, true, 0, 2><<<gr, STENCIL3_THREADS, 0, c->stream>>>(a)));
      else
        LAUNCH(c, kid, (k_stiffness3d<Real, MODE, false, 0, 2><<<gr, STENCIL3_THREADS, 0, c->stream>>>(a)));
      return JFFT_OK;
    }
    if (cubic)
      LAUNCH(c, kid, (k_stiffness3d<Real, MODE, true><<<gr, STENCIL3_THREADS, 0, c->stream>>>(a)));
    else
      LAUNCH(c, kid, (k_stiffness3d<Real, MODE, false><<<gr, STENCIL3_THREADS, 0, c->stream>>>(a)));
  } else if (c->elem == JFFT_ELEM_TRI) {
    switch (tt) {
      case 2: LAUNCH(c, kid, (k_stiffness2d<Real, MODE, true, 2, TILE><<<gr, STENCIL_THREADS, 0, c->stream>>>(a))); break;
      case 3: LAUNCH(c, kid, (k_stiffness2d<Real, MODE, true, 1, 2 * TILE><<<gr, STENCIL_THREADS, 0, c->stream>>>(a))); break;
      case 4: LAUNCH(c, kid, (k_stiffness2d<Real, MODE, true, 2, 2 * TILE><<<gr, STENCIL_THREADS, 0, c->stream>>>(a))); break;
      default: LAUNCH(c, kid, (k_stiffness2d<Real, MODE, true, 1, TILE><<<gr, STENCIL_THREADS, 0, c->stream>>>(a))); break;
    }
  } else {
    switch (tt) {
      case 2: LAUNCH(c, kid, (k_stiffness2d<Real, MODE, false, 2, TILE><<<gr, STENCIL_THREADS, 0, c->stream>>>(a))); break;
      case 3: LAUNCH(c, kid, (k_stiffness2d<Real, MODE, false, 1, 2 * TILE><<<gr, STENCIL_THREADS, 0, c->stream>>>(a))); break;
      case 4: LAUNCH(c, kid, (k_stiffness2d<Real, MODE, false, 2, 2 * TILE><<<gr, STENCIL_THREADS, 0, c->stream>>>(a))); break;
      default: LAUNCH(c, kid, (k_stiffness2d<Real, MODE, false, 1, TILE><<<gr, STENCIL_THREADS, 0, c->stream>>>(a))); break;
    }
  }
  return JFFT_OK;
}

// out = K in for `cells` cells of the group (pointers of cell 0, slice stride).
template <typename Real>
jfft_status apply_K(jfft_cell_s *c, const Real *E, const Real *in, Real *out, int cells) {
  StencilArgs<Real> a = stencil_args<Real>(c, E);
  a.in = in;
  a.out = out;
  return launch_stiffness<Real, SM_APPLY>(c, a, cells);
}

template <typename Real>
XArgs<Real> x_args(jfft_cell_s *c, bool check_done) {
  XArgs<Real> a{};
  a.st = c->st;
  a.tw = c->tw[0];
  a.plan = c->plan_x;
  a.nx = c->g.nx;
  a.mx = c->g.mx;
  a.ntx = ntx_of<Real>(c);
  a.ny = c->g.ny;
  a.nrows = (long long)c->dim * c->g.ny * c->g.nz;
  a.rows_per_block = x_rows_per_block<Real>(c->g.nx / 2);
  if (c->tun.xrows && c->tun.xrows < a.rows_per_block && loop_precision(c, sizeof(Real) == 8))
    a.rows_per_block = c->tun.xrows;
  a.log2_rb = 0;
  while ((1 << a.log2_rb) < a.rows_per_block) ++a.log2_rb;
  a.dm = FastDiv(c->g.nx / 2);
  a.dhalf = FastDiv(c->g.nx / 4 + 1);
  a.check_done = check_done ? 1 : 0;
  a.cs = c->cs;
  return a;
}

// Forward x pass: spec = rfft_x(J^1/2 (r - alpha q)), partA = ||r||^2 partials.
template <typename Real>
jfft_status launch_xfwd(jfft_cell_s *c, Real *r, const Real *q, const Real *Jh,
                        typename CxT<Real>::T *spec, double *partA, bool update, bool check_done,
                        long long *nblk, bool fuse = false, History h = {nullptr, nullptr, nullptr}) {
  using C = typename CxT<Real>::T;
  XArgs<Real> a = x_args<Real>(c, check_done);
  a.ctl = fuse ? c->st : nullptr;
  a.h = h;
  a.r = r;
  a.q = q;
  a.Jh = Jh;
  a.spec = spec;
  a.partA = partA;
  const int m = c->g.nx / 2;
  const long long nb = (a.nrows + a.rows_per_block - 1) / a.rows_per_block;
  const size_t smem = sizeof(C) * (c->g.nx + (size_t)a.rows_per_block * (m + 1));
  *nblk = nb;
  dim3 gr((unsigned)nb, c->B);
  if (update) {
    if (Jh)
      LAUNCH(c, KID_XFWD, k_xfwd<Real, true, true><<<gr, FFT_THREADS, smem, c->stream>>>(a));
    else
      LAUNCH(c, KID_XFWD, k_xfwd<Real, true, false><<<gr, FFT_THREADS, smem, c->stream>>>(a));
  } else {
    if (Jh)
      LAUNCH(c, KID_XFWD, k_xfwd<Real, false, true><<<gr, FFT_THREADS, smem, c->stream>>>(a));
    else
      LAUNCH(c, KID_XFWD, k_xfwd<Real, false, false><<<gr, FFT_THREADS, smem, c->stream>>>(a));
  }
  return JFFT_OK;
}

// Inverse x pass: out = J^1/2 irfft_x(spec) (r.z comes from the Green pass).
template <typename Real>
jfft_status launch_xinv(jfft_cell_s *c, const Real *Jh, typename CxT<Real>::T *spec, Real *out,
                        bool check_done) {
  using C = typename CxT<Real>::T;
  XArgs<Real> a = x_args<Real>(c, check_done);
  a.Jh = Jh;
  a.out = out;
  a.spec = spec;
  const int m = c->g.nx / 2;
  const long long nb = (a.nrows + a.rows_per_block - 1) / a.rows_per_block;
  const size_t smem = sizeof(C) * (c->g.nx + (size_t)a.rows_per_block * (m + 1));
  dim3 gr((unsigned)nb, c->B);
  if (Jh)
    LAUNCH(c, KID_XINV, k_xinv<Real, true><<<gr, FFT_THREADS, smem, c->stream>>>(a));
  else
    LAUNCH(c, KID_XINV, k_xinv<Real, false><<<gr, FFT_THREADS, smem, c->stream>>>(a));
  return JFFT_OK;
}

// threads for a tile of `pts` complex points (MaxPt points per thread)
template <typename Real>
int tile_threads(long long pts) {
  return pts <= (long long)MaxPt<Real>::value * 256 ? 256 : 512;
}

template <typename Real>
jfft_status launch_ypass(jfft_cell_s *c, typename CxT<Real>::T *spec, bool inv, bool check_done) {
  using C = typename CxT<Real>::T;
  YArgs<Real> a{};
  a.spec = spec;
  a.st = c->st;
  a.tw = c->tw[1];
  a.plan = c->plan_y;
  a.ntx = ntx_of<Real>(c);
  a.ny = c->g.ny;
  a.nz = c->g.nz;
  a.check_done = check_done ? 1 : 0;
  a.cs = c->cs;
  // persistent blocks, each walking tiles of one (component, cell)
  const long long per_comp = (long long)a.ntx * c->g.nz;
  const long long want = std::max<long long>(1, c->tun.ygrid / ((long long)c->dim * c->B));
  dim3 gr((unsigned)std::min(per_comp, want), c->dim, c->B);
  const long long pts = (long long)c->g.ny * TileW<Real>::value;
  const size_t smem = sizeof(C) * ((size_t)c->g.ny + (size_t)pts);
  const int kid = inv ? KID_YINV : KID_YFWD;
  if (tile_threads<Real>(pts) == 256) {
    if (inv) LAUNCH(c, kid, k_ypass<Real, true, 256><<<gr, 256, smem, c->stream>>>(a));
    else LAUNCH(c, kid, k_ypass<Real, false, 256><<<gr, 256, smem, c->stream>>>(a));
  } else {
    if (inv) LAUNCH(c, kid, k_ypass<Real, true, 512><<<gr, 512, smem, c->stream>>>(a));
    else LAUNCH(c, kid, k_ypass<Real, false, 512><<<gr, 512, smem, c->stream>>>(a));
  }
  return JFFT_OK;
}

// Green pass (last axis): also writes the r.z partials to partB; *nblk
// receives their number per cell.
template <typename Real>
jfft_status launch_green(jfft_cell_s *c, typename CxT<Real>::T *spec, bool check_done,
                         long long *nblk, bool fuse = false, History h = {nullptr, nullptr, nullptr}) {
  using C = typename CxT<Real>::T;
  GArgs<Real> a{};
  a.spec = spec;
  a.partB = c->partB;
  a.st = c->st;
  a.ctl = fuse ? c->st : nullptr;
  a.h = h;
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
  a.ntx = ntx_of<Real>(c);
  a.ny = c->g.ny;
  a.nz = c->g.nz;
  a.check_done = check_done ? 1 : 0;
  a.cs = c->cs;
  a.tri = c->elem == JFFT_ELEM_TRI ? 1 : 0;
  std::memcpy(a.tS, c->tS, sizeof(a.tS));
  a.hx = c->len[0] / c->n[0];
  a.hy = c->len[1] / c->n[1];
  constexpr int TW = TileW<Real>::value;
  const int L = c->dim == 3 ? c->g.nz : c->g.ny;
  if (c->dim == 3) {
    // ky rows per tile for full 128-byte lines, while the tile fits 512 threads
    const int KY = (long long)L * ZRows<Real>::value * TW <= (long long)MaxPt<Real>::value * 512
                       ? ZRows<Real>::value
                       : 1;
    const long long pts = (long long)L * KY * TW;
    const size_t smem = sizeof(C) * ((size_t)L + (size_t)pts) + sizeof(Real) * 3 * (size_t)L;
    dim3 gr((unsigned)(a.ntx * (c->g.ny / KY)), 1, c->B);
    *nblk = gr.x;
    const int nt = tile_threads<Real>(pts);
    if (KY == 2 && nt == 256)
      LAUNCH(c, KID_GREEN, k_green_axis<Real, 3, 2, 256><<<gr, 256, smem, c->stream>>>(a));
    else if (KY == 2)
      LAUNCH(c, KID_GREEN, k_green_axis<Real, 3, 2, 512><<<gr, 512, smem, c->stream>>>(a));
    else if (nt == 256)
      LAUNCH(c, KID_GREEN, k_green_axis<Real, 3, 1, 256><<<gr, 256, smem, c->stream>>>(a));
    else
      LAUNCH(c, KID_GREEN, k_green_axis<Real, 3, 1, 512><<<gr, 512, smem, c->stream>>>(a));
  } else {
    const long long pts = (long long)L * TW;
    const size_t smem = sizeof(C) * ((size_t)L + (size_t)pts) + sizeof(Real) * 3 * (size_t)L;
    dim3 gr((unsigned)a.ntx, 1, c->B);
    *nblk = gr.x;
    if (tile_threads<Real>(pts) == 256)
      LAUNCH(c, KID_GREEN, k_green_axis<Real, 2, 1, 256><<<gr, 256, smem, c->stream>>>(a));
    else
      LAUNCH(c, KID_GREEN, k_green_axis<Real, 2, 1, 512><<<gr, 512, smem, c->stream>>>(a));
  }
  return JFFT_OK;
}

// z = M^-1 r.  update: r <- r - alpha q first.  Partials: partA = ||r||^2,
// partB = r.z.  In the loop, the CG control steps run between the pieces:
// in the last blocks of the x-forward and Green passes (fused control), or
// as single-block kernels.
template <typename Real>
jfft_status precond(jfft_cell_s *c, Real *r, const Real *q, const Real *Jh, Real *z,
                    typename CxT<Real>::T *spec, bool update, bool in_loop, long long *nA,
                    long long *nB, History h) {
  const int Bc = c->B;
  if (!useG(c)) {
    const long long n = (long long)c->dim * c->g.N;
    const int nb = vec_blocks(n);
    *nA = *nB = nb;
    const int cd = in_loop ? 1 : 0;
    dim3 gr(nb, Bc);
    const Real *J = useJ(c) ? Jh : nullptr;
    if (update) {
      if (J)
        LAUNCH(c, KID_DIAGPC, k_diag_pc<Real, true, true><<<gr, 256, 0, c->stream>>>(r, q, J, z, n, c->st, cd, c->partA, c->partB, c->cs));
      else
        LAUNCH(c, KID_DIAGPC, k_diag_pc<Real, true, false><<<gr, 256, 0, c->stream>>>(r, q, J, z, n, c->st, cd, c->partA, c->partB, c->cs));
    } else {
      if (J)
        LAUNCH(c, KID_DIAGPC, k_diag_pc<Real, false, true><<<gr, 256, 0, c->stream>>>(r, q, J, z, n, c->st, cd, c->partA, c->partB, c->cs));
      else
        LAUNCH(c, KID_DIAGPC, k_diag_pc<Real, false, false><<<gr, 256, 0, c->stream>>>(r, q, J, z, n, c->st, cd, c->partA, c->partB, c->cs));
    }
    if (in_loop) {
      LAUNCH(c, KID_CTRL, k_cg_rr<<<Bc, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, *nA, h, c->cs));
      LAUNCH(c, KID_CTRL, k_cg_beta<<<Bc, CTRL_THREADS, 0, c->stream>>>(c->st, c->partB, *nB, h, c->cs));
    }
    return JFFT_OK;
  }
  const Real *J = useJ(c) ? Jh : nullptr;
  const bool fuse = in_loop && c->tun.fused_control;
  TRY(launch_xfwd<Real>(c, r, q, J, spec, c->partA, update, in_loop, nA, fuse, h));
  if (in_loop && !fuse) LAUNCH(c, KID_CTRL, k_cg_rr<<<Bc, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, *nA, h, c->cs));
  if (c->dim == 3) {
    TRY(launch_ypass<Real>(c, spec, false, in_loop));
    TRY(launch_green<Real>(c, spec, in_loop, nB, fuse, h));
    TRY(launch_ypass<Real>(c, spec, true, in_loop));
  } else {
    TRY(launch_green<Real>(c, spec, in_loop, nB, fuse, h));
  }
  TRY(launch_xinv<Real>(c, J, spec, z, in_loop));
  if (in_loop && !fuse) LAUNCH(c, KID_CTRL, k_cg_beta<<<Bc, CTRL_THREADS, 0, c->stream>>>(c->st, c->partB, *nB, h, c->cs));
  return JFFT_OK;
}

// One PCG iteration j (p_old = p[j & 1], p_new = p[(j + 1) & 1]).
template <typename Real>
jfft_status pcg_iteration(jfft_cell_s *c, const PcgBufs<Real> &b, int j, History h) {
  StencilArgs<Real> a = stencil_args<Real>(c, b.E);
  a.in = b.p[j & 1];
  a.zin = b.z;
  a.pout = b.p[(j + 1) & 1];
  a.u = b.u;
  a.out = b.q;
  a.partial = c->partA;
  // the Green path fuses the alpha step into the stiffness kernel (the
  // diagonal preconditioners launch all three steps on their own)
  const bool fuse = c->tun.fused_control && useG(c);
  a.ctl = fuse ? c->st : nullptr;
  a.h = h;
  a.parity = (j + 1) & 1;
  TRY((launch_stiffness<Real, SM_CG>(c, a, c->B)));
  const long long nK = stencil_blocks_per_cell(c, sizeof(Real) == 8);
  if (!fuse)
    LAUNCH(c, KID_CTRL, k_cg_alpha<<<c->B, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, nK, h, (j + 1) & 1, c->cs));
  long long nA, nB;
  return precond<Real>(c, b.r, b.q, b.Jh, b.z, b.spec, true, true, &nA, &nB, h);
}

// Iterations until the slowest running cell of the group stops, predicted
// from its average convergence rate so far (||r||^2 decays about
// geometrically), so that few launches go out after the stop; 0 when every
// cell has stopped.  Launches past a cell's stop are harmless (its kernels
// return at once) but cost launch time and would blur per-kernel timings.
int predict_remaining(const jfft_cell_s *c) {
  int need = 0;
  for (int i = 0; i < c->B; ++i) {
    const CgState &s = c->st_h[i];
    if (s.done) continue;
    int rem = 32;
    if (s.iter > 0 && s.rr > 0.0 && s.rr0 > s.rr && s.tol2 > 0.0) {
      const double rate = std::log(s.rr0 / s.rr) / s.iter;
      rem = (int)std::ceil(0.85 * std::log(s.rr / s.tol2) / rate);
    }
    rem = std::max(1, std::min(rem, s.maxit - s.iter));
    need = std::max(need, rem);
  }
  return need;
}

jfft_status fetch_states(jfft_cell_s *c) {
  HIP_TRY(hipMemcpy2DAsync(c->st_h, sizeof(CgState), c->st, (size_t)c->cs, sizeof(CgState), c->B,
                           hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return JFFT_OK;
}

// Start of the PCG loop on prepared buffers (u = start vector, r = f - K u)
// for every cell of the group: state, z_0 = M^-1 r_0, ||r_0||^2 and r.z.
// cont (mixed refinement sweeps after the first): continue the previous
// sweep's CG with its rescaled search direction (k_cg_init_continue).
template <typename Real>
jfft_status pcg_begin(jfft_cell_s *c, const PcgBufs<Real> &b, bool mixed, int maxit, History h,
                      bool cont) {
  long long nA = 0, nB = 0;
  const double itol = c->mixed_continue ? c->update_tol : c->inner_tol;
  if (cont) {
    LAUNCH(c, KID_CTRL, k_cg_init_continue<<<c->B, 1, 0, c->stream>>>(c->st, itol, maxit, c->inner_cap, c->cs));
    const long long n = (long long)c->dim * c->g.N;
    LAUNCH(c, KID_VEC, k_scale_direction<Real><<<dim3(vec_blocks(n), c->B), 256, 0, c->stream>>>(b.p[0], b.p[1], n, c->st, c->cs));
  } else {
    LAUNCH(c, KID_CTRL, k_cg_init<<<c->B, 1, 0, c->stream>>>(c->st, itol, mixed ? 1 : 0, maxit, h.alpha ? c->hist_cap : 0, c->inner_cap, c->cs));
  }
  TRY(precond<Real>(c, b.r, nullptr, b.Jh, b.z, b.spec, false, false, &nA, &nB, h));
  if (cont)
    LAUNCH(c, KID_CTRL, k_cg_start_continue<<<c->B, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, nA, c->partB, nB, c->cs));
  else
    LAUNCH(c, KID_CTRL, k_cg_start<<<c->B, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, nA, c->partB, nB, c->cs));
  return JFFT_OK;
}

// The captured chunk of G = tun.graph_iters iterations for this precision
// and the c->B cells launched, built when missing.  Its arguments never
// change (the buffers of this handle are fixed) and the CG state lives in
// device memory, so one capture serves every later loop.
template <typename Real>
jfft_status ensure_graph(jfft_cell_s *c, const PcgBufs<Real> &b, History h,
                         hipGraphExec_t *out) {
  const int fp64 = sizeof(Real) == 8 ? 1 : 0;
  const int G = c->tun.graph_iters;
  for (const auto &g : c->graphs)
    if (g.fp64 == fp64 && g.cells == c->B && g.iters == G) {
      *out = g.exec;
      return JFFT_OK;
    }
  hipGraph_t gr = nullptr;
  HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  jfft_status s = JFFT_OK;
  for (int j = 1; j <= G && s == JFFT_OK; ++j) s = pcg_iteration<Real>(c, b, j, h);
  c->capturing = false;
  hipError_t e = hipStreamEndCapture(c->stream, &gr);
  if (s) return s;
  if (e != hipSuccess) return fail(JFFT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) return fail(JFFT_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  c->graphs.push_back({fp64, c->B, G, ex});
  *out = ex;
  return JFFT_OK;
}

// At least `iters` PCG iterations of every running cell among the c->B
// launched: whole replays of the captured chunk, or direct launches (an
// even count, so that every chunk starts on the same search-direction
// buffer).
template <typename Real>
jfft_status pcg_iterations(jfft_cell_s *c, const PcgBufs<Real> &b, int iters, History h) {
  const int G = c->tun.graph_iters;
  if (G > 0 && !c->timing) {
    hipGraphExec_t ex = nullptr;
    TRY(ensure_graph<Real>(c, b, h, &ex));
    const int reps = std::max(1, (iters + G / 2) / G);
    for (int k = 0; k < reps; ++k) HIP_TRY(hipGraphLaunch(ex, c->stream));
  } else {
    const int n = iters + (iters & 1);
    for (int j = 1; j <= n; ++j) TRY(pcg_iteration<Real>(c, b, j, h));
  }
  return JFFT_OK;
}

// the owed update u += alpha p_k of every cell after its loop stopped
template <typename Real>
jfft_status pcg_finish(jfft_cell_s *c, const PcgBufs<Real> &b) {
  const long long n = (long long)c->dim * c->g.N;
  LAUNCH(c, KID_VEC, k_finish_u<Real><<<dim3(vec_blocks(n), c->B), 256, 0, c->stream>>>(b.u, b.p[0], b.p[1], n, c->st, c->cs));
  return JFFT_OK;
}

// PCG loop after pcg_begin for every cell of the group; returns when every
// cell's flag is set, with the owed updates applied.
template <typename Real>
jfft_status pcg_loop(jfft_cell_s *c, const PcgBufs<Real> &b, History h) {
  int chunk = 2;
  for (;;) {
    TRY(pcg_iterations<Real>(c, b, chunk, h));
    TRY(fetch_states(c));
    const int need = predict_remaining(c);
    if (need == 0) break;
    chunk = std::max(1, std::min(need, std::min(chunk * 2, 32)));
  }
  return pcg_finish<Real>(c, b);
}

jfft_status reduce_to(jfft_cell_s *c, const double *part, long long n, int groups, int slot,
                      int cells) {
  LAUNCH(c, KID_REDUCE, k_reduce_groups<<<cells, CTRL_THREADS, 0, c->stream>>>(part, n, groups, c->small + slot, c->cs));
  return JFFT_OK;
}

// CG states and reduction results of every cell, with one synchronisation.
jfft_status fetch_all(jfft_cell_s *c) {
  HIP_TRY(hipMemcpy2DAsync(c->st_h, sizeof(CgState), c->st, (size_t)c->cs, sizeof(CgState), c->B,
                           hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpy2DAsync(c->small_h, sizeof(double) * kSmall, c->small, (size_t)c->cs,
                           sizeof(double) * kSmall, c->B, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return JFFT_OK;
}

jfft_status fetch_small(jfft_cell_s *c) {
  HIP_TRY(hipMemcpy2DAsync(c->small_h, sizeof(double) * kSmall, c->small, (size_t)c->cs,
                           sizeof(double) * kSmall, c->B, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return JFFT_OK;
}

// Macro strains (host, [cells][d*]) into each cell's slice, then f (and |f|).
jfft_status assemble_rhs(jfft_cell_s *c, const double *macros_h, double *f, double *fabs_out,
                         int cells) {
  const int ds = c->dim * (c->dim + 1) / 2;
  HIP_TRY(hipMemcpy2DAsync(c->macro, (size_t)c->cs, macros_h, sizeof(double) * ds, sizeof(double) * ds,
                           cells, hipMemcpyHostToDevice, c->stream));
  LAUNCH(c, KID_RHS, k_unit_force<<<cells, 1, 0, c->stream>>>(c->F, c->macro, c->dim, c->lam * c->g.w, c->mu * c->g.w, c->g.ihx, c->g.ihy, c->g.ihz, c->cs, c->elem == JFFT_ELEM_TRI ? 1 : 0));
  const long long N = c->g.N;
  LAUNCH(c, KID_RHS, k_rhs<double><<<dim3((unsigned)((N + 255) / 256), cells), 256, 0, c->stream>>>(c->E, c->F, f, fabs_out, c->dim, c->g.nx, c->g.ny, c->g.nz, N, c->cs));
  return JFFT_OK;
}

jfft_status run_alg2(jfft_cell_s *c, double *diag_out, int cells) {
  StencilArgs<double> a = stencil_args<double>(c, c->E);
  a.diag = diag_out;
  const int nloc = 1 << c->dim;
  for (int comp = 0; comp < c->dim; ++comp)
    for (int off = 0; off < nloc; ++off) {
      a.comb_comp = comp;
      a.comb_off = off;
      TRY((launch_stiffness<double, SM_COMB>(c, a, cells)));
    }
  return JFFT_OK;
}

// Algorithm 2's diagonal in closed form (isotropic Q1): diag = k_alpha * box sum of E.
jfft_status run_diag_closed(jfft_cell_s *c, double *diag_out, int cells) {
  const GridDev &g = c->g;
  const int d = c->dim;
  const double ih[3] = {g.ihx, g.ihy, g.ihz};
  double vol = 1.0;
  for (int a = 0; a < d; ++a) vol /= ih[a];
  const double p3 = d == 3 ? 9.0 : 3.0;  // 3^(d-1)
  double gb[3] = {0, 0, 0}, gs = 0.0;
  for (int a = 0; a < d; ++a) {
    gb[a] = vol * ih[a] * ih[a] / p3;
    gs += gb[a];
  }
  double k[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) k[a] = c->lam * gb[a] + c->mu * (gb[a] + gs);
  const dim3 gr(vec_blocks(g.N), cells);
  if (d == 3)
    LAUNCH(c, KID_SETUP, k_diag_closed<3><<<gr, 256, 0, c->stream>>>(c->E, diag_out, g.nx, g.ny, g.nz, g.N, k[0], k[1], k[2], c->cs));
  else
    LAUNCH(c, KID_SETUP, k_diag_closed<2><<<gr, 256, 0, c->stream>>>(c->E, diag_out, g.nx, g.ny, g.nz, g.N, k[0], k[1], k[2], c->cs));
  return JFFT_OK;
}

// Stencil of K_ref (unit modulus, Lame constants lam, mu) for the 2D linear
// triangles: the pixel matrix Ke (both triangles of elem_tri2, one point of
// weight A = hx hy / 2 each) folded by corner offset, S_d = sum over corner
// pairs (a, b) with x_b - x_a = d of the 2 x 2 block Ke[a][b]; stored as
// (S_00, S_11, S_01) at index (dy + 1) * 3 + dx + 1.
void tri_stencil(jfft_cell_s *c, double lam, double mu) {
  const double ix = c->g.ihx, iy = c->g.ihy, A = 0.5 / (ix * iy);
  // corner gradients per triangle: T0 = (0, 1, 2), T1 = (3, 2, 1)
  const int corners[2][3] = {{0, 1, 2}, {3, 2, 1}};
  const double grads[2][3][2] = {{{-ix, -iy}, {ix, 0.0}, {0.0, iy}},
                                 {{ix, iy}, {-ix, 0.0}, {0.0, -iy}}};
  double Ke[4][4][2][2] = {};  // [a][b][i][j]
  for (int t = 0; t < 2; ++t)
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        const double ax = grads[t][p][0], ay = grads[t][p][1];
        const double bx = grads[t][q][0], by = grads[t][q][1];
        // B_a^T C B_b for plane strain: the 2 x 2 block of corner pair (a, b)
        double k[2][2];
        k[0][0] = (lam + 2 * mu) * ax * bx + mu * ay * by;
        k[1][1] = (lam + 2 * mu) * ay * by + mu * ax * bx;
        k[0][1] = lam * ax * by + mu * ay * bx;
        k[1][0] = lam * ay * bx + mu * ax * by;
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) Ke[corners[t][p]][corners[t][q]][i][j] += A * k[i][j];
      }
  std::memset(c->tS, 0, sizeof(c->tS));
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      const int dx = (b & 1) - (a & 1), dy = (b >> 1) - (a >> 1);
      const int o = (dy + 1) * 3 + dx + 1;
      c->tS[o][0] += Ke[a][b][0][0];
      c->tS[o][1] += Ke[a][b][1][1];
      c->tS[o][2] += Ke[a][b][0][1];
    }
}

// E_dev holds the moduli of the cells one after another ([B][N]), or with
// broadcast one field for every cell of the group.
bool slots_busy(const jfft_cell_s *c);
constexpr const char *kSlotsBusy = "the group's slots hold running or unharvested solves";

// defer_check (slot admission): the count of bad entries of E stays in the
// cell's reduction results (small[0]) for k_slot_validate instead of being
// read back here, so that admission does not synchronise.
jfft_status set_material_impl(jfft_cell_s *c, const double *E_dev, double lam, double mu,
                              bool broadcast = false, bool defer_check = false) {
  if (!E_dev) return fail(JFFT_E_INVALID, "E_dev is NULL");
  if (slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!(mu > 0.0) || !(lam + 2.0 * mu / c->dim > 0.0) || !std::isfinite(lam) || !std::isfinite(mu))
    return fail(JFFT_E_INVALID, "Lame constants must satisfy mu > 0 and lambda + 2 mu / d > 0");
  TRY(ensure_ready(c));
  if (c->nl) {  // back from the power-law material: its captured kernels differ
    c->nl = false;
    c->drop_graphs();
    TRY(refresh_tz(c));
  }
  // captured iterations carry lambda and mu as kernel arguments; the moduli
  // are read from the workspace, so a new E alone keeps them valid
  if (c->lam != lam || c->mu != mu) c->drop_graphs();
  c->has_material = false;
  c->lam = lam;
  c->mu = mu;
  if (c->elem == JFFT_ELEM_TRI) tri_stencil(c, lam, mu);
  const long long N = c->g.N;
  const long long es = broadcast ? 0 : (long long)sizeof(double) * N;  // caller's layout
  const int nb = vec_blocks(N);
  LAUNCH(c, KID_SETUP, k_check_E<<<dim3(nb, c->B), 256, 0, c->stream>>>(E_dev, es, N, c->partA, c->cs));
  TRY(reduce_to(c, c->partA, nb, 1, 0, c->B));
  if (!defer_check) {
    TRY(fetch_small(c));
    for (int i = 0; i < c->B; ++i)
      if (c->small_h[(size_t)i * kSmall] != 0.0)
        return fail(JFFT_E_INVALID, "E contains negative or non-finite entries (cell " + std::to_string(i) + ")");
  }
  LAUNCH(c, KID_SETUP, k_copy<double><<<dim3(nb, c->B), 256, 0, c->stream>>>(E_dev, es, c->E, c->cs, N));
  const long long nd = (long long)c->dim * N;
  const int nbd = vec_blocks(nd);
  if (useJ(c)) {
    // the closed form is that of the quadrilateral; triangles take Algorithm 2
    if (c->diag_method == JFFT_DIAG_PROBING || c->elem == JFFT_ELEM_TRI)
      TRY(run_alg2(c, c->diag, c->B));
    else
      TRY(run_diag_closed(c, c->diag, c->B));
    LAUNCH(c, KID_SETUP, k_jhalf<double><<<dim3(nbd, c->B), 256, 0, c->stream>>>(c->diag, c->Jh, nd, c->void_value, c->cs));
  }
  if (c->prec == JFFT_MIXED) {
    LAUNCH(c, KID_SETUP, (k_convert<double, float><<<dim3(nb, c->B), 256, 0, c->stream>>>(c->E, c->E32, N, 1.0, nullptr, c->cs)));
    if (useJ(c))
      LAUNCH(c, KID_SETUP, k_jhalf<float><<<dim3(nbd, c->B), 256, 0, c->stream>>>(c->diag, c->Jh32, nd, c->void_value, c->cs));
  }
  c->has_material = true;
  return JFFT_OK;
}

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
  return ms;
}

// sigma_bar of every cell from the fetched reduction results.
void read_sigma_bar(const jfft_cell_s *c, double *sigma_bar) {
  const int ds = c->dim * (c->dim + 1) / 2;
  for (int i = 0; i < c->B; ++i)
    for (int r = 0; r < ds; ++r)
      sigma_bar[(size_t)i * ds + r] = c->small_h[(size_t)i * kSmall + 16 + r] / c->g.vol;
}

// True residual, mean removal (Sec. 5), stresses and sigma_bar; results to
// the caller's arrays.  fetch = false: the caller fetches the results
// (fetch_all) and reads sigma_bar (read_sigma_bar) itself.
jfft_status post_process(jfft_cell_s *c, double *u_out, double *sigma_dev, double *sigma_bar,
                         bool fetch = true) {
  const long long N = c->g.N;
  const int d = c->dim;
  const long long nd = (long long)d * N;
  const int ds = d * (d + 1) / 2;
  const int Bc = c->B;
  TRY(apply_K<double>(c, c->E, c->u, c->q, Bc));
  const int nb = vec_blocks(nd);
  LAUNCH(c, KID_VEC, k_sub_norm<double><<<dim3(nb, Bc), 256, 0, c->stream>>>(c->f, c->q, nullptr, nd, c->partA, c->cs));
  TRY(reduce_to(c, c->partA, nb, 1, 0, Bc));
  const int nbN = vec_blocks(N);
  LAUNCH(c, KID_VEC, k_comp_sum<double><<<dim3(nbN, d, Bc), 256, 0, c->stream>>>(c->u, N, c->partB, c->cs));
  TRY(reduce_to(c, c->partB, nbN, d, 8, Bc));
  LAUNCH(c, KID_VEC, k_sub_mean<double><<<dim3(nbN, d, Bc), 256, 0, c->stream>>>(c->u, N, c->small + 8, c->cs));
  const unsigned nbs = (unsigned)((N + 255) / 256);
  const int tri = c->elem == JFFT_ELEM_TRI ? 1 : 0;
  const long long sig_cs = (long long)sizeof(double) * ds * (tri ? 2 : (1 << d)) * N;
  LAUNCH(c, KID_STRESS, k_stress<double><<<dim3(nbs, Bc), 256, 0, c->stream>>>(c->u, c->E, c->macro, c->lam, c->mu, c->g.w, c->g.ihx, c->g.ihy, c->g.ihz, d, c->g.nx, c->g.ny, c->g.nz, N, sigma_dev, c->partB, c->cs, sig_cs, tri));
  TRY(reduce_to(c, c->partB, nbs, ds, 16, Bc));
  // u to the caller's [B][d][N] array
  if (u_out)  // internal callers read the fluctuations from the workspace
    LAUNCH(c, KID_VEC, k_copy<double><<<dim3(nb, Bc), 256, 0, c->stream>>>(c->u, c->cs, u_out, (long long)sizeof(double) * nd, nd));
  if (fetch) {
    TRY(fetch_small(c));
    read_sigma_bar(c, sigma_bar);
  }
  return JFFT_OK;
}

PcgBufs<double> bufs64(jfft_cell_s *c) {
  return {c->u, c->r, c->z, c->q, {c->p[0], c->p[1]}, c->E, c->Jh, c->spec};
}
PcgBufs<float> bufs32(jfft_cell_s *c) {
  return {c->c32, c->r32, c->z32, c->q32, {c->p32[0], c->p32[1]}, c->E32, c->Jh32, c->spec32};
}

// Mixed refinement, first half of a sweep: the FP64 residual r = f - K u
// (from_u; else u = 0 and r = f) and its stopping test (k_outer_check).
jfft_status sweep_residual(jfft_cell_s *c, int maxit, bool from_u) {
  const long long nd = (long long)c->dim * c->g.N;
  const int nb = vec_blocks(nd);
  if (from_u) {
    TRY(apply_K<double>(c, c->E, c->u, c->q, c->B));
    LAUNCH(c, KID_VEC, k_sub_norm<double><<<dim3(nb, c->B), 256, 0, c->stream>>>(c->f, c->q, c->r, nd, c->partA, c->cs));
  } else {
    LAUNCH(c, KID_VEC, k_sub_norm<double><<<dim3(nb, c->B), 256, 0, c->stream>>>(c->f, c->u, c->r, nd, c->partA, c->cs));
  }
  LAUNCH(c, KID_CTRL, k_outer_check<<<c->B, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, nb, c->max_outer, maxit, c->cs));
  return JFFT_OK;
}

// Second half: the FP32 inner solve for the correction c on r / ||r||
// (c = 0), started (pcg_begin), or continued (cont).
jfft_status sweep_start(jfft_cell_s *c, int maxit, bool cont) {
  const long long nd = (long long)c->dim * c->g.N;
  const int nb = vec_blocks(nd);
  LAUNCH(c, KID_VEC, (k_convert<double, float><<<dim3(nb, c->B), 256, 0, c->stream>>>(c->r, c->r32, nd, 1.0, c->st, c->cs)));
  LAUNCH(c, KID_VEC, k_fill<float><<<dim3(nb, c->B), 256, 0, c->stream>>>(c->c32, 0.0f, nd, c->cs));
  return pcg_begin<float>(c, bufs32(c), true, maxit, History{nullptr, nullptr, nullptr}, cont);
}

// After the inner solve stopped (its owed update of c applied): count it,
// u += ||r|| c.
jfft_status sweep_end(jfft_cell_s *c) {
  const long long nd = (long long)c->dim * c->g.N;
  LAUNCH(c, KID_CTRL, k_outer_update<<<c->B, 1, 0, c->stream>>>(c->st, c->cs));
  LAUNCH(c, KID_VEC, k_axpy_f32_to_f64<<<dim3(vec_blocks(nd), c->B), 256, 0, c->stream>>>(c->c32, c->u, nd, c->st, c->cs));
  return JFFT_OK;
}

// Mixed precision: FP64 residual r = f - K u and iterate u, FP32 inner PCG
// on r / ||r|| (FP64 dots and CG scalars), u += ||r|| c, until the FP64
// residual meets the cell's stopping rule (state set by k_solve_norms).
// have_u: u holds a start vector (else u = 0 and r = f).
jfft_status mixed_refine(jfft_cell_s *c, int maxit, bool have_u) {
  for (int sweep = 0;; ++sweep) {
    TRY(sweep_residual(c, maxit, sweep > 0 || have_u));
    TRY(fetch_states(c));
    bool all = true;
    for (int i = 0; i < c->B; ++i) all = all && c->st_h[i].outer_done;
    if (all) break;
    TRY(sweep_start(c, maxit, sweep > 0 && c->mixed_continue));
    TRY(pcg_loop<float>(c, bufs32(c), History{nullptr, nullptr, nullptr}));
    TRY(sweep_end(c));
  }
  return JFFT_OK;
}

// Right-hand side f = -B^T W C E_bar (|f| into q), the norms and the
// homogeneous test, and the start vector u (u0, else zero), for every cell.
jfft_status solve_setup(jfft_cell_s *c, const double *macros_h, double tol, const double *u0) {
  const long long nd = (long long)c->dim * c->g.N;
  const int Bc = c->B;
  TRY(assemble_rhs(c, macros_h, c->f, c->q, Bc));
  const int nb = vec_blocks(nd);
  LAUNCH(c, KID_VEC, k_dot<double><<<dim3(nb, Bc), 256, 0, c->stream>>>(c->f, c->f, nd, c->partA, c->cs));
  LAUNCH(c, KID_VEC, k_dot<double><<<dim3(nb, Bc), 256, 0, c->stream>>>(c->q, c->q, nd, c->partB, c->cs));
  LAUNCH(c, KID_CTRL, k_solve_norms<<<Bc, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, c->partB, nb, tol, c->stop_abs ? 1 : 0, c->cs));
  LAUNCH(c, KID_VEC, k_start_vector<<<dim3(nb, Bc), 256, 0, c->stream>>>(u0, (long long)sizeof(double) * nd, c->u, nd, c->st, c->cs));
  return JFFT_OK;
}

// FP64 solve: r = f - K u (or f) and the start of the PCG loop.
jfft_status fp64_start(jfft_cell_s *c, int maxit, bool have_u, History h) {
  const long long nd = (long long)c->dim * c->g.N;
  const int nb = vec_blocks(nd);
  if (have_u) {
    TRY(apply_K<double>(c, c->E, c->u, c->q, c->B));
    LAUNCH(c, KID_VEC, k_sub_norm<double><<<dim3(nb, c->B), 256, 0, c->stream>>>(c->f, c->q, c->r, nd, c->partA, c->cs));
  } else {
    LAUNCH(c, KID_VEC, k_copy<double><<<dim3(nb, c->B), 256, 0, c->stream>>>(c->f, c->cs, c->r, c->cs, nd));
  }
  return pcg_begin<double>(c, bufs64(c), false, maxit, h, false);
}

// Report of cell i from the fetched state and reduction results.
jfft_report make_report(const jfft_cell_s *c, int i) {
  const CgState &s = c->st_h[i];
  const double fn = std::sqrt(s.fnorm2);
  jfft_report R{};
  R.iters = s.total_iters;
  R.outer = s.outer;
  R.status = s.final_status;
  R.rel_res = (c->prec == JFFT_FP64) ? (fn > 0 && !s.homog ? std::sqrt(s.rr) / fn : 0.0)
                                     : (fn > 0 && !s.homog ? s.rn / fn : 0.0);
  R.rel_res_true = (fn > 0 && !s.homog) ? std::sqrt(c->small_h[(size_t)i * kSmall]) / fn : 0.0;
  return R;
}

jfft_status solve_impl(jfft_cell_s *c, const double *macros_h, double tol, int maxit,
                       const double *u0, double *u_out, double *sigma_dev, double *sigma_bar,
                       jfft_report *reps) {
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  if (!macros_h || !sigma_bar) return fail(JFFT_E_INVALID, "NULL macro_strain or sigma_bar");
  if (!(tol > 0.0) || maxit < 0) return fail(JFFT_E_INVALID, "tol must be > 0 and maxit >= 0");
  if (slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  const int Bc = c->B;
  for (auto &e : c->phase_ev)
    if (!e) HIP_TRY(hipEventCreate(&e));
  HIP_TRY(hipEventRecord(c->phase_ev[0], c->stream));
  TRY(solve_setup(c, macros_h, tol, u0));
  HIP_TRY(hipEventRecord(c->phase_ev[1], c->stream));
  if (c->prec == JFFT_FP64) {
    History h{nullptr, nullptr, nullptr};
    if (c->hist_cap > 0) h = {c->hist[0], c->hist[1], c->hist[2]};
    TRY(fp64_start(c, maxit, u0 != nullptr, h));
    TRY(pcg_loop<double>(c, bufs64(c), h));
    LAUNCH(c, KID_CTRL, k_fp64_final<<<Bc, 1, 0, c->stream>>>(c->st, c->cs));
  } else {
    TRY(mixed_refine(c, maxit, u0 != nullptr));
  }
  HIP_TRY(hipEventRecord(c->phase_ev[2], c->stream));
  TRY(post_process(c, u_out, sigma_dev, sigma_bar, false));
  HIP_TRY(hipEventRecord(c->phase_ev[3], c->stream));
  TRY(fetch_all(c));
  read_sigma_bar(c, sigma_bar);
  const double setup_ms = elapsed_ms(c->phase_ev[0], c->phase_ev[1]);
  const double loop_ms = elapsed_ms(c->phase_ev[1], c->phase_ev[2]);
  const double post_ms = elapsed_ms(c->phase_ev[2], c->phase_ev[3]);
  int worst = JFFT_OK;
  for (int i = 0; i < Bc; ++i) {
    jfft_report R = make_report(c, i);
    R.setup_ms = setup_ms;
    R.loop_ms = loop_ms;
    R.post_ms = post_ms;
    if (reps) reps[i] = R;
    if (R.status != JFFT_OK && worst == JFFT_OK) worst = R.status;
    if (R.status == JFFT_E_BREAKDOWN) worst = JFFT_E_BREAKDOWN;
  }
  if (worst == JFFT_E_NOT_CONVERGED) g_last_error = "PCG reached maxit";
  if (worst == JFFT_E_BREAKDOWN) g_last_error = "PCG breakdown (p.q <= 0 or non-finite scalar)";
  return (jfft_status)worst;
}

// ------------------------------------------ continuous batching over slots
// The cells of a group as slots that solves enter and leave between chunks
// of PCG iterations (serving: a request admitted while others run joins the
// next chunk).  Each cell has its own CG state, stopping flag and
// fixed-order reductions, and every chunk starts on the same
// search-direction buffer, so a cell computes the same iterates whatever
// the other slots hold and whenever it was admitted: a slot's result is
// bitwise that of the same cell solved alone with the same tile shapes.

enum { SLOT_FREE = 0, SLOT_RUNNING = 1, SLOT_FINISHED = 2 };

bool slots_busy(const jfft_cell_s *c) {
  if (c->in_view) return false;
  for (int s : c->slot_state)
    if (s != SLOT_FREE) return true;
  return false;
}

// The group's per-cell pointers moved to cell i, with B = 1, for the
// lifetime of the view: the set-up, sweep and post-processing code then runs
// on that slot alone.  The shared tables stay.
class CellView {
 public:
  CellView(jfft_cell_s *c, int i)
      : c_(c), off_((long long)i * c->cs), B_(c->B), st_h_(c->st_h), small_h_(c->small_h) {
    shift(off_);
    c->B = 1;
    c->st_h += i;
    c->small_h += (size_t)i * kSmall;
    c->in_view = true;
  }
  ~CellView() {
    shift(-off_);
    c_->B = B_;
    c_->st_h = st_h_;
    c_->small_h = small_h_;
    c_->in_view = false;
  }
  CellView(const CellView &) = delete;
  CellView &operator=(const CellView &) = delete;

 private:
  template <typename T>
  static void mv(T *&p, long long d) {
    if (p) p = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(p) + d);
  }
  void shift(long long d) {
    jfft_cell_s *c = c_;
    mv(c->E, d), mv(c->Jh, d), mv(c->diag, d), mv(c->f, d), mv(c->r, d), mv(c->z, d);
    mv(c->q, d), mv(c->p[0], d), mv(c->p[1], d), mv(c->u, d), mv(c->spec, d);
    mv(c->E32, d), mv(c->Jh32, d), mv(c->r32, d), mv(c->z32, d), mv(c->q32, d);
    mv(c->p32[0], d), mv(c->p32[1], d), mv(c->c32, d), mv(c->spec32, d);
    mv(c->F, d), mv(c->macro, d), mv(c->st, d), mv(c->partA, d), mv(c->partB, d);
    mv(c->small, d);
    for (auto &h : c->hist) mv(h, d);
  }
  jfft_cell_s *c_;
  long long off_;
  int B_;
  CgState *st_h_;
  double *small_h_;
};

jfft_status slots_init(jfft_cell_s *c) {
  if (!c->slot_state.empty()) return JFFT_OK;
  TRY(ensure_ready(c));
  LAUNCH(c, KID_CTRL, k_slot_park<<<c->B, 1, 0, c->stream>>>(c->st, c->cs));
  c->slot_state.assign(c->B, SLOT_FREE);
  c->slot_maxit.assign(c->B, 0);
  c->slot_sweep.assign(c->B, 0);
  c->slot_t0.assign(c->B, {});
  c->slot_ms.assign(c->B, 0.0);
  return JFFT_OK;
}

jfft_status slot_admit(jfft_cell_s *c, int slot, const double *E_dev, double lam, double mu,
                       const double *macro_h, double tol, int maxit) {
  if (c->nl) return fail(JFFT_E_INVALID, "slots take the linear material only");
  if (!macro_h) return fail(JFFT_E_INVALID, "NULL macro_strain");
  if (!(tol > 0.0) || maxit < 0) return fail(JFFT_E_INVALID, "tol must be > 0 and maxit >= 0");
  if (slot < 0 || slot >= c->B) return fail(JFFT_E_INVALID, "slot out of range");
  TRY(slots_init(c));
  if (c->slot_state[slot] != SLOT_FREE)
    return fail(JFFT_E_INVALID, "slot " + std::to_string(slot) + " is not free (harvest it first)");
  // captured iterations carry the Lame constants: one pair for all running slots
  if ((c->lam != lam || c->mu != mu) && slots_busy(c))
    return fail(JFFT_E_INVALID, "another slot runs with other elastic constants");
  {
    // no synchronisation: a bad E is reported by the slot's harvest, and a
    // cell that needs no iteration (homogeneous) starts stopped
    CellView v(c, slot);
    TRY(set_material_impl(c, E_dev, lam, mu, false, true));
    TRY(solve_setup(c, macro_h, tol, nullptr));
    LAUNCH(c, KID_CTRL, k_slot_validate<<<1, 1, 0, c->stream>>>(c->st, c->small, c->cs));
    if (c->prec == JFFT_FP64) {
      TRY(fp64_start(c, maxit, false, History{nullptr, nullptr, nullptr}));
    } else {
      TRY(sweep_residual(c, maxit, false));
      TRY(sweep_start(c, maxit, false));
    }
  }
  c->slot_state[slot] = SLOT_RUNNING;
  c->slot_maxit[slot] = maxit;
  c->slot_sweep[slot] = 0;
  c->slot_t0[slot] = std::chrono::steady_clock::now();
  return JFFT_OK;
}

jfft_status slots_step(jfft_cell_s *c, int iters, int *states) {
  if (iters < 1) return fail(JFFT_E_INVALID, "iterations must be >= 1");
  TRY(slots_init(c));
  int hi = 0;  // slots [0, hi) hold every running one
  for (int i = 0; i < c->B; ++i)
    if (c->slot_state[i] == SLOT_RUNNING) hi = i + 1;
  if (hi > 0) {
    // launch over a prefix of the group (a power of two of slots, or all):
    // empty slots past it cost no blocks; one captured graph per prefix
    int pb = 1;
    while (pb < hi) pb *= 2;
    const int B = c->B;
    c->B = std::min(pb, B);
    jfft_status st;
    if (c->prec == JFFT_FP64)
      st = pcg_iterations<double>(c, bufs64(c), iters, History{nullptr, nullptr, nullptr});
    else
      st = pcg_iterations<float>(c, bufs32(c), iters, History{nullptr, nullptr, nullptr});
    c->B = B;
    TRY(st);
    TRY(fetch_states(c));
    std::vector<int> ended;
    for (int i = 0; i < c->B; ++i) {
      if (c->slot_state[i] != SLOT_RUNNING || !c->st_h[i].done) continue;
      CellView v(c, i);
      if (c->prec == JFFT_FP64) {
        TRY(pcg_finish<double>(c, bufs64(c)));
        LAUNCH(c, KID_CTRL, k_fp64_final<<<1, 1, 0, c->stream>>>(c->st, c->cs));
        ended.push_back(i);
      } else if (c->st_h[0].outer_done) {
        ended.push_back(i);  // stopped at admission (homogeneous, or f already small)
      } else {
        TRY(pcg_finish<float>(c, bufs32(c)));
        TRY(sweep_end(c));
        TRY(sweep_residual(c, c->slot_maxit[i], true));
        ended.push_back(i);
      }
    }
    if (!ended.empty()) {
      if (c->prec == JFFT_MIXED) TRY(fetch_states(c));  // the sweeps' outer tests
      for (int i : ended) {
        if (c->prec == JFFT_MIXED && !c->st_h[i].outer_done) {
          CellView v(c, i);
          TRY(sweep_start(c, c->slot_maxit[i], c->mixed_continue));
          ++c->slot_sweep[i];
          continue;
        }
        c->slot_state[i] = SLOT_FINISHED;
        c->slot_ms[i] = std::chrono::duration<double, std::milli>(
                            std::chrono::steady_clock::now() - c->slot_t0[i]).count();
      }
    }
  }
  if (states)
    for (int i = 0; i < c->B; ++i) states[i] = c->slot_state[i];
  return JFFT_OK;
}

// Chunks of PCG iterations (the captured graph's depth, else 2) until a slot
// finishes, none runs, or max_ms of wall time have passed (checked after
// each chunk): a serving loop then wakes only when there is something to
// harvest, or to admit arrivals at that interval.
jfft_status slots_run(jfft_cell_s *c, double max_ms, int *states) {
  if (!(max_ms >= 0.0)) return fail(JFFT_E_INVALID, "max_ms must be >= 0");
  TRY(slots_init(c));
  const int chunk = c->tun.graph_iters > 0 ? c->tun.graph_iters : 2;
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    bool running = false;
    for (int s : c->slot_state) running = running || s == SLOT_RUNNING;
    if (!running) break;
    TRY(slots_step(c, chunk, nullptr));
    bool finished = false;
    for (int s : c->slot_state) finished = finished || s == SLOT_FINISHED;
    if (finished) break;
    if (std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() >= max_ms)
      break;
  }
  if (states)
    for (int i = 0; i < c->B; ++i) states[i] = c->slot_state[i];
  return JFFT_OK;
}

jfft_status slot_harvest(jfft_cell_s *c, int slot, double *u_out, double *sigma_dev,
                         double *sigma_bar, jfft_report *rep) {
  if (slot < 0 || slot >= c->B) return fail(JFFT_E_INVALID, "slot out of range");
  if (!sigma_bar) return fail(JFFT_E_INVALID, "NULL sigma_bar");
  if (c->slot_state.empty() || c->slot_state[slot] != SLOT_FINISHED)
    return fail(JFFT_E_INVALID, "slot " + std::to_string(slot) + " holds no finished solve");
  jfft_report R{};
  {
    CellView v(c, slot);
    TRY(post_process(c, u_out, sigma_dev, sigma_bar, false));
    TRY(fetch_all(c));
    read_sigma_bar(c, sigma_bar);
    R = make_report(c, 0);
    LAUNCH(c, KID_CTRL, k_slot_park<<<1, 1, 0, c->stream>>>(c->st, c->cs));
  }
  R.loop_ms = c->slot_ms[slot];
  if (rep) *rep = R;
  c->slot_state[slot] = SLOT_FREE;
  if (R.status == JFFT_E_INVALID) g_last_error = "E contains negative or non-finite entries";
  if (R.status == JFFT_E_NOT_CONVERGED) g_last_error = "PCG reached maxit";
  if (R.status == JFFT_E_BREAKDOWN) g_last_error = "PCG breakdown (p.q <= 0 or non-finite scalar)";
  return (jfft_status)R.status;
}

// ------------------------------------------------- power-law Newton solve
// The nonlinear example of Sec. 4 by Newton linearisation (Sec. 2.2, eq.
// lin_system): f(u) = -B^T W sigma(E + B u), K(u) = B^T W C(E + B u) B; each
// step solves K(u) du = f(u) with the library's PCG and preconditioners
// (Jacobi diagonal by Algorithm 2 on K(u), Green operator of the inclusion's
// isotropic moduli) and sets u += du.

jfft_status set_material_powerlaw_impl(jfft_cell_s *c, const double *phase_dev, double K,
                                       double sigma0, double eps0, double n, double K_incl,
                                       double mu_incl) {
  if (!phase_dev) return fail(JFFT_E_INVALID, "phase_dev is NULL");
  if (slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (c->dim != 3 || c->B != 1)
    return fail(JFFT_E_INVALID, "the power-law material needs a single 3D cell");
  const double prm[6] = {K, sigma0, eps0, n, K_incl, mu_incl};
  for (double v : prm)
    if (!std::isfinite(v)) return fail(JFFT_E_INVALID, "power-law parameters must be finite");
  if (!(K > 0.0 && sigma0 > 0.0 && eps0 > 0.0 && n >= 1.0 && K_incl > 0.0 && mu_incl > 0.0))
    return fail(JFFT_E_INVALID, "need K, sigma0, eps0, K_incl, mu_incl > 0 and n >= 1");
  TRY(ensure_ready(c));
  const long long N = c->g.N;
  if (!c->uk) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(double) * 3 * N);
    if (e != hipSuccess) return fail(JFFT_E_OOM, std::string("hipMalloc Newton iterate: ") + hipGetErrorString(e));
    c->uk = static_cast<double *>(p);
  }
  if (c->prec == JFFT_MIXED && !c->uk32) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(float) * 3 * N);
    if (e != hipSuccess) return fail(JFFT_E_OOM, std::string("hipMalloc Newton iterate: ") + hipGetErrorString(e));
    c->uk32 = static_cast<float *>(p);
  }
  c->drop_graphs();
  c->has_material = false;
  c->nl = false;
  const int nb = vec_blocks(N);
  LAUNCH(c, KID_SETUP, k_check_E<<<dim3(nb, 1), 256, 0, c->stream>>>(phase_dev, 0, N, c->partA, c->cs));
  TRY(reduce_to(c, c->partA, nb, 1, 0, 1));
  TRY(fetch_small(c));
  if (c->small_h[0] != 0.0) return fail(JFFT_E_INVALID, "phase contains negative or non-finite entries");
  LAUNCH(c, KID_SETUP, k_copy<double><<<dim3(nb, 1), 256, 0, c->stream>>>(phase_dev, 0, c->E, 0, N));
  if (c->prec == JFFT_MIXED)
    LAUNCH(c, KID_SETUP, (k_convert<double, float><<<dim3(nb, 1), 256, 0, c->stream>>>(c->E, c->E32, N, 1.0, nullptr, c->cs)));
  c->pl = PowerLawArgs{};
  c->pl.K = K;
  c->pl.gcoef = sigma0 * (2.0 / 3.0) / std::pow(eps0, n);
  c->pl.n = n;
  c->pl.ipow = (n == std::floor(n) && n - 1.0 <= 64.0) ? (int)(n - 1.0) : -1;
  c->pl.Ki = K_incl;
  c->pl.mui = mu_incl;
  c->lam = K_incl - 2.0 * mu_incl / 3.0;  // Green reference: the inclusion
  c->mu = mu_incl;
  c->nl = true;
  TRY(refresh_tz(c));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return JFFT_OK;
}

// Macroscopic strain into the kernel arguments; captured iterations carry
// it, so a new value drops them.
void set_macro_pl(jfft_cell_s *c, const double *macro_h) {
  bool same = true;
  for (int k = 0; k < 6; ++k) same = same && c->pl.macro[k] == macro_h[k];
  if (!same) {
    for (int k = 0; k < 6; ++k) c->pl.macro[k] = macro_h[k];
    c->drop_graphs();
  }
}

long long node_blocks(const jfft_cell_s *c) { return (c->g.N + 255) / 256; }

// f = f(uk) into `f`, ||f||^2 into small[0] (not fetched); with diag != NULL
// also diag(K(uk)) in closed form (the result of Algorithm 2).
jfft_status nl_force(jfft_cell_s *c, double *f, double *diag) {
  const GridDev &g = c->g;
  const long long nb = node_blocks(c);
  if (diag)
    LAUNCH(c, KID_RHS, (k_nl_force<double, true><<<(unsigned)nb, 256, 0, c->stream>>>(c->uk, c->E, f, diag, c->partA, c->pl, g.w, g.ihx, g.ihy, g.ihz, g.nx, g.ny, g.nz, g.N)));
  else
    LAUNCH(c, KID_RHS, (k_nl_force<double, false><<<(unsigned)nb, 256, 0, c->stream>>>(c->uk, c->E, f, nullptr, c->partA, c->pl, g.w, g.ihx, g.ihy, g.ihz, g.nx, g.ny, g.nz, g.N)));
  return reduce_to(c, c->partA, nb, 1, 0, 1);
}

// diag(K(uk)) is formed with the force (closed form) unless Algorithm 2's
// probing is selected.
bool nl_closed_diag(const jfft_cell_s *c) { return c->diag_method == JFFT_DIAG_CLOSED_FORM; }

// sum over Gauss points of sigma(E + B uk) / (8 N) into small[16..21] (not fetched).
jfft_status nl_stress_avg(jfft_cell_s *c) {
  const GridDev &g = c->g;
  const long long nb = node_blocks(c);
  LAUNCH(c, KID_STRESS, k_nl_stress_sum<double><<<(unsigned)nb, 256, 0, c->stream>>>(c->uk, c->E, c->partB, c->pl, g.ihx, g.ihy, g.ihz, g.nx, g.ny, g.nz, g.N));
  return reduce_to(c, c->partB, nb, 6, 16, 1);
}

// J^1/2 of the tangent at uk from c->diag (formed with the force in closed
// form, or here by Algorithm 2's probing); nothing without a Jacobi factor.
jfft_status nl_jacobi(jfft_cell_s *c) {
  if (!useJ(c)) return JFFT_OK;
  const long long nd = 3 * c->g.N;
  if (!nl_closed_diag(c)) TRY(run_alg2(c, c->diag, 1));
  if (c->prec == JFFT_MIXED)  // only the FP32 inner solves use J^1/2
    LAUNCH(c, KID_SETUP, k_jhalf<float><<<dim3(vec_blocks(nd), 1), 256, 0, c->stream>>>(c->diag, c->Jh32, nd, c->void_value, c->cs));
  else
    LAUNCH(c, KID_SETUP, k_jhalf<double><<<dim3(vec_blocks(nd), 1), 256, 0, c->stream>>>(c->diag, c->Jh, nd, c->void_value, c->cs));
  return JFFT_OK;
}

jfft_status newton_impl(jfft_cell_s *c, const double *macro_h, double newton_tol, double pcg_tol,
                        int max_newton, int maxit, double *u_out, double *sigma_bar,
                        int *pcg_iters, double *res_norms, int *steps_out) {
  if (!c->nl) return fail(JFFT_E_NO_MATERIAL, "set the power-law material first");
  if (!macro_h || !u_out || !sigma_bar) return fail(JFFT_E_INVALID, "NULL macro_strain, u_dev or sigma_bar");
  if (!(newton_tol > 0.0) || !(pcg_tol > 0.0) || (!c->stop_abs && !(pcg_tol < 1.0)) ||
      max_newton < 0 || maxit < 0)
    return fail(JFFT_E_INVALID, "need newton_tol > 0, pcg_tol > 0 (< 1 for the relative rule), "
                                "max_newton >= 0, maxit >= 0");
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(macro_h[k])) return fail(JFFT_E_INVALID, "macro_strain must be finite");
  set_macro_pl(c, macro_h);
  const long long N = c->g.N, nd = 3 * N;
  const int nb = vec_blocks(nd);
  LAUNCH(c, KID_VEC, k_fill<double><<<dim3(nb, 1), 256, 0, c->stream>>>(c->uk, 0.0, nd, 0));
  PcgBufs<double> b{c->u, c->r, c->z, c->q, {c->p[0], c->p[1]}, c->E, c->Jh, c->spec};
  int steps = 0;
  bool converged = false, broke = false;
  for (;;) {
    TRY(nl_force(c, c->f, useJ(c) && nl_closed_diag(c) ? c->diag : nullptr));
    TRY(fetch_small(c));
    const double fn = std::sqrt(c->small_h[0]);
    if (res_norms) res_norms[steps] = fn;
    if (!std::isfinite(fn)) return fail(JFFT_E_BREAKDOWN, "Newton residual is not finite");
    if (fn < newton_tol) {
      converged = true;
      break;
    }
    if (steps == max_newton) break;
    TRY(nl_jacobi(c));
    // relative rule: inexact Newton, no inner solve below a tenth of the
    // Newton tolerance; absolute rule: ||r||^2 <= pcg_tol as in Sec. 4
    const double itol = c->stop_abs ? pcg_tol : std::max(pcg_tol, 0.1 * newton_tol / fn);
    LAUNCH(c, KID_VEC, k_dot<double><<<dim3(nb, 1), 256, 0, c->stream>>>(c->f, c->f, nd, c->partA, c->cs));
    LAUNCH(c, KID_CTRL, k_solve_norms<<<1, CTRL_THREADS, 0, c->stream>>>(c->st, c->partA, c->partA, nb, itol, c->stop_abs ? 1 : 0, c->cs));
    LAUNCH(c, KID_VEC, k_fill<double><<<dim3(nb, 1), 256, 0, c->stream>>>(c->u, 0.0, nd, 0));
    if (c->prec == JFFT_MIXED) {
      // FP32 tangent solves refined against the FP64 tangent residual
      LAUNCH(c, KID_VEC, (k_convert<double, float><<<dim3(nb, 1), 256, 0, c->stream>>>(c->uk, c->uk32, nd, 1.0, nullptr, c->cs)));
      TRY(mixed_refine(c, maxit, false));
    } else {
      LAUNCH(c, KID_VEC, k_copy<double><<<dim3(nb, 1), 256, 0, c->stream>>>(c->f, 0, c->r, 0, nd));
      TRY(pcg_begin<double>(c, b, false, maxit, History{nullptr, nullptr, nullptr}, false));
      TRY(pcg_loop<double>(c, b, History{nullptr, nullptr, nullptr}));
      LAUNCH(c, KID_CTRL, k_fp64_final<<<1, 1, 0, c->stream>>>(c->st, c->cs));
    }
    LAUNCH(c, KID_VEC, k_add<double><<<nb, 256, 0, c->stream>>>(c->u, c->uk, nd));
    TRY(fetch_states(c));
    if (pcg_iters) pcg_iters[steps] = c->st_h[0].total_iters;
    if (c->st_h[0].final_status == JFFT_E_BREAKDOWN) broke = true;
    ++steps;
  }
  if (steps_out) *steps_out = steps;
  TRY(nl_stress_avg(c));
  // mean of u removed (Sec. 5), u to the caller
  const int nbN = vec_blocks(N);
  LAUNCH(c, KID_VEC, k_comp_sum<double><<<dim3(nbN, 3, 1), 256, 0, c->stream>>>(c->uk, N, c->partA, c->cs));
  TRY(reduce_to(c, c->partA, nbN, 3, 8, 1));
  LAUNCH(c, KID_VEC, k_sub_mean<double><<<dim3(nbN, 3, 1), 256, 0, c->stream>>>(c->uk, N, c->small + 8, c->cs));
  LAUNCH(c, KID_VEC, k_copy<double><<<dim3(nb, 1), 256, 0, c->stream>>>(c->uk, 0, u_out, 0, nd));
  TRY(fetch_small(c));
  for (int k = 0; k < 6; ++k) sigma_bar[k] = c->small_h[16 + k] / (8.0 * (double)N);
  if (!converged) {
    g_last_error = broke ? "Newton did not converge (a PCG solve broke down)"
                         : "Newton reached max_newton steps";
    return JFFT_E_NOT_CONVERGED;
  }
  return JFFT_OK;
}

// Operators of the Newton step at a caller's iterate (copied into uk).
jfft_status nl_operator_prep(jfft_cell_s *c, const double *macro_h, const double *uk_dev) {
  if (!c->nl) return fail(JFFT_E_NO_MATERIAL, "set the power-law material first");
  if (!macro_h || !uk_dev) return fail(JFFT_E_INVALID, "NULL argument");
  set_macro_pl(c, macro_h);
  const long long nd = 3 * c->g.N;
  LAUNCH(c, KID_VEC, k_copy<double><<<dim3(vec_blocks(nd), 1), 256, 0, c->stream>>>(uk_dev, 0, c->uk, 0, nd));
  return JFFT_OK;
}

// ------------------------------------------ phase-field topology optimisation
// The workload of eq. aim_fun / eq. lin_system_topopt: a group of three 2D
// triangle cells holds the unit load cases e_g on one density rho (E = rho,
// C = rho C0); f = sum_g ||sigma_bar_g - t_g||^2 + f_pf(rho), its gradient
// from the three solutions (mutual-energy identity) and the phase field, and
// a projected L-BFGS on [0, 1] driving it.

jfft_status topo_check(jfft_cell_s *c) {
  if (c->dim != 2 || c->B != 3 || c->elem != JFFT_ELEM_TRI)
    return fail(JFFT_E_INVALID, "topology optimisation needs a group of 3 2D triangle cells");
  if (slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  return JFFT_OK;
}

double dev_dot(jfft_cell_s *c, const double *a, const double *b, long long n, jfft_status *st) {
  const int nb = vec_blocks(n);
  k_dot<double><<<dim3(nb, 1), 256, 0, c->stream>>>(a, b, n, c->partA, c->cs);
  k_reduce_groups<<<1, CTRL_THREADS, 0, c->stream>>>(c->partA, nb, 1, c->small, c->cs);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(c->small_h, c->small, sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) *st = fail(JFFT_E_HIP, std::string("dot: ") + hipGetErrorString(e));
  return c->small_h[0];
}

double dev_absmax(jfft_cell_s *c, const double *x, long long n, jfft_status *st) {
  const int nb = vec_blocks(n);
  k_absmax<<<nb, 256, 0, c->stream>>>(x, n, c->partA);
  std::vector<double> h(nb);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), c->partA, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) *st = fail(JFFT_E_HIP, std::string("absmax: ") + hipGetErrorString(e));
  double m = 0.0;
  for (double v : h) m = std::max(m, v);
  return m;
}

// f = (f, f_sigma, f_pf), grad [N] (device), iters[3] of the three solves.
jfft_status topo_eval_impl(jfft_cell_s *c, const double *rho, double lam0, double mu0,
                           const double *t, double eta, double tol, int maxit, double *f,
                           double *grad, int *iters) {
  TRY(topo_check(c));
  if (!rho || !t || !f || !grad) return fail(JFFT_E_INVALID, "NULL argument");
  if (!(eta > 0.0)) return fail(JFFT_E_INVALID, "eta must be > 0");
  TRY(set_material_impl(c, rho, lam0, mu0, true));
  const double macros[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double sb[9];
  jfft_report reps[3];
  const jfft_status st = solve_impl(c, macros, tol, maxit, nullptr, nullptr, nullptr, sb, reps);
  if (st != JFFT_OK) return st;
  const GridDev &g = c->g;
  const long long N = g.N;
  TopoW W{};
  double fs = 0.0;
  for (int gm = 0; gm < 3; ++gm)
    for (int a = 0; a < 3; ++a) {
      const double d = sb[gm * 3 + a] - t[gm * 3 + a];
      fs += d * d;
      W.w[gm][a] = 2.0 * d / g.vol;
    }
  const unsigned nb = (unsigned)((N + 255) / 256);
  const double A = 2.0 * g.w, cell = 4.0 * g.w;  // triangle area, pixel area
  LAUNCH(c, KID_VEC, k_topo_sens_tri<<<nb, 256, 0, c->stream>>>(c->u, c->cs, W, lam0, mu0, A, g.ihx, g.ihy, g.nx, g.ny, N, grad));
  LAUNCH(c, KID_VEC, k_topo_pf_tri<<<nb, 256, 0, c->stream>>>(rho, eta, A, cell, g.ihx, g.ihy, g.nx, g.ny, N, grad, c->partB));
  TRY(reduce_to(c, c->partB, nb, 1, 0, 1));
  HIP_TRY(hipMemcpyAsync(c->small_h, c->small, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const double fpf = c->small_h[0];
  f[0] = fs + fpf;
  f[1] = fs;
  f[2] = fpf;
  if (iters)
    for (int i = 0; i < 3; ++i) iters[i] = reps[i].iters;
  return JFFT_OK;
}

jfft_status topo_lbfgs_impl(jfft_cell_s *c, double *x, double lam0, double mu0, const double *t,
                            double eta, double tol, int maxit, int n_iter, int m, double *f_hist,
                            double *gnorm_hist, int *iters_hist, int *steps_out, int *evals_out,
                            long long *pcg_total) {
  TRY(topo_check(c));
  if (!x || !t) return fail(JFFT_E_INVALID, "NULL argument");
  if (n_iter < 0 || m < 1 || m > 64) return fail(JFFT_E_INVALID, "need n_iter >= 0 and 1 <= m <= 64");
  const long long n = c->g.N;
  // vectors: g, gt, q (also z), d, xt, st, then m slots of s and of y
  const long long nvec = 6 + 2 * (long long)m;
  if (!c->topo || c->topo_m < m) {
    if (c->topo) {
      (void)hipStreamSynchronize(c->stream);
      (void)hipFree(c->topo);
      c->topo = nullptr;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(double) * n * nvec);
    if (e != hipSuccess) return fail(JFFT_E_OOM, std::string("hipMalloc L-BFGS vectors: ") + hipGetErrorString(e));
    c->topo = static_cast<double *>(p);
    c->topo_m = m;
  }
  double *g = c->topo, *gt = g + n, *q = gt + n, *d = q + n, *xt = d + n, *st = xt + n;
  double *S = st + n, *Y = S + (long long)m * n;
  const int nb = vec_blocks(n);
  jfft_status err = JFFT_OK;
  // x on the box
  LAUNCH(c, KID_VEC, k_topo_trial<<<nb, 256, 0, c->stream>>>(x, x, 0.0, xt, st, n));
  LAUNCH(c, KID_VEC, k_copy<double><<<dim3(nb, 1), 256, 0, c->stream>>>(xt, 0, x, 0, n));
  double fv[3];
  int its[3];
  TRY(topo_eval_impl(c, x, lam0, mu0, t, eta, tol, maxit, fv, g, its));
  int evals = 1, steps = 0;
  long long total = (long long)its[0] + its[1] + its[2];
  auto record = [&](int k, double fk, const double *gk, const int *ik) {
    if (f_hist) f_hist[k] = fk;
    if (gnorm_hist) gnorm_hist[k] = dev_absmax(c, gk, n, &err);
    if (iters_hist)
      for (int i = 0; i < 3; ++i) iters_hist[3 * k + i] = ik[i];
  };
  double f = fv[0];
  record(0, f, g, its);
  TRY(err);
  // pair history (oldest first): slot index, 1 / y.s, s.y, y.y
  std::vector<int> slot;
  std::vector<double> rinv, sy_h, yy_h;
  const double c1 = 1e-4;
  const int max_halvings = 30;
  for (int k = 0; k < n_iter; ++k) {
    LAUNCH(c, KID_VEC, k_topo_free<<<nb, 256, 0, c->stream>>>(x, g, q, n));
    const int np = (int)slot.size();
    std::vector<double> al(np);
    for (int i = np - 1; i >= 0; --i) {
      const double *si = S + (long long)slot[i] * n, *yi = Y + (long long)slot[i] * n;
      al[i] = rinv[i] * dev_dot(c, si, q, n, &err);
      LAUNCH(c, KID_VEC, k_axpby<<<nb, 256, 0, c->stream>>>(-al[i], yi, 1.0, q, n));
    }
    TRY(err);
    double h0;
    if (np)
      h0 = sy_h[np - 1] / yy_h[np - 1];
    else
      h0 = 0.1 / std::max(dev_absmax(c, q, n, &err), 1e-300);
    TRY(err);
    LAUNCH(c, KID_VEC, k_axpby<<<nb, 256, 0, c->stream>>>(0.0, q, h0, q, n));  // z = h0 q (in q)
    for (int i = 0; i < np; ++i) {
      const double *si = S + (long long)slot[i] * n, *yi = Y + (long long)slot[i] * n;
      const double b = rinv[i] * dev_dot(c, yi, q, n, &err);
      LAUNCH(c, KID_VEC, k_axpby<<<nb, 256, 0, c->stream>>>(al[i] - b, si, 1.0, q, n));
    }
    TRY(err);
    LAUNCH(c, KID_VEC, k_topo_dir<<<nb, 256, 0, c->stream>>>(x, g, q, d, n));
    double alpha = 1.0, ft = 0.0, gs = 0.0;
    bool accepted = false;
    for (int h = 0; h < max_halvings; ++h) {
      LAUNCH(c, KID_VEC, k_topo_trial<<<nb, 256, 0, c->stream>>>(x, d, alpha, xt, st, n));
      gs = dev_dot(c, g, st, n, &err);
      TRY(err);
      if (gs < 0.0) {
        TRY(topo_eval_impl(c, xt, lam0, mu0, t, eta, tol, maxit, fv, gt, its));
        ++evals;
        total += (long long)its[0] + its[1] + its[2];
        ft = fv[0];
        if (ft <= f + c1 * gs) {
          accepted = true;
          break;
        }
      }
      alpha *= 0.5;
    }
    if (!accepted) break;
    // candidate pair s = st, y = gt - g (y formed in q, free once d exists);
    // kept in the next free slot, or in place of the oldest pair
    LAUNCH(c, KID_VEC, k_sub<<<nb, 256, 0, c->stream>>>(gt, g, q, n));
    const double sy = dev_dot(c, st, q, n, &err);
    const double ss = dev_dot(c, st, st, n, &err);
    const double yy = dev_dot(c, q, q, n, &err);
    TRY(err);
    if (sy > 1e-12 * std::sqrt(ss) * std::sqrt(yy)) {
      const int cand = np < m ? np : slot[0];
      double *sc = S + (long long)cand * n, *yc = Y + (long long)cand * n;
      LAUNCH(c, KID_VEC, k_copy<double><<<dim3(nb, 1), 256, 0, c->stream>>>(st, 0, sc, 0, n));
      LAUNCH(c, KID_VEC, k_copy<double><<<dim3(nb, 1), 256, 0, c->stream>>>(q, 0, yc, 0, n));
      if (np == m) {
        slot.erase(slot.begin());
        rinv.erase(rinv.begin());
        sy_h.erase(sy_h.begin());
        yy_h.erase(yy_h.begin());
      }
      slot.push_back(cand);
      rinv.push_back(1.0 / sy);
      sy_h.push_back(sy);
      yy_h.push_back(yy);
    }
    LAUNCH(c, KID_VEC, k_copy<double><<<dim3(nb, 1), 256, 0, c->stream>>>(xt, 0, x, 0, n));
    std::swap(g, gt);
    f = ft;
    ++steps;
    record(steps, f, g, its);
    TRY(err);
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (steps_out) *steps_out = steps;
  if (evals_out) *evals_out = evals;
  if (pcg_total) *pcg_total = total;
  return JFFT_OK;
}

bool supported_length(int n) {
  if (n < 2 || n > 512 || n % 2) return false;
  FftPlan p;
  return factor_plan(n, p) && factor_plan(n / 2, p);
}

jfft_status create_impl(int dim, const int n[3], const double len[3], jfft_precision prec,
                        jfft_precond pc, int batch, void *hip_stream, jfft_cell_t *out) {
  if (!out || !n) return fail(JFFT_E_INVALID, "NULL argument");
  *out = nullptr;
  if (dim != 2 && dim != 3) return fail(JFFT_E_INVALID, "dim must be 2 or 3");
  if (prec != JFFT_FP64 && prec != JFFT_MIXED) return fail(JFFT_E_INVALID, "unknown precision");
  if (pc < JFFT_PC_NONE || pc > JFFT_PC_GREEN_JACOBI) return fail(JFFT_E_INVALID, "unknown preconditioner");
  if (batch < 1 || batch > 65535) return fail(JFFT_E_INVALID, "batch must lie in [1, 65535]");
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
  c->B = batch;
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
  c->npart = max_partials(c);
  hipError_t e = set_smem_attributes();
  if (e == hipSuccess) e = hipGetDevice(&c->device);
  if (e == hipSuccess && dim == 3) {
    const int tz = auto_tz(c, &e);
    if (e == hipSuccess) {
      c->tun.tz = tz;
      if ((long long)((g.nz + c->tun.tz - 1) / c->tun.tz) * batch > 65535) {
        delete c;
        return fail(JFFT_E_INVALID, "batch too large for this grid (stiffness grid z-dimension above 65535)");
      }
    }
  }
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&c->st_h), sizeof(CgState) * batch, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&c->small_h), sizeof(double) * kSmall * batch, hipHostMallocDefault);
  // the solve's phase events, created here so that a solve creates none
  for (auto &pe : c->phase_ev)
    if (e == hipSuccess) e = hipEventCreate(&pe);
  if (e != hipSuccess) {
    delete c;
    return fail(JFFT_E_HIP, std::string("create: ") + hipGetErrorString(e));
  }
  *out = c;
  return JFFT_OK;
}

// Static workspace of jfft_solve_static: one per GPU, held until the process
// ends.  In host code `scratch` only names the symbol; its device address
// (a different one on every GPU) comes from hipGetSymbolAddress, taken once
// per device with that device current and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

jfft_status scratch_address(int device, unsigned char **out) {
  if (device < 0 || device >= kMaxDevices) return fail(JFFT_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) HIP_TRY(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      return fail(JFFT_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<unsigned char *>(p);
  }
  *out = g_scratch_ptr[device];
  return JFFT_OK;
}

}  // namespace

// ============================================================== C ABI ====
extern "C" {

jfft_status jfft_create_cell(int dim, const int n[3], const double len[3], jfft_precision prec,
                             jfft_precond pc, void *hip_stream, jfft_cell_t *out) {
  return create_impl(dim, n, len, prec, pc, 1, hip_stream, out);
}

jfft_status jfft_create_batch(int dim, const int n[3], const double len[3], jfft_precision prec,
                              jfft_precond pc, int batch, void *hip_stream, jfft_cell_t *out) {
  return create_impl(dim, n, len, prec, pc, batch, hip_stream, out);
}

jfft_status jfft_batch_size(jfft_cell_t c, int *batch) {
  if (!c || !batch) return fail(JFFT_E_INVALID, "NULL argument");
  *batch = c->B;
  return JFFT_OK;
}

jfft_status jfft_workspace_bytes(jfft_cell_t c, size_t *bytes) {
  if (!c || !bytes) return fail(JFFT_E_INVALID, "NULL argument");
  *bytes = layout_workspace(c, nullptr);
  return JFFT_OK;
}

jfft_status jfft_bind_workspace(jfft_cell_t c, void *dev_ptr, size_t bytes) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
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
  if (c->B != 1) return fail(JFFT_E_INVALID, "batched handle: use jfft_solve_batch");
  if (!u_dev) return fail(JFFT_E_INVALID, "NULL u_dev");
  return solve_impl(c, macro_strain, tol, maxit, u0_dev, u_dev, sigma_dev, sigma_bar, report);
}

jfft_status jfft_solve_static(jfft_cell_t c, const double *E_dev, double nu,
                              const double *macro_strain, double tol, int maxit,
                              const double *u0_dev, double *u_dev, double *sigma_dev,
                              double *sigma_bar, jfft_report *report) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  if (c->B != 1) return fail(JFFT_E_INVALID, "batched handle: the static workspace serves single cells");
  if (!E_dev || !u_dev) return fail(JFFT_E_INVALID, "NULL E_dev or u_dev");
  if (!(nu > -1.0 && nu < 0.5)) return fail(JFFT_E_INVALID, "nu must lie in (-1, 0.5)");
  if (c->ws_owned) return fail(JFFT_E_INVALID, "the cell owns a library-allocated workspace; use a fresh cell");
  if (c->timing) return fail(JFFT_E_INVALID, "kernel timing creates events; switch it off for jfft_solve_static");
  const size_t need = layout_workspace(c, nullptr);
  if (need > kScratchBytes)
    return fail(JFFT_E_INVALID, "the cell needs " + std::to_string(need) +
                                    " bytes of workspace; the static workspace holds " +
                                    std::to_string(kScratchBytes));
  unsigned char *ws = nullptr;
  TRY(scratch_address(c->device, &ws));
  // another cell may have used the array since this one did: lay the
  // workspace out again and upload the tables (no allocation, ws is set)
  c->ws = ws;
  c->ws_bytes = kScratchBytes;
  c->ws_owned = false;
  c->ready = false;
  c->has_material = false;
  TRY(ensure_ready(c));
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  TRY(set_material_impl(c, E_dev, lam, mu));
  // direct launches: instantiating a graph may allocate
  const int graph_iters = c->tun.graph_iters;
  c->tun.graph_iters = 0;
  const jfft_status st = solve_impl(c, macro_strain, tol, maxit, u0_dev, u_dev, sigma_dev, sigma_bar, report);
  c->tun.graph_iters = graph_iters;
  return st;
}

jfft_status jfft_solve_batch(jfft_cell_t c, const double *macro_strains, double tol, int maxit,
                             const double *u0_dev, double *u_dev, double *sigma_dev,
                             double *sigma_bars, jfft_report *reports) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  if (!u_dev) return fail(JFFT_E_INVALID, "NULL u_dev");
  return solve_impl(c, macro_strains, tol, maxit, u0_dev, u_dev, sigma_dev, sigma_bars, reports);
}

jfft_status jfft_slot_admit(jfft_cell_t c, int slot, const double *E_dev, double nu,
                            const double *macro_strain, double tol, int maxit) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  if (!(nu > -1.0 && nu < 0.5)) return fail(JFFT_E_INVALID, "nu must lie in (-1, 0.5)");
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = 1.0 / (2.0 * (1.0 + nu));
  return slot_admit(c, slot, E_dev, lam, mu, macro_strain, tol, maxit);
}

jfft_status jfft_slots_step(jfft_cell_t c, int iterations, int *states) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  return slots_step(c, iterations, states);
}

jfft_status jfft_slots_run(jfft_cell_t c, double max_ms, int *states) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  return slots_run(c, max_ms, states);
}

jfft_status jfft_slot_harvest(jfft_cell_t c, int slot, double *u_dev, double *sigma_dev,
                              double *sigma_bar, jfft_report *report) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  return slot_harvest(c, slot, u_dev, sigma_dev, sigma_bar, report);
}

jfft_status jfft_apply_stiffness(jfft_cell_t c, const double *in_dev, double *out_dev) {
  if (!c || !in_dev || !out_dev) return fail(JFFT_E_INVALID, "NULL argument");
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  if (c->B != 1) return fail(JFFT_E_INVALID, "operator entry points take a single-cell handle");
  if (slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  return apply_K<double>(c, c->E, in_dev, out_dev, 1);
}

jfft_status jfft_apply_precond(jfft_cell_t c, const double *in_dev, double *out_dev) {
  if (!c || !in_dev || !out_dev) return fail(JFFT_E_INVALID, "NULL argument");
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  if (c->B != 1) return fail(JFFT_E_INVALID, "operator entry points take a single-cell handle");
  if (slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  const long long nd = (long long)c->dim * c->g.N;
  LAUNCH(c, KID_VEC, k_copy<double><<<dim3(vec_blocks(nd), 1), 256, 0, c->stream>>>(in_dev, 0, c->r, 0, nd));
  long long nA, nB;
  History h{nullptr, nullptr, nullptr};
  TRY(precond<double>(c, c->r, nullptr, c->Jh, c->z, c->spec, false, false, &nA, &nB, h));
  LAUNCH(c, KID_VEC, k_copy<double><<<dim3(vec_blocks(nd), 1), 256, 0, c->stream>>>(c->z, 0, out_dev, 0, nd));
  return JFFT_OK;
}

jfft_status jfft_apply_precond_fp32(jfft_cell_t c, const double *in_dev, double *out_dev) {
  if (!c || !in_dev || !out_dev) return fail(JFFT_E_INVALID, "NULL argument");
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  if (c->B != 1) return fail(JFFT_E_INVALID, "operator entry points take a single-cell handle");
  if (slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (c->prec != JFFT_MIXED) return fail(JFFT_E_INVALID, "the FP32 preconditioner belongs to a mixed-precision cell");
  const long long nd = (long long)c->dim * c->g.N;
  LAUNCH(c, KID_VEC, (k_convert<double, float><<<dim3(vec_blocks(nd), 1), 256, 0, c->stream>>>(in_dev, c->r32, nd, 1.0, nullptr, 0)));
  long long nA, nB;
  History h{nullptr, nullptr, nullptr};
  TRY(precond<float>(c, c->r32, nullptr, c->Jh32, c->z32, c->spec32, false, false, &nA, &nB, h));
  LAUNCH(c, KID_VEC, (k_convert<float, double><<<dim3(vec_blocks(nd), 1), 256, 0, c->stream>>>(c->z32, out_dev, nd, 1.0, nullptr, 0)));
  return JFFT_OK;
}

jfft_status jfft_assemble_rhs(jfft_cell_t c, const double *macro_strain, double *f_dev) {
  if (!c || !macro_strain || !f_dev) return fail(JFFT_E_INVALID, "NULL argument");
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  if (c->B != 1) return fail(JFFT_E_INVALID, "operator entry points take a single-cell handle");
  if (slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  TRY(assemble_rhs(c, macro_strain, f_dev, nullptr, 1));
  HIP_TRY(hipStreamSynchronize(c->stream));  // macro_strain is a host pointer
  return JFFT_OK;
}

jfft_status jfft_jacobi_diag(jfft_cell_t c, double *diag_dev) {
  if (!c || !diag_dev) return fail(JFFT_E_INVALID, "NULL argument");
  if (!c->has_material) return fail(JFFT_E_NO_MATERIAL, "set the material first");
  if (c->B != 1) return fail(JFFT_E_INVALID, "operator entry points take a single-cell handle");
  if (slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  return run_alg2(c, diag_dev, 1);
}

jfft_status jfft_enable_history(jfft_cell_t c, int cap) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!c || cap < 0 || cap > kHistMax) return fail(JFFT_E_INVALID, "history capacity must lie in [0, 4096]");
  c->hist_cap = cap;
  c->drop_graphs();
  return JFFT_OK;
}

jfft_status jfft_get_batch_history(jfft_cell_t c, int index, double *alpha, double *beta,
                                   double *res, int cap, int *count) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  if (index < 0 || index >= c->B) return fail(JFFT_E_INVALID, "cell index out of range");
  if (count) *count = 0;
  if (!c->ready) return JFFT_OK;  // nothing solved yet
  TRY(fetch_states(c));
  // the device-side capacity is 0 when the last loop did not record (mixed inner solves)
  const int k = std::min(std::min(cap, c->st_h[index].hist_cap), c->st_h[index].iter);
  if (count) *count = k;
  if (k <= 0) return JFFT_OK;
  double *const dst[3] = {alpha, beta, res};
  for (int t = 0; t < 3; ++t)
    if (dst[t])
      HIP_TRY(hipMemcpy(dst[t], reinterpret_cast<unsigned char *>(c->hist[t]) + (size_t)index * c->cs,
                        sizeof(double) * k, hipMemcpyDeviceToHost));
  return JFFT_OK;
}

jfft_status jfft_get_history(jfft_cell_t c, double *alpha, double *beta, double *res, int cap,
                             int *count) {
  return jfft_get_batch_history(c, 0, alpha, beta, res, cap, count);
}

jfft_status jfft_set_graph_iterations(jfft_cell_t c, int iterations) {
  if (!c || iterations < 0 || iterations > 64 || (iterations % 2))
    return fail(JFFT_E_INVALID, "graph iterations must be an even number in [0, 64]");
  if (iterations > 0 && c->stream == nullptr)
    return fail(JFFT_E_INVALID, "graph replay needs a stream other than the legacy default stream");
  c->tun.graph_iters = iterations;
  c->drop_graphs();
  return JFFT_OK;
}

jfft_status jfft_set_tunables(jfft_cell_t c, const jfft_tunables *t) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!c || !t) return fail(JFFT_E_INVALID, "NULL argument");
  if (t->ygrid < 1 || t->ygrid > 65535) return fail(JFFT_E_INVALID, "ygrid must lie in [1, 65535]");
  // tz: 0 restores the automatic choice; a value other than the one in
  // effect fixes it
  const bool tz_set = c->dim == 3 && t->tz != 0 && t->tz != std::min(c->tun.tz, c->g.nz);
  if (tz_set) {
    if (t->tz < std::min(2, c->g.nz) || t->tz > c->g.nz)
      return fail(JFFT_E_INVALID, "tz must be 0 or lie in [2, nz]");
    const long long nbz = (c->g.nz + t->tz - 1) / t->tz;
    const long long tiles = stencil_tiles_max(3, c->g.nx, c->g.ny);
    if (nbz * c->B > 65535) return fail(JFFT_E_INVALID, "tz too small for this group (grid z-dimension)");
    if (tiles * nbz > c->npart) return fail(JFFT_E_INVALID, "tz too small for the partial-sum buffer");
  }
  if (t->tiles2d < 0 || t->tiles2d > 4) return fail(JFFT_E_INVALID, "tiles2d must lie in [0, 4]");
  if (t->tiles3d < 0 || t->tiles3d > 2) return fail(JFFT_E_INVALID, "tiles3d must lie in [0, 2]");
  if (t->xrows < 0 || (t->xrows & (t->xrows - 1)) != 0)
    return fail(JFFT_E_INVALID, "xrows must be 0 or a power of two");
  if (tz_set) {
    c->tun.tz = t->tz;
    c->tun.tz_auto = false;
  } else if (c->dim == 3 && t->tz == 0) {
    c->tun.tz_auto = true;
  }
  c->tun.ygrid = t->ygrid;
  c->tun.tiles2d = c->dim == 2 ? t->tiles2d : 0;
  // tiles3d: like tz, the value in effect (as reported) keeps the automatic
  // choice (which follows the material kind); another one fixes it, 0 restores it
  if (c->dim == 3 && t->tiles3d != tiles3d_of(c, c->prec == JFFT_FP64)) c->tun.tiles3d = t->tiles3d;
  c->tun.xrows = t->xrows;
  c->tun.fused_control = t->fused_control ? 1 : 0;
  c->drop_graphs();
  return c->dim == 3 && t->tz == 0 ? refresh_tz(c) : JFFT_OK;
}

jfft_status jfft_get_tunables(jfft_cell_t c, jfft_tunables *t) {
  if (!c || !t) return fail(JFFT_E_INVALID, "NULL argument");
  t->tz = c->dim == 3 ? std::min(c->tun.tz, c->g.nz) : 1;
  t->ygrid = c->tun.ygrid;
  t->tiles2d = c->dim == 2 ? tiles2d_of(c, c->prec == JFFT_FP64) : 0;
  t->tiles3d = c->dim == 3 ? tiles3d_of(c, c->prec == JFFT_FP64) : 0;
  const int rb = c->prec == JFFT_FP64 ? x_rows_per_block<double>(c->g.nx / 2)
                                      : x_rows_per_block<float>(c->g.nx / 2);
  t->xrows = c->tun.xrows && c->tun.xrows < rb ? c->tun.xrows : rb;
  t->fused_control = c->tun.fused_control;
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

jfft_status jfft_set_stop_rule(jfft_cell_t c, int rule) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!c || (rule != JFFT_STOP_RELATIVE && rule != JFFT_STOP_ABSOLUTE))
    return fail(JFFT_E_INVALID, "unknown stopping rule");
  c->stop_abs = rule == JFFT_STOP_ABSOLUTE;
  return JFFT_OK;
}

jfft_status jfft_set_diag_method(jfft_cell_t c, int method) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!c || (method != JFFT_DIAG_CLOSED_FORM && method != JFFT_DIAG_PROBING))
    return fail(JFFT_E_INVALID, "unknown diagonal method");
  if (c->diag_method != method) c->has_material = false;  // J^1/2 must be formed again
  c->diag_method = method;
  return JFFT_OK;
}

jfft_status jfft_set_element(jfft_cell_t c, int element) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!c || (element != JFFT_ELEM_QUAD && element != JFFT_ELEM_TRI))
    return fail(JFFT_E_INVALID, "unknown element");
  if (element == JFFT_ELEM_TRI && c->dim != 2)
    return fail(JFFT_E_INVALID, "linear triangles are a 2D element");
  if (c->elem != element) {
    c->has_material = false;  // K, f, diag(K) and G^ change
    c->drop_graphs();
  }
  c->elem = element;
  return JFFT_OK;
}

jfft_status jfft_set_void_value(jfft_cell_t c, double value) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!c || !(value > 0.0) || !std::isfinite(value)) return fail(JFFT_E_INVALID, "void value must be positive");
  c->void_value = value;
  return JFFT_OK;
}

jfft_status jfft_set_mixed_inner_cap(jfft_cell_t c, int cap) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!c || cap < 0) return fail(JFFT_E_INVALID, "the inner iteration cap must be >= 0");
  c->inner_cap = cap;
  return JFFT_OK;
}

jfft_status jfft_set_mixed_continue(jfft_cell_t c, int on, double reduction) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!c || (on != 0 && on != 1) || !(reduction > 0.0 && reduction < 1.0))
    return fail(JFFT_E_INVALID, "on must be 0 or 1 and reduction in (0, 1)");
  c->mixed_continue = on == 1;
  c->update_tol = reduction;
  return JFFT_OK;
}

jfft_status jfft_set_mixed_params(jfft_cell_t c, double inner_tol, int max_outer) {
  if (c && slots_busy(c)) return fail(JFFT_E_INVALID, kSlotsBusy);
  if (!c || !(inner_tol > 0.0 && inner_tol < 1.0) || max_outer < 1)
    return fail(JFFT_E_INVALID, "inner_tol must lie in (0, 1) and max_outer >= 1");
  c->inner_tol = inner_tol;
  c->max_outer = max_outer;
  return JFFT_OK;
}

jfft_status jfft_set_material_powerlaw(jfft_cell_t c, const double *phase_dev, double K,
                                       double sigma0, double eps0, double n, double K_incl,
                                       double mu_incl) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  return set_material_powerlaw_impl(c, phase_dev, K, sigma0, eps0, n, K_incl, mu_incl);
}

jfft_status jfft_solve_newton(jfft_cell_t c, const double *macro_strain, double newton_tol,
                              double pcg_tol, int max_newton, int maxit, double *u_dev,
                              double *sigma_bar, int *pcg_iters, double *res_norms, int *steps) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  return newton_impl(c, macro_strain, newton_tol, pcg_tol, max_newton, maxit, u_dev, sigma_bar,
                     pcg_iters, res_norms, steps);
}

jfft_status jfft_powerlaw_force(jfft_cell_t c, const double *macro_strain, const double *uk_dev,
                                double *f_dev) {
  if (!c || !f_dev) return fail(JFFT_E_INVALID, "NULL argument");
  TRY(nl_operator_prep(c, macro_strain, uk_dev));
  TRY(nl_force(c, f_dev, nullptr));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return JFFT_OK;
}

jfft_status jfft_powerlaw_tangent(jfft_cell_t c, const double *macro_strain, const double *uk_dev,
                                  const double *in_dev, double *out_dev) {
  if (!c || !in_dev || !out_dev) return fail(JFFT_E_INVALID, "NULL argument");
  TRY(nl_operator_prep(c, macro_strain, uk_dev));
  TRY(apply_K<double>(c, c->E, in_dev, out_dev, 1));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return JFFT_OK;
}

jfft_status jfft_powerlaw_jacobi_diag(jfft_cell_t c, const double *macro_strain,
                                      const double *uk_dev, double *diag_dev) {
  if (!c || !diag_dev) return fail(JFFT_E_INVALID, "NULL argument");
  TRY(nl_operator_prep(c, macro_strain, uk_dev));
  if (nl_closed_diag(c))
    TRY(nl_force(c, c->f, diag_dev));
  else
    TRY(run_alg2(c, diag_dev, 1));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return JFFT_OK;
}

jfft_status jfft_topopt_eval(jfft_cell_t c, const double *rho_dev, double lambda0, double mu0,
                             const double *targets, double eta, double tol, int maxit,
                             double *f_out, double *grad_dev, int *iters) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  return topo_eval_impl(c, rho_dev, lambda0, mu0, targets, eta, tol, maxit, f_out, grad_dev, iters);
}

jfft_status jfft_topopt_lbfgs(jfft_cell_t c, double *rho_dev, double lambda0, double mu0,
                              const double *targets, double eta, double tol, int maxit,
                              int n_iter, int m, double *f_hist, double *gnorm_hist,
                              int *iters_hist, int *steps, int *evals, long long *pcg_total) {
  if (!c) return fail(JFFT_E_INVALID, "NULL cell");
  return topo_lbfgs_impl(c, rho_dev, lambda0, mu0, targets, eta, tol, maxit, n_iter, m, f_hist,
                         gnorm_hist, iters_hist, steps, evals, pcg_total);
}

void jfft_destroy_cell(jfft_cell_t c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char *jfft_last_error(void) { return g_last_error.c_str(); }

const char *jfft_version(void) { return "jfft-mi355x 0.2 (gfx950)"; }

}  // extern "C"
