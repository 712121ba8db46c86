/*
 * jfft.h -- C ABI of the MI355X (gfx950) J-FFT solver: preconditioned
 * conjugate gradients for the periodic small-strain linear-elastic cell
 * problem on a regular grid, with the Green-Jacobi preconditioner
 *     M^-1 = J^1/2 F^-1 G^ F J^1/2
 * of Ladecky et al., "Jacobi-accelerated FFT-based solver for smooth
 * high-contrast data" (arXiv:2508.02613), Sec. 3.3, eq. prec_lin_systemJG_2.
 *
 * Discretisation (Sec. 2.1, eq. disc_wf / lin_system_exp): bilinear quads
 * (2D, plane strain) or trilinear hexes (3D) with 2^d Gauss points, nodal
 * unknowns u in R^{d N}, stiffness K = B^T W C(E) B with C_e = E_e C^,
 * C^ isotropic.  Pixel-wise constant material: E_e is the value of the element
 * whose lowest-index corner is node e (Sec. 4, material data sampling).
 *
 * Conventions shared by every entry point:
 *   - Grid: n[0] x n[1] (x n[2]) nodes, x fastest; periodic; lengths len[a]
 *     (NULL = unit cell); every n[a] must be even (Algorithm 2 needs it) and
 *     a product of 2, 3, 5 (FFT radices), 2 <= n[a] <= 512.
 *   - Device arrays are raw device pointers on the cell's device, allocated
 *     and owned by the caller.  Scalar fields E have N = prod n[a] doubles;
 *     vector fields have d*N doubles, component-major ([a][node]).
 *   - Mandel notation, order (11,22,33,23,13,12) in 3D and (11,22,12) in 2D,
 *     shear entries carry sqrt(2).
 *   - All device work is stream-ordered on the stream given at creation; the
 *     entry points that return host values synchronise that stream.
 *   - No entry point throws; each returns a jfft_status.  jfft_last_error()
 *     returns a thread-local message describing the last failure.
 *   - A cell is not thread-safe.  Distinct cells may be used from distinct
 *     threads on distinct streams.
 */
#ifndef JFFT_H
#define JFFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jfft_cell_s *jfft_cell_t;

typedef enum {
  JFFT_OK = 0,
  JFFT_E_INVALID = 1,       /* bad argument (dim, sizes, tol, NaN/negative E, nu) */
  JFFT_E_ODD_GRID = 2,      /* Algorithm 2 (Sec. 3.2) needs an even node count per axis */
  JFFT_E_NO_MATERIAL = 3,   /* jfft_set_material not called yet */
  JFFT_E_NOT_CONVERGED = 4, /* maxit reached; the last iterate is still written */
  JFFT_E_BREAKDOWN = 5,     /* p^T q <= 0 or a non-finite CG scalar */
  JFFT_E_OOM = 6,           /* workspace too small or allocation failure */
  JFFT_E_HIP = 7            /* a HIP runtime call failed */
} jfft_status;

typedef enum {
  JFFT_PC_NONE = 0,         /* M^-1 = I */
  JFFT_PC_GREEN = 1,        /* M^-1 = F^-1 G^ F (eq. prec_lin_systemG_FFT) */
  JFFT_PC_JACOBI = 2,       /* M^-1 = diag(K)^-1 (eq. prec_lin_systemJ) */
  JFFT_PC_GREEN_JACOBI = 3  /* M^-1 = J^1/2 F^-1 G^ F J^1/2 (eq. prec_lin_systemJG_2) */
} jfft_precond;

typedef enum {
  JFFT_FP64 = 0,  /* every step in double precision */
  JFFT_MIXED = 1  /* FP32 stencil/FFT/preconditioner/vectors, FP64 dots, alpha/beta,
                     iterate and an outer iterative-refinement residual with an FP64 K */
} jfft_precision;

/* Per-solve report (host struct filled by jfft_solve). */
typedef struct {
  int iters;            /* PCG iterations = updates of u (FP64), or total inner iterations (MIXED) */
  int outer;            /* iterative-refinement sweeps (MIXED), 1 for FP64 */
  int status;           /* jfft_status of the solve */
  double rel_res;       /* ||r_k|| / ||f|| of the recursive residual at stop (FP64 path) */
  double rel_res_true;  /* ||f - K u|| / ||f|| recomputed with the FP64 stiffness after the solve */
  double setup_ms;      /* device time of the right-hand side and start residual */
  double loop_ms;       /* device time of the PCG loop (all sweeps) */
  double post_ms;       /* device time of mean removal, true residual and stresses */
} jfft_report;

/* Create a cell for a dim-dimensional grid.  dim in {2, 3}; n[a] nodes per axis
   (n[2] ignored in 2D); len = cell side lengths (NULL = 1); hip_stream is a
   hipStream_t (NULL = default stream).  Allocates nothing on the device. */
jfft_status jfft_create_cell(int dim, const int n[3], const double len[3], jfft_precision prec,
                             jfft_precond pc, void *hip_stream, jfft_cell_t *out);

/* Create a group of `batch` cells of identical grid, lengths, precision and
   preconditioner on one stream, for throughput on many small cells (Sec. 4
   workloads run one solve per cell and load case).  Each cell of the group has
   its own material, macro strain, CG scalars and stopping test; every kernel
   launch serves the whole group, and a cell that has stopped skips its share.
   1 <= batch <= 65535.  jfft_create_cell is this call with batch = 1.  Only
   jfft_solve_batch and the material, history, timing and option calls accept
   a group with batch > 1; the single-cell operators reject it. */
jfft_status jfft_create_batch(int dim, const int n[3], const double len[3], jfft_precision prec,
                              jfft_precond pc, int batch, void *hip_stream, jfft_cell_t *out);

/* Number of cells in the group (1 for jfft_create_cell handles). */
jfft_status jfft_batch_size(jfft_cell_t cell, int *batch);

/* Bytes of device workspace the cell (or the whole group: the figure grows
   linearly with batch) needs, for caller-side allocation and admission
   control. */
jfft_status jfft_workspace_bytes(jfft_cell_t cell, size_t *bytes);

/* Hand the cell a caller-owned device buffer of at least jfft_workspace_bytes
   bytes (256-byte aligned).  The buffer must outlive every later call on the
   cell.  Without a bound workspace the cell allocates its own at the first call
   that needs it and frees it in jfft_destroy_cell. */
jfft_status jfft_bind_workspace(jfft_cell_t cell, void *dev_ptr, size_t bytes);

/* Material field (Sec. 4): E_dev[N] >= 0 per element (copied, no aliasing
   survives; a group takes E_dev[batch][N], one field per cell), Poisson ratio
   nu in (-1, 0.5) for C^ with unit modulus, shared by the group.  Runs
   Algorithm 2 (Sec. 3.2, d 2^d stiffness applications to unit combs) on the
   device when the preconditioner uses J; the Green symbol G^ (Algorithm 1) is
   evaluated per frequency from the closed-form Fourier symbol of K_ref with
   C_ref = C^ (E_ref = 1). */
jfft_status jfft_set_material(jfft_cell_t cell, const double *E_dev, double nu);

/* Same with explicit Lame constants (lambda, mu) of C^, e.g. the paper's
   reference law lambda^0 = 2/3, mu^0 = 1/2 (Sec. 4).  Requires mu > 0 and
   lambda + 2 mu / d > 0. */
jfft_status jfft_set_material_lame(jfft_cell_t cell, const double *E_dev, double lambda,
                                   double mu);

/* Solve K u = f(macro) with f = -B^T W C(E) macro (eq. lin_system_exp) by PCG
   (Saad Alg. 9.1 in the split form of the footnote to eq.
   prec_lin_system_general), stopping when ||r_k||_2 <= tol ||f||_2 for the
   recursive residual, or after maxit iterations.
     macro_strain: host, d* Mandel entries;
     u0_dev: start vector [d][N] or NULL for u0 = 0;
     u_dev:  out [d][N], the fluctuation with its per-component mean removed
             (Sec. 5: Green-Jacobi iterates carry a mean);
     sigma_dev: out [d*][2^d][N] quadrature-point stresses (Mandel) or NULL
             ([3][2][N] for 2D linear triangles, see jfft_set_element);
     sigma_bar: host out, d* homogenised stresses (1/|Y|) sum w sigma_q;
     report: host out (may be NULL).
   A homogeneous material (||f|| <= 1e-13 ||f_abs||, f_abs assembled from
   absolute element contributions) returns u = 0 after zero iterations.
   Returns JFFT_OK, or JFFT_E_NOT_CONVERGED / JFFT_E_BREAKDOWN with the last
   iterate still written. */
jfft_status jfft_solve(jfft_cell_t cell, const double *macro_strain, double tol, int maxit,
                       const double *u0_dev, double *u_dev, double *sigma_dev,
                       double *sigma_bar, jfft_report *report);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc):
   jfft_set_material (E_dev, nu) followed by jfft_solve, with the cell's
   workspace taken from a static array of the library instead of a bound or
   library-allocated one.  The call makes no hipMalloc, hipFree, graph or
   event creation: kernels, copies of small host tables and one stream
   synchronisation only.  Limit: the cell's jfft_workspace_bytes must not
   exceed 128 MiB (a 64^3 cell in FP64 or mixed precision, 2D cells up to
   512^2); larger cells, group handles, cells whose workspace the library
   allocated itself and cells with kernel timing on return JFFT_E_INVALID
   before any device work.  The array exists once per GPU for the life of
   the process and keeps the last call's contents; every call lays the
   workspace out again, uploads its tables and sets the material, and no
   part of it has to start at zero.  Calls that overlap on one GPU (two
   streams, two threads) race on it.  The cell stays bound to the array
   until jfft_bind_workspace.  Arguments and results as for jfft_solve;
   PCG iterations are launched directly (no graph replay). */
jfft_status jfft_solve_static(jfft_cell_t cell, const double *E_dev, double nu,
                              const double *macro_strain, double tol, int maxit,
                              const double *u0_dev, double *u_dev, double *sigma_dev,
                              double *sigma_bar, jfft_report *report);

/* jfft_solve for every cell of a group at once.  Arrays are those of
   jfft_solve with a leading cell index:
     macro_strains: host [batch][d*];
     u0_dev: [batch][d][N] or NULL;  u_dev: out [batch][d][N];
     sigma_dev: out [batch][d*][2^d][N] or NULL;
     sigma_bars: host out [batch][d*];  reports: host out [batch] or NULL.
   tol and maxit apply to every cell; each cell stops on its own test.  Returns
   JFFT_OK when every cell converged, else JFFT_E_BREAKDOWN if any cell broke
   down, else JFFT_E_NOT_CONVERGED; per-cell outcomes are in reports[i].status.
   The results of a cell do not depend on the other cells of the group. */
jfft_status jfft_solve_batch(jfft_cell_t cell, const double *macro_strains, double tol, int maxit,
                             const double *u0_dev, double *u_dev, double *sigma_dev,
                             double *sigma_bars, jfft_report *reports);

/* Continuous batching (serving): the cells of a group as slots that solves
   enter and leave between chunks of PCG iterations, so a solve that arrives
   while others run joins the next chunk instead of waiting for the group to
   drain.  Every cell keeps its own CG state, stopping test and fixed-order
   reductions, and each chunk starts on the same search-direction buffer, so
   a slot's results are bitwise those of the same cell solved alone (same
   grid, precision, preconditioner, element, options and tunables),
   whatever the other slots hold and whenever it was admitted.  The
   algorithm per slot is that of jfft_solve (Sec. 3.3 and Alg. 1/2; the
   mixed-precision refinement sweeps run per slot as its inner solves stop).
   Slot states (the `states` array): 0 free, 1 running, 2 finished (results
   waiting for jfft_slot_harvest).  While any slot is running or finished,
   calls that act on the whole group (jfft_set_material*, jfft_solve*,
   operators, power-law and topology calls) and the option setters that
   would change a running slot's arithmetic (tunables, stopping rule,
   diagonal method, element, void value, mixed-precision parameters,
   history, workspace binding) fail with JFFT_E_INVALID;
   jfft_set_graph_iterations stays allowed (it changes no result).

   jfft_slot_admit: material E_dev (device, [N] moduli of this slot's cell),
     Poisson ratio nu (the running slots share the Lame constants: a
     different nu is refused while another slot runs), macro strain (host,
     d* values), tol and maxit as in jfft_solve (stopping rule and options of
     the group apply).  The slot must be free.  Enqueues the slot's set-up
     on the group's stream without synchronising: E is checked on the
     device, and an E with negative or non-finite entries finishes the slot
     at once with the status JFFT_E_INVALID (returned by its harvest).
     Errors: JFFT_E_INVALID (slot out of range or busy, bad arguments),
     JFFT_E_HIP.
   jfft_slots_step: at least `iterations` (>= 1) PCG iterations of every
     running slot (whole replays of the captured chunk when graph replay is
     on, else an even number of direct launches), then the bookkeeping of
     slots whose loop stopped (FP64: the owed update; mixed: the next
     refinement sweep, or the end); writes the group's slot states to
     `states` (host, batch ints) if not NULL.  Synchronises the stream.
   jfft_slots_run: chunks of PCG iterations (the captured graph's depth when
     graph replay is on, else 2) with the bookkeeping of jfft_slots_step,
     until at least one slot has finished, no slot runs, or max_ms (>= 0)
     of wall time have passed, checked after each chunk; writes the states
     like jfft_slots_step.  For serving loops: the host wakes only to harvest,
     or every max_ms to admit arrivals.
   jfft_slot_harvest: post-processing of a finished slot as in jfft_solve:
     u_dev (device out [d][N], mean-free fluctuation, or NULL),
     sigma_dev (device out [d*][2^d][N] or NULL), sigma_bar (host out d*),
     report (host out or NULL; loop_ms = host time from admission to the
     stop).  Frees the slot.  Returns the solve's status. */
jfft_status jfft_slot_admit(jfft_cell_t group, int slot, const double *E_dev, double nu,
                            const double *macro_strain, double tol, int maxit);
jfft_status jfft_slots_step(jfft_cell_t group, int iterations, int *states);
jfft_status jfft_slots_run(jfft_cell_t group, double max_ms, int *states);
jfft_status jfft_slot_harvest(jfft_cell_t group, int slot, double *u_dev, double *sigma_dev,
                              double *sigma_bar, jfft_report *report);

/* Launch mode of the PCG loop.  iterations = 0 (default): kernels are
   launched one by one and the host polls the stop flags after 2, 4, ..., 32
   iterations.  An even iterations in [2, 64]: the loop body of that many
   iterations is captured once into a HIP graph (hipStreamBeginCapture on the
   cell's stream) and replayed between polls; iterations past a cell's stop
   cost only their launches.  Needs a stream other than the legacy default
   stream; kernel timing (jfft_enable_timing) switches graph replay off.  The
   graph is rebuilt after a change of the Lame constants, of the history
   capacity or of this setting; a new E field alone keeps it. */
jfft_status jfft_set_graph_iterations(jfft_cell_t cell, int iterations);

/* Launch parameters that do not change what is computed up to rounding:
     tz:    z planes per block of the 3D stiffness kernel (2..nz; 2D ignores
            it).  It sets how the p.q partial sums are grouped, so results
            may differ in the last bits between settings.  By default it is
            chosen from the device's occupancy, the block shape in effect and
            the material kind (linear or power-law), and re-chosen when the
            material kind changes; a value other than the one in effect
            fixes it, and 0 restores (and re-makes) the automatic choice for
            the block shape in effect;
     ygrid: persistent blocks of the y FFT pass per launch (all components
            and cells; 1..65535);
     tiles2d: output nodes per block of the 2D stiffness kernel: 1 = 16 x 16,
            2 = 16 wide x 32 high, 3 = 32 wide x 16, 4 = 32 x 32 (0 restores
            the default, 3 in FP32 and 1 in FP64; 3D ignores it).  Like tz
            it regroups the p.q partial sums;
     xrows: grid rows per block of the x FFT passes, a power of two; values
            above the most that fit in LDS are clamped to it (0 restores the
            default, the most that fit).  It regroups the ||r||^2 partial
            sums;
     tiles3d: output nodes per block of the 3D stiffness kernel: 1 = 16
            wide x 14 high, 2 = 32 x 6 (whole 128-byte rows in FP32).  The
            default is 2 for the FP32 linear-elastic kernels and 1 for FP64
            and the power-law tangent (it follows the material kind); as for
            tz, a value other than the one in effect fixes it and 0 restores
            the default; 2D ignores it.  It regroups the p.q partial sums;
     fused_control: 0 (default) launches a single-block kernel for each
            scalar step of a PCG iteration (alpha, the stopping test, beta);
            1 runs each step in the last block to finish of the kernel that
            produces its partial sums (stiffness, x-forward and Green passes;
            Green and Green-Jacobi preconditioners), saving three launches
            per iteration.  Every block then makes its partial visible with
            a device-scope fence, which on a multi-XCD GPU writes back the
            block's L2 and costs more than a launch on large grids; it can
            pay on small ones.  The two sum the partials in different fixed
            orders.
   tiles2d, tiles3d and xrows act on the kernels of the PCG loop's precision
   (the FP32 kernels of a mixed-precision cell; its FP64 residual and
   post-processing kernels keep the defaults).  jfft_get_tunables reports
   the values in effect (tiles2d, tiles3d and xrows as resolved for the
   grid and the loop's precision).  A change drops any captured graph. */
typedef struct {
  int tz;
  int ygrid;
  int tiles2d;
  int xrows;
  int fused_control;
  int tiles3d;
} jfft_tunables;
jfft_status jfft_set_tunables(jfft_cell_t cell, const jfft_tunables *t);
jfft_status jfft_get_tunables(jfft_cell_t cell, jfft_tunables *t);

/* Operators, for verification and composition (all FP64, device in/out
   [d][N], stream-ordered, no synchronisation):
   out = K in (eq. lin_system_exp, the current material). */
jfft_status jfft_apply_stiffness(jfft_cell_t cell, const double *in_dev, double *out_dev);
/* out = M^-1 in for the cell's preconditioner. */
jfft_status jfft_apply_precond(jfft_cell_t cell, const double *in_dev, double *out_dev);
/* out = M^-1 in as the inner FP32 solves of a JFFT_MIXED cell apply it
   (Sec. 3.3, eq. prec_lin_systemJG_2, with the FP32 J^1/2, spectrum and FFT
   passes): in is rounded to FP32, out widened to FP64 (device [d][N] each).
   JFFT_E_INVALID for an FP64 cell or a group handle. */
jfft_status jfft_apply_precond_fp32(jfft_cell_t cell, const double *in_dev, double *out_dev);
/* f = -B^T W C(E) macro (no mean projection). */
jfft_status jfft_assemble_rhs(jfft_cell_t cell, const double *macro_strain, double *f_dev);
/* diag(K) from Algorithm 2 before the void rule (zero entries kept). */
jfft_status jfft_jacobi_diag(jfft_cell_t cell, double *diag_dev);

/* Per-iteration scalar history of the last FP64 solve: alpha_k, beta_k and
   ||r_k|| for k = 1..min(iters, cap) (host arrays of length cap, any may be
   NULL); the final iteration forms no beta, its entry is NaN.  History is recorded only when enabled before the solve, with
   0 <= cap <= 4096. */
jfft_status jfft_enable_history(jfft_cell_t cell, int cap);
jfft_status jfft_get_history(jfft_cell_t cell, double *alpha, double *beta, double *res,
                             int cap, int *count);
/* The same for cell `index` of a group (jfft_get_history reads cell 0). */
jfft_status jfft_get_batch_history(jfft_cell_t cell, int index, double *alpha, double *beta,
                                   double *res, int cap, int *count);

/* Kernel timing: when enabled, every kernel launch of the cell is bracketed by
   HIP events on the cell's stream and its duration accumulated per kernel
   name.  jfft_kernel_stats returns (name, launches, total ms) of entry i;
   *count receives the number of entries.  Names are static strings. */
jfft_status jfft_enable_timing(jfft_cell_t cell, int on);
jfft_status jfft_kernel_stats(jfft_cell_t cell, int i, const char **name, long *launches,
                              double *total_ms, int *count);
jfft_status jfft_reset_timing(jfft_cell_t cell);

/* How set_material forms diag(K) for the Jacobi part of the preconditioner
   (Sec. 3.2):
   JFFT_DIAG_CLOSED_FORM (default): for the isotropic Q1 elements of this
   library, Algorithm 2's result has a closed form, diag_{alpha I} = k_alpha
   times the sum of the moduli of the 2^d elements around node I, with
   k_alpha = lam g_alpha + mu (g_alpha + sum_b g_b), g_b = vol_e /
   (3^(d-1) h_b^2) (exact Gauss integration); one pass over E, equal to the
   probing result up to rounding;
   JFFT_DIAG_PROBING: Algorithm 2 as stated, d 2^d applications of K to unit
   combs.
   Takes effect at the next set_material (a change clears the material); for
   the power-law material (jfft_set_material_powerlaw), at the next Newton
   solve or operator call. */
#define JFFT_DIAG_CLOSED_FORM 0
#define JFFT_DIAG_PROBING 1
jfft_status jfft_set_diag_method(jfft_cell_t cell, int method);

/* 2D element (Sec. 2; the paper's 2D examples use linear triangles):
   JFFT_ELEM_QUAD (default): bilinear quadrilateral per pixel, 2 x 2 Gauss
   points; JFFT_ELEM_TRI: the pixel split along its anti-diagonal into two
   linear triangles (corners (0,0), (1,0), (0,1) and (1,1), (0,1), (1,0) in
   units of the element edges), one exact quadrature point each.  2D cells
   only (JFFT_E_INVALID otherwise).  With triangles, diag(K) always comes
   from Algorithm 2's probing, the Green operator from K_ref of the
   triangles, and jfft_solve's sigma_dev holds [B][3][2][N] (one point per
   triangle).  A change clears the material. */
#define JFFT_ELEM_QUAD 0
#define JFFT_ELEM_TRI 1
jfft_status jfft_set_element(jfft_cell_t cell, int element);

/* Value of the void rule replacement for exact zeros of diag(K) (Sec. 3.2,
   default 1.0). */
jfft_status jfft_set_void_value(jfft_cell_t cell, double value);

/* Stopping rule of jfft_solve / jfft_solve_batch:
   JFFT_STOP_RELATIVE (default): ||r_k||_2 <= tol ||f||_2;
   JFFT_STOP_ABSOLUTE: ||r_k||_2^2 <= tol, the rule of the paper's numerical
   examples (Sec. 4).  The mixed-precision refinement applies the same rule to
   its FP64 residual. */
#define JFFT_STOP_RELATIVE 0
#define JFFT_STOP_ABSOLUTE 1
jfft_status jfft_set_stop_rule(jfft_cell_t cell, int rule);

/* Mixed precision controls: relative tolerance of each inner FP32 PCG solve
   (default 1e-6) and the cap on refinement sweeps (default 30). */
jfft_status jfft_set_mixed_params(jfft_cell_t cell, double inner_tol, int max_outer);
/* Cap on the iterations of one FP32 inner solve of the mixed refinement
   (default 2000; 0: none).  An inner solve that stalls short of its
   tolerance (FP32 rounding on a very ill-conditioned cell, e.g. with voids)
   then ends and the next FP64 sweep restarts from the corrected residual;
   the maxit of the solve still bounds the inner iterations of all sweeps. */
jfft_status jfft_set_mixed_inner_cap(jfft_cell_t cell, int cap);
/* Refinement sweeps after the first continue the FP32 CG of the previous
   sweep (on = 1, the default: its search direction is kept, rescaled to the
   new residual's norm, and only the residual is replaced by the FP64 one, a
   "reliable update"; in exact arithmetic the iterates are those of one
   uninterrupted CG run) or restart it from the new residual (on = 0, each
   sweep then reduces the residual by the inner tolerance of
   jfft_set_mixed_params).  With on = 1 a sweep ends after the residual has
   dropped by `reduction` (in (0, 1), default 1e-2): the FP32 recursive
   residual drifts from the true one by FP32 rounding times the residual the
   sweep started from, so the replacement must come while that drift is
   still small against the current residual. */
jfft_status jfft_set_mixed_continue(jfft_cell_t cell, int on, double reduction);

/* ---- Power-law material and Newton solve (nonlinear example, Sec. 4;
   Newton linearisation, Sec. 2.2, eq. lin_system) -------------------------
   Single 3D cell only (else JFFT_E_INVALID).  FP64 cells solve every
   Newton step's tangent system by FP64 PCG; JFFT_MIXED cells by FP32 PCG
   (FP32 tangent at an FP32 copy of u, FP64 dots and CG scalars) refined
   against the FP64 tangent residual, as jfft_solve does, so their inner
   stopping rule applies to the true FP64 residual.
   jfft_set_material_powerlaw: phase_dev [N] on the device, element phase
   (entries > 0.5: matrix, else inclusion; negative or non-finite entries:
   JFFT_E_INVALID); copied, the caller keeps ownership.  Matrix: sigma =
   K tr(eps) I + g(eps_eq) dev(eps), g(s) = sigma0 (2/3) s^(n-1) / eps0^n,
   eps_eq = sqrt(2/3 dev(eps):dev(eps)); inclusion: sigma = K_incl tr(eps) I +
   2 mu_incl dev(eps).  Needs K, sigma0, eps0, K_incl, mu_incl > 0, n >= 1.
   The Green reference material is the inclusion's (lambda = K_incl -
   2 mu_incl / 3, mu = mu_incl); the Jacobi factor, if the preconditioner
   has one, is Algorithm 2's diagonal of the tangent K(u) at every Newton
   step: by default in closed form, formed in the pass that evaluates f(u)
   (per Gauss point, w beta^T C beta for the unit strains beta of each
   node's displacement components); with JFFT_DIAG_PROBING by the d 2^d
   applications of K(u) to unit combs.  The
   handle allocates one [3][N] iterate on first use (freed with the handle).
   A later jfft_set_material returns the handle to the linear problem; the
   linear entry points report JFFT_E_NO_MATERIAL while the power-law
   material is set. */
jfft_status jfft_set_material_powerlaw(jfft_cell_t cell, const double *phase_dev, double K,
                                       double sigma0, double eps0, double n, double K_incl,
                                       double mu_incl);
/* Newton from u = 0 on f(u) = -B^T W sigma(E + B u): stop when ||f||_2 <
   newton_tol, else solve K(u) du = f(u) by PCG from du = 0 (at most maxit
   iterations; a PCG breakdown ends that inner solve and the step goes on)
   and set u += du; at most max_newton steps.  The inner solve stops, under
   the relative stop rule (default), at ||r|| <= max(pcg_tol, newton_tol /
   (10 ||f||)) ||f|| (0 < pcg_tol < 1); under JFFT_STOP_ABSOLUTE
   (jfft_set_stop_rule) at ||r||^2 <= pcg_tol, the rule of Sec. 4.  Outputs: u_dev [3][N] device (mean
   removed, Sec. 5), sigma_bar[6] host (volume average of sigma(E + B u),
   Mandel), and optionally (host, may be NULL) pcg_iters[max_newton] (PCG
   iterations per step), res_norms[max_newton + 1] (||f|| before each step
   and at the end) and *steps (Newton steps taken).  Returns JFFT_OK when
   converged, else JFFT_E_NOT_CONVERGED with every output written. */
jfft_status jfft_solve_newton(jfft_cell_t cell, const double *macro_strain, double newton_tol,
                              double pcg_tol, int max_newton, int maxit, double *u_dev,
                              double *sigma_bar, int *pcg_iters, double *res_norms, int *steps);
/* Operators of a Newton step at the iterate uk_dev [3][N] (device) for the
   macroscopic strain macro_strain[6] (host): f = -B^T W sigma(E + B uk);
   out = K(uk) in; diag(K(uk)) by Algorithm 2 (no void rule).  Device
   outputs [3][N]; synchronous.  The diagonal follows jfft_set_diag_method. */
jfft_status jfft_powerlaw_force(jfft_cell_t cell, const double *macro_strain, const double *uk_dev,
                                double *f_dev);
jfft_status jfft_powerlaw_tangent(jfft_cell_t cell, const double *macro_strain, const double *uk_dev,
                                  const double *in_dev, double *out_dev);
jfft_status jfft_powerlaw_jacobi_diag(jfft_cell_t cell, const double *macro_strain,
                                      const double *uk_dev, double *diag_dev);

/* ---- Phase-field topology optimisation (Sec. 4, eq. aim_fun and eq.
   lin_system_topopt) ------------------------------------------------------
   The handle is a group of 3 2D cells with JFFT_ELEM_TRI (jfft_create_batch
   with batch 3, then jfft_set_element; else JFFT_E_INVALID); cell g holds the
   unit load case e_g (Mandel) on the common density rho_dev [N] (device,
   node-sampled: pixel e takes rho of its lowest node; C = rho C0 with Lame
   constants lambda0, mu0).
   jfft_topopt_eval: f = sum_g ||sigma_bar_g - t_g||^2 + f_pf with targets t
   (host, 9 values, row g = t_g in Mandel form) and f_pf = eta int |grad
   rho|^2 + (1/eta) int rho^2 (1 - rho)^2 (rho linear on the triangles for
   the gradient term, the double well by nodal quadrature).  Solves the three
   load cases from u = 0 to relative residual tol (at most maxit iterations,
   the cell's stop rule and precision), then writes f_out[3] = (f, f_sigma,
   f_pf) (host), grad_dev [N] (device; f_sigma's part by the mutual-energy
   identity, no adjoint solve) and iters[3] (host, may be NULL).  Returns the
   solve's status (JFFT_E_NOT_CONVERGED, JFFT_E_BREAKDOWN) if a solve fails.
   jfft_topopt_lbfgs: projected L-BFGS on [0, 1] from rho_dev (in: start, out:
   the last accepted iterate), memory m (1..64), at most n_iter steps: bound
   variables held by their gradient are frozen for a step; the trial
   clip(rho + alpha d), alpha halved from 1 (at most 30 times) until
   f(trial) <= f + 1e-4 g . (trial - rho); a pair (s, y) is kept when
   y.s > 1e-12 |s| |y|; the first direction is -g scaled to a largest entry
   of 0.1, later ones use H0 = s.y / y.y of the newest pair; stops early when
   no halving decreases f.  Host outputs (each may be NULL): f_hist and
   gnorm_hist (max |g|) of the accepted iterates [n_iter + 1], iters_hist
   [(n_iter + 1) * 3] (the three solves' iterations), *steps, *evals
   (objective evaluations), *pcg_total (PCG iterations of every evaluation,
   rejected trials included).  The handle allocates (6 + 2 m) N doubles on
   first use (freed with the handle).  Mixed-precision groups follow the
   refinement loop of jfft_solve; on rough densities of very high contrast
   (or with exact voids) the FP32 operator's rounding exceeds what the
   refinement can correct (then JFFT_E_NOT_CONVERGED): use FP64 groups for
   whole optimisation runs. */
jfft_status jfft_topopt_eval(jfft_cell_t group, const double *rho_dev, double lambda0, double mu0,
                             const double *targets, double eta, double tol, int maxit,
                             double *f_out, double *grad_dev, int *iters);
jfft_status jfft_topopt_lbfgs(jfft_cell_t group, double *rho_dev, double lambda0, double mu0,
                              const double *targets, double eta, double tol, int maxit,
                              int n_iter, int m, double *f_hist, double *gnorm_hist,
                              int *iters_hist, int *steps, int *evals, long long *pcg_total);

void jfft_destroy_cell(jfft_cell_t cell);
const char *jfft_last_error(void);
const char *jfft_version(void);

#ifdef __cplusplus
}
#endif
#endif /* JFFT_H */
