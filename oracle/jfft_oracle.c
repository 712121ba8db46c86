/*
 * jfft_oracle.c -- plain, slow FP64 CPU oracle for the Green-Jacobi (J-FFT)
 * preconditioned conjugate-gradient cell problem of
 *   M. Ladecky, I. Pultarova, F. Bignonnet, I. Jodicke, J. Zeman, L. Pastewka,
 *   "Jacobi-accelerated FFT-based solver for smooth high-contrast data",
 *   arXiv:2508.02613.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; it is written for a reader who
 * checks it against the paper, not for speed:
 *   - explicit element loops with the full strain-displacement matrix B_q of
 *     every quadrature point (Sec. 2.1, eq. disc_wf);
 *   - a naive separable DFT with its own twiddle table (eq. prec_lin_systemG_FFT);
 *   - Algorithm 1 (Green symbol from unit impulse responses) and Algorithm 2
 *     (Jacobi diagonal from d*2^d comb applications) taken step by step;
 *   - textbook PCG (Saad, Alg. 9.1) with the split Green-Jacobi operator
 *     J^1/2 F^-1 G^ F J^1/2 (eq. prec_lin_systemJG_2).
 * or_solve has two options that no paper passage asks for, both used only to
 * measure how far rounding moves the stopping iteration (two FP64 programs of
 * the same method round differently): a nonzero noise_seed moves every entry
 * of each K p and M^-1 r result by one ulp in a seeded direction (ulp_noise);
 * dot_mode = 1 forms every inner product and norm with Dot2 (as if in twice
 * the working precision) instead of the serial sum in index order.  With
 * noise_seed = 0 and dot_mode = 0 the arithmetic is plain.
 * The only parallelism is OpenMP over independent DFT lines and over
 * same-colour elements (elements that share no node), which changes no
 * arithmetic result.  Reductions are serial and in index order.
 *
 * Conventions (fixed where the paper is silent):
 *   grid: n[0] x n[1] (x n[2]) nodes, x fastest; node (i,j,k) at (i h0, j h1, k h2),
 *         h_a = len[a] / n[a]; periodic.  Element (i,j,k) spans nodes (i+c0, j+c1, k+c2)
 *         mod n, c in {0,1}^d, local corner index c = c0 + 2 c1 + 4 c2.
 *   element: bilinear quad / trilinear hex, 2-point Gauss-Legendre rule per axis,
 *         xi in {1/2 - 1/(2 sqrt 3), 1/2 + 1/(2 sqrt 3)}, weight = element volume / 2^d.
 *   Mandel order: 3D (11,22,33,23,13,12), 2D (11,22,12); shear entries carry sqrt 2.
 *   material: C_e = E_e * C^ with C^ isotropic (lambda, mu): lambda + 2 mu on the normal
 *         diagonal, lambda between normals, 2 mu on the shear diagonal.  2D is plane strain.
 *   fields: u[a*N + idx] for component a, N = number of nodes.
 *   DFT: forward sum x_j exp(-2 pi i jk/n) (unnormalised), inverse exp(+...) / N.
 */
#include <complex.h>
#include <stdint.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVALID 1
#define OR_E_ODD_GRID 2
#define OR_E_NOT_CONVERGED 4
#define OR_E_BREAKDOWN 5
#define OR_E_OOM 6

#define PC_NONE 0
#define PC_GREEN 1
#define PC_JACOBI 2
#define PC_GREEN_JACOBI 3

#define MAXD 3
#define MAXDS 6
#define MAXLOC 8 /* 2^d corners / quadrature points */

typedef struct {
  int dim;      /* d */
  int n[MAXD];  /* nodes per axis (n[2] = 1 in 2D) */
  double h[MAXD];
  double vol;   /* |Y| */
  long N;       /* number of nodes = number of elements */
  int nloc;     /* 2^d */
  int ds;       /* d* */
  double w;     /* quadrature weight (element volume / 2^d) */
  /* B[q][row][col]: Mandel strain at qp q from local dof col = corner*d + comp */
  double B[MAXLOC][MAXDS][MAXD * MAXLOC];
} grid_t;

static int grid_init(grid_t *g, int dim, const int *n, const double *len) {
  if (dim != 2 && dim != 3) return OR_E_INVALID;
  memset(g, 0, sizeof(*g));
  g->dim = dim;
  g->N = 1;
  g->vol = 1.0;
  double evol = 1.0;
  for (int a = 0; a < MAXD; ++a) {
    if (a < dim) {
      if (n[a] < 1) return OR_E_INVALID;
      g->n[a] = n[a];
      double l = len ? len[a] : 1.0;
      if (!(l > 0.0)) return OR_E_INVALID;
      g->h[a] = l / n[a];
      g->vol *= l;
      evol *= g->h[a];
    } else {
      g->n[a] = 1;
      g->h[a] = 1.0;
    }
    g->N *= g->n[a];
  }
  g->nloc = 1 << dim;
  g->ds = dim * (dim + 1) / 2;
  g->w = evol / g->nloc;

  /* Shape-function gradients at the Gauss points and the Mandel B matrices
     (Sec. 2.1: B^beta_{Q,I} = d phi_I / d x_beta at x_Q). */
  const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  const double s2 = 1.0 / sqrt(2.0); /* sqrt2 * (1/2) symmetrisation */
  for (int q = 0; q < g->nloc; ++q) {
    double xi[MAXD];
    for (int a = 0; a < dim; ++a) xi[a] = gp[(q >> a) & 1];
    double grad[MAXLOC][MAXD];
    for (int c = 0; c < g->nloc; ++c) {
      for (int a = 0; a < dim; ++a) {
        double v = (((c >> a) & 1) ? 1.0 : -1.0) / g->h[a];
        for (int b = 0; b < dim; ++b) {
          if (b == a) continue;
          v *= ((c >> b) & 1) ? xi[b] : (1.0 - xi[b]);
        }
        grad[c][a] = v;
      }
    }
    for (int c = 0; c < g->nloc; ++c) {
      int c0 = c * dim;
      if (dim == 2) {
        g->B[q][0][c0 + 0] = grad[c][0];
        g->B[q][1][c0 + 1] = grad[c][1];
        g->B[q][2][c0 + 0] = s2 * grad[c][1];
        g->B[q][2][c0 + 1] = s2 * grad[c][0];
      } else {
        g->B[q][0][c0 + 0] = grad[c][0];
        g->B[q][1][c0 + 1] = grad[c][1];
        g->B[q][2][c0 + 2] = grad[c][2];
        /* 23 */
        g->B[q][3][c0 + 1] = s2 * grad[c][2];
        g->B[q][3][c0 + 2] = s2 * grad[c][1];
        /* 13 */
        g->B[q][4][c0 + 0] = s2 * grad[c][2];
        g->B[q][4][c0 + 2] = s2 * grad[c][0];
        /* 12 */
        g->B[q][5][c0 + 0] = s2 * grad[c][1];
        g->B[q][5][c0 + 1] = s2 * grad[c][0];
      }
    }
  }
  return OR_OK;
}

/* Isotropic Mandel stiffness (Sec. 4 constitutive law, index form
   lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk)). */
static void mandel_iso(int dim, double lam, double mu, double C[MAXDS][MAXDS]) {
  int ds = dim * (dim + 1) / 2;
  memset(C, 0, sizeof(double) * MAXDS * MAXDS);
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) C[i][j] = lam + (i == j ? 2.0 * mu : 0.0);
  for (int i = dim; i < ds; ++i) C[i][i] = 2.0 * mu;
}

static long node_of(const grid_t *g, long e, int c) {
  long i = e % g->n[0];
  long j = (e / g->n[0]) % g->n[1];
  long k = e / ((long)g->n[0] * g->n[1]);
  i = (i + (c & 1)) % g->n[0];
  j = (j + ((c >> 1) & 1)) % g->n[1];
  k = (k + ((c >> 2) & 1)) % g->n[2];
  return i + (long)g->n[0] * (j + (long)g->n[1] * k);
}

/* Element vector y_e = E_e sum_q w B_q^T C B_q u_e  (eq. lin_system_exp). */
static void element_apply(const grid_t *g, const double C[MAXDS][MAXDS], double Ee,
                          const double *ue, double *ye) {
  const int nd = g->dim * g->nloc;
  for (int k = 0; k < nd; ++k) ye[k] = 0.0;
  for (int q = 0; q < g->nloc; ++q) {
    double eps[MAXDS], sig[MAXDS];
    for (int r = 0; r < g->ds; ++r) {
      double s = 0.0;
      for (int k = 0; k < nd; ++k) s += g->B[q][r][k] * ue[k];
      eps[r] = s;
    }
    for (int r = 0; r < g->ds; ++r) {
      double s = 0.0;
      for (int t = 0; t < g->ds; ++t) s += C[r][t] * eps[t];
      sig[r] = Ee * s;
    }
    for (int k = 0; k < nd; ++k) {
      double s = 0.0;
      for (int r = 0; r < g->ds; ++r) s += g->B[q][r][k] * sig[r];
      ye[k] += g->w * s;
    }
  }
}

static int all_even(const grid_t *g) {
  for (int a = 0; a < g->dim; ++a)
    if (g->n[a] % 2) return 0;
  return 1;
}

static void stiffness_apply(const grid_t *g, double lam, double mu, const double *E,
                            const double *u, double *out) {
  double C[MAXDS][MAXDS];
  mandel_iso(g->dim, lam, mu, C);
  const long N = g->N;
  const int d = g->dim;
  memset(out, 0, sizeof(double) * d * N);
  /* Colour elements by the parity of their index so that, on even grids,
     elements of one colour share no node and can be processed in parallel. */
  int ncolor = all_even(g) ? g->nloc : 1;
  for (int color = 0; color < ncolor; ++color) {
#pragma omp parallel for schedule(static) if (ncolor > 1)
    for (long e = 0; e < N; ++e) {
      if (ncolor > 1) {
        long i = e % g->n[0], j = (e / g->n[0]) % g->n[1], k = e / ((long)g->n[0] * g->n[1]);
        int par = (int)(i & 1) | ((int)(j & 1) << 1) | ((int)(k & 1) << 2);
        if (par != color) continue;
      }
      double ue[MAXD * MAXLOC], ye[MAXD * MAXLOC];
      long nodes[MAXLOC];
      for (int c = 0; c < g->nloc; ++c) {
        nodes[c] = node_of(g, e, c);
        for (int a = 0; a < d; ++a) ue[c * d + a] = u[a * N + nodes[c]];
      }
      element_apply(g, C, E[e], ue, ye);
      for (int c = 0; c < g->nloc; ++c)
        for (int a = 0; a < d; ++a) out[a * N + nodes[c]] += ye[c * d + a];
    }
  }
}

/* ---------------------------------------------------------------- exports */

int or_stiffness(int dim, const int *n, const double *len, double lam, double mu,
                 const double *E, const double *u, double *out) {
  grid_t g;
  int st = grid_init(&g, dim, n, len);
  if (st) return st;
  stiffness_apply(&g, lam, mu, E, u, out);
  return OR_OK;
}

/* (K u) at one node only: sum over the 2^d elements that contain it. */
int or_stiffness_at_node(int dim, const int *n, const double *len, double lam, double mu,
                         const double *E, const double *u, long node, double *out_d) {
  grid_t g;
  int st = grid_init(&g, dim, n, len);
  if (st) return st;
  double C[MAXDS][MAXDS];
  mandel_iso(dim, lam, mu, C);
  const long N = g.N;
  long i = node % g.n[0], j = (node / g.n[0]) % g.n[1], k = node / ((long)g.n[0] * g.n[1]);
  for (int a = 0; a < dim; ++a) out_d[a] = 0.0;
  for (int c = 0; c < g.nloc; ++c) {
    /* element whose local corner c is this node */
    long ei = (i - (c & 1) + g.n[0]) % g.n[0];
    long ej = (j - ((c >> 1) & 1) + g.n[1]) % g.n[1];
    long ek = (k - ((c >> 2) & 1) + g.n[2]) % g.n[2];
    long e = ei + (long)g.n[0] * (ej + (long)g.n[1] * ek);
    double ue[MAXD * MAXLOC], ye[MAXD * MAXLOC];
    for (int cc = 0; cc < g.nloc; ++cc) {
      long nd = node_of(&g, e, cc);
      for (int a = 0; a < dim; ++a) ue[cc * dim + a] = u[a * N + nd];
    }
    element_apply(&g, C, E[e], ue, ye);
    for (int a = 0; a < dim; ++a) out_d[a] += ye[c * dim + a];
  }
  return OR_OK;
}

/* f = -B^T W C(E) Ebar (eq. lin_system_exp).  If fabs_out is non-NULL it also
   receives the same assembly of absolute element contributions, used as the
   scale of the cancellation test for a homogeneous material. */
int or_rhs(int dim, const int *n, const double *len, double lam, double mu, const double *E,
           const double *macro, double *f, double *fabs_out) {
  grid_t g;
  int st = grid_init(&g, dim, n, len);
  if (st) return st;
  double C[MAXDS][MAXDS];
  mandel_iso(dim, lam, mu, C);
  const long N = g.N;
  const int nd = dim * g.nloc;
  double sig0[MAXDS];
  for (int r = 0; r < g.ds; ++r) {
    double s = 0.0;
    for (int t = 0; t < g.ds; ++t) s += C[r][t] * macro[t];
    sig0[r] = s;
  }
  double ye0[MAXD * MAXLOC];
  for (int k = 0; k < nd; ++k) {
    double s = 0.0;
    for (int q = 0; q < g.nloc; ++q)
      for (int r = 0; r < g.ds; ++r) s += g.w * g.B[q][r][k] * sig0[r];
    ye0[k] = s;
  }
  memset(f, 0, sizeof(double) * dim * N);
  if (fabs_out) memset(fabs_out, 0, sizeof(double) * dim * N);
  for (long e = 0; e < N; ++e) {
    for (int c = 0; c < g.nloc; ++c) {
      long node = node_of(&g, e, c);
      for (int a = 0; a < dim; ++a) {
        double v = -E[e] * ye0[c * dim + a];
        f[a * N + node] += v;
        if (fabs_out) fabs_out[a * N + node] += fabs(v);
      }
    }
  }
  return OR_OK;
}

/* Quadrature-point stresses sigma_q = C_e (Ebar + B_q u_e) and the homogenised
   stress sigma_bar = (1/|Y|) sum_e sum_q w sigma_q (Sec. 4.3 objective). */
int or_stress(int dim, const int *n, const double *len, double lam, double mu, const double *E,
              const double *macro, const double *u, double *sigma_q, double *sigma_bar) {
  grid_t g;
  int st = grid_init(&g, dim, n, len);
  if (st) return st;
  double C[MAXDS][MAXDS];
  mandel_iso(dim, lam, mu, C);
  const long N = g.N;
  const int nd = dim * g.nloc;
  double acc[MAXDS] = {0};
  for (long e = 0; e < N; ++e) {
    double ue[MAXD * MAXLOC];
    for (int c = 0; c < g.nloc; ++c) {
      long node = node_of(&g, e, c);
      for (int a = 0; a < dim; ++a) ue[c * dim + a] = u ? u[a * N + node] : 0.0;
    }
    for (int q = 0; q < g.nloc; ++q) {
      double eps[MAXDS];
      for (int r = 0; r < g.ds; ++r) {
        double s = macro[r];
        for (int k = 0; k < nd; ++k) s += g.B[q][r][k] * ue[k];
        eps[r] = s;
      }
      for (int r = 0; r < g.ds; ++r) {
        double s = 0.0;
        for (int t = 0; t < g.ds; ++t) s += C[r][t] * eps[t];
        s *= E[e];
        if (sigma_q) sigma_q[((long)r * g.nloc + q) * N + e] = s;
        acc[r] += g.w * s;
      }
    }
  }
  for (int r = 0; r < g.ds; ++r) sigma_bar[r] = acc[r] / g.vol;
  return OR_OK;
}

/* Algorithm 2: diag(K) from d * 2^d applications of K to unit combs placed on
   the stride-2 sub-grid of every offset.  Needs an even number of nodes per
   axis.  *napply receives the number of operator applications performed. */
int or_jacobi_diag(int dim, const int *n, const double *len, double lam, double mu,
                   const double *E, double *diag, int *napply) {
  grid_t g;
  int st = grid_init(&g, dim, n, len);
  if (st) return st;
  if (!all_even(&g)) return OR_E_ODD_GRID;
  const long N = g.N;
  double *comb = (double *)malloc(sizeof(double) * dim * N);
  double *resp = (double *)malloc(sizeof(double) * dim * N);
  if (!comb || !resp) {
    free(comb);
    free(resp);
    return OR_E_OOM;
  }
  int count = 0;
  for (int a = 0; a < dim; ++a) {
    for (int off = 0; off < g.nloc; ++off) {
      memset(comb, 0, sizeof(double) * dim * N);
      for (long nI = 0; nI < N; ++nI) {
        long i = nI % g.n[0], j = (nI / g.n[0]) % g.n[1], k = nI / ((long)g.n[0] * g.n[1]);
        int par = (int)(i & 1) | ((int)(j & 1) << 1) | ((int)(k & 1) << 2);
        if (par == off) comb[a * N + nI] = 1.0;
      }
      stiffness_apply(&g, lam, mu, E, comb, resp);
      ++count;
      for (long nI = 0; nI < N; ++nI)
        if (comb[a * N + nI] == 1.0) diag[a * N + nI] = resp[a * N + nI];
    }
  }
  free(comb);
  free(resp);
  if (napply) *napply = count;
  return OR_OK;
}

/* Naive separable DFT over all d axes of a complex field of g->N points.
   sign = -1: forward (unnormalised); sign = +1: inverse without 1/N. */
static int dft_nd(const grid_t *g, double complex *x, int sign) {
  for (int ax = 0; ax < g->dim; ++ax) {
    const int n = g->n[ax];
    double complex *tw = (double complex *)malloc(sizeof(double complex) * n);
    if (!tw) return OR_E_OOM;
    for (int j = 0; j < n; ++j) {
      double ang = 2.0 * M_PI * (double)j / (double)n;
      tw[j] = cos(ang) + sign * sin(ang) * I;
    }
    long stride = 1;
    for (int b = 0; b < ax; ++b) stride *= g->n[b];
    const long nlines = g->N / n;
    int fail = 0;
#pragma omp parallel
    {
      double complex *line = (double complex *)malloc(sizeof(double complex) * n);
      double complex *outl = (double complex *)malloc(sizeof(double complex) * n);
      if (!line || !outl) {
#pragma omp atomic write
        fail = 1;
      } else {
#pragma omp for schedule(static)
        for (long L = 0; L < nlines; ++L) {
          long lo = L % stride, hi = L / stride;
          long base = lo + hi * stride * n;
          for (int j = 0; j < n; ++j) line[j] = x[base + (long)j * stride];
          for (int k = 0; k < n; ++k) {
            double complex s = 0.0;
            for (int j = 0; j < n; ++j) s += line[j] * tw[((long)j * k) % n];
            outl[k] = s;
          }
          for (int k = 0; k < n; ++k) x[base + (long)k * stride] = outl[k];
        }
      }
      free(line);
      free(outl);
    }
    free(tw);
    if (fail) return OR_E_OOM;
  }
  return OR_OK;
}

int or_dft(int dim, const int *n, const double *in_re, const double *in_im, double *out_re,
           double *out_im, int sign) {
  grid_t g;
  int st = grid_init(&g, dim, n, NULL);
  if (st) return st;
  double complex *x = (double complex *)malloc(sizeof(double complex) * g.N);
  if (!x) return OR_E_OOM;
  for (long i = 0; i < g.N; ++i) x[i] = in_re[i] + (in_im ? in_im[i] : 0.0) * I;
  st = dft_nd(&g, x, sign);
  for (long i = 0; i < g.N; ++i) {
    out_re[i] = creal(x[i]);
    out_im[i] = cimag(x[i]);
  }
  free(x);
  return st;
}

/* In-place inverse of a small complex matrix by Gauss-Jordan elimination with
   partial pivoting.  Returns 0 on success, 1 if singular. */
static int cinv(int d, double complex A[MAXD][MAXD], double complex Ainv[MAXD][MAXD]) {
  double complex M[MAXD][2 * MAXD];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < 2 * d; ++j) M[i][j] = (j < d) ? A[i][j] : (j - d == i ? 1.0 : 0.0);
  for (int col = 0; col < d; ++col) {
    int piv = col;
    for (int r = col + 1; r < d; ++r)
      if (cabs(M[r][col]) > cabs(M[piv][col])) piv = r;
    if (cabs(M[piv][col]) == 0.0) return 1;
    if (piv != col)
      for (int j = 0; j < 2 * d; ++j) {
        double complex t = M[col][j];
        M[col][j] = M[piv][j];
        M[piv][j] = t;
      }
    double complex p = M[col][col];
    for (int j = 0; j < 2 * d; ++j) M[col][j] /= p;
    for (int r = 0; r < d; ++r) {
      if (r == col) continue;
      double complex fct = M[r][col];
      for (int j = 0; j < 2 * d; ++j) M[r][j] -= fct * M[col][j];
    }
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) Ainv[i][j] = M[i][j + d];
  return 0;
}

/* Algorithm 1: Green symbol G^[beta][alpha](k), stored as G[(beta*d+alpha)*N + k].
   Step 1 applies K_ref (E = 1, reference Lame constants) to a unit impulse of
   every component at node 0; step 2 takes the DFT of every response component;
   step 3 inverts the d x d block at every frequency except k = 0, where the
   zero-mean constraint sets G^ = 0. */
int or_green(int dim, const int *n, const double *len, double lam_ref, double mu_ref,
             double *G_re, double *G_im) {
  grid_t g;
  int st = grid_init(&g, dim, n, len);
  if (st) return st;
  const long N = g.N;
  const int d = dim;
  double *ones = (double *)malloc(sizeof(double) * N);
  double *imp = (double *)calloc((size_t)d * N, sizeof(double));
  double *resp = (double *)malloc(sizeof(double) * d * N);
  double complex *Kh = (double complex *)malloc(sizeof(double complex) * d * d * N);
  if (!ones || !imp || !resp || !Kh) {
    free(ones);
    free(imp);
    free(resp);
    free(Kh);
    return OR_E_OOM;
  }
  for (long i = 0; i < N; ++i) ones[i] = 1.0;
  /* Step 1 + 2 */
  for (int a = 0; a < d; ++a) {
    memset(imp, 0, sizeof(double) * d * N);
    imp[a * N + 0] = 1.0;
    stiffness_apply(&g, lam_ref, mu_ref, ones, imp, resp);
    for (int b = 0; b < d; ++b) {
      double complex *dst = Kh + (long)(b * d + a) * N;
      for (long i = 0; i < N; ++i) dst[i] = resp[b * N + i];
      st = dft_nd(&g, dst, -1);
      if (st) goto done;
    }
  }
  /* Step 3 */
  for (long kf = 0; kf < N; ++kf) {
    double complex A[MAXD][MAXD], Ai[MAXD][MAXD];
    if (kf == 0) {
      for (int b = 0; b < d; ++b)
        for (int a = 0; a < d; ++a) Ai[b][a] = 0.0;
    } else {
      for (int b = 0; b < d; ++b)
        for (int a = 0; a < d; ++a) A[b][a] = Kh[(long)(b * d + a) * N + kf];
      if (cinv(d, A, Ai)) {
        st = OR_E_INVALID;
        goto done;
      }
    }
    for (int b = 0; b < d; ++b)
      for (int a = 0; a < d; ++a) {
        G_re[(long)(b * d + a) * N + kf] = creal(Ai[b][a]);
        G_im[(long)(b * d + a) * N + kf] = cimag(Ai[b][a]);
      }
  }
done:
  free(ones);
  free(imp);
  free(resp);
  free(Kh);
  return st;
}

/* z = M^-1 r for the four preconditioners (eqs. prec_lin_systemG_FFT,
   prec_lin_systemJ, prec_lin_systemJG_2):
     NONE: z = r;  JACOBI: z = r / diag;  GREEN: z = Re F^-1 G^ F r;
     GREEN_JACOBI: z = J^1/2 Re F^-1 G^ F J^1/2 r,  J^1/2 = diag^-1/2.
   `diag` is diag(K) after the void rule.  imag_ratio (optional) receives
   max|Im| / max|Re| of the inverse transform. */
static int precond_apply(const grid_t *g, int pc, const double *diag, const double *G_re,
                         const double *G_im, const double *r, double *z, double *imag_ratio,
                         double complex *work) {
  const long N = g->N;
  const int d = g->dim;
  if (pc == PC_NONE) {
    memcpy(z, r, sizeof(double) * d * N);
    return OR_OK;
  }
  if (pc == PC_JACOBI) {
    for (long i = 0; i < d * N; ++i) z[i] = r[i] / diag[i];
    return OR_OK;
  }
  double complex *S = work;          /* d spectra */
  double complex *Z = work + d * N;  /* d spectra */
  for (int a = 0; a < d; ++a) {
    for (long i = 0; i < N; ++i) {
      double s = r[a * N + i];
      if (pc == PC_GREEN_JACOBI) s *= 1.0 / sqrt(diag[a * N + i]);
      S[a * N + i] = s;
    }
    int st = dft_nd(g, S + a * N, -1);
    if (st) return st;
  }
  for (int b = 0; b < d; ++b)
    for (long k = 0; k < N; ++k) {
      double complex acc = 0.0;
      for (int a = 0; a < d; ++a) {
        double complex Gba = G_re[(long)(b * d + a) * N + k] + G_im[(long)(b * d + a) * N + k] * I;
        acc += Gba * S[a * N + k];
      }
      Z[b * N + k] = acc;
    }
  double maxre = 0.0, maxim = 0.0;
  for (int b = 0; b < d; ++b) {
    int st = dft_nd(g, Z + b * N, +1);
    if (st) return st;
    for (long i = 0; i < N; ++i) {
      double complex v = Z[b * N + i] / (double)N;
      if (fabs(creal(v)) > maxre) maxre = fabs(creal(v));
      if (fabs(cimag(v)) > maxim) maxim = fabs(cimag(v));
      double t = creal(v);
      if (pc == PC_GREEN_JACOBI) t *= 1.0 / sqrt(diag[b * N + i]);
      z[b * N + i] = t;
    }
  }
  if (imag_ratio) *imag_ratio = (maxre > 0.0) ? maxim / maxre : maxim;
  return OR_OK;
}

/* Void rule of Sec. 3.2: exact zeros of diag(K) are replaced by `void_value`. */
static void void_rule(long n, double *diag, double void_value) {
  for (long i = 0; i < n; ++i)
    if (diag[i] == 0.0) diag[i] = void_value;
}

int or_precond(int dim, const int *n, const double *len, int pc, const double *diag_raw,
               double void_value, const double *G_re, const double *G_im, const double *r,
               double *z, double *imag_ratio) {
  grid_t g;
  int st = grid_init(&g, dim, n, len);
  if (st) return st;
  const long N = g.N;
  double *diag = NULL;
  if (pc == PC_JACOBI || pc == PC_GREEN_JACOBI) {
    diag = (double *)malloc(sizeof(double) * dim * N);
    if (!diag) return OR_E_OOM;
    memcpy(diag, diag_raw, sizeof(double) * dim * N);
    void_rule(dim * N, diag, void_value);
  }
  double complex *work = (double complex *)malloc(sizeof(double complex) * 2 * dim * N);
  if (!work) {
    free(diag);
    return OR_E_OOM;
  }
  st = precond_apply(&g, pc, diag, G_re, G_im, r, z, imag_ratio, work);
  free(work);
  free(diag);
  return st;
}

static double dot(long n, const double *a, const double *b) {
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Dot product as if accumulated in twice the working precision and then
   rounded: algorithm Dot2 of Ogita, Rump and Oishi, "Accurate sum and dot
   product" (SIAM J. Sci. Comput. 26, 2005), with the error-free product from
   fma and Knuth's error-free sum.  Used by or_solve when dot_mode = 1. */
static double dot2(long n, const double *a, const double *b) {
  if (n <= 0) return 0.0;
  double p = a[0] * b[0];
  double s = fma(a[0], b[0], -p);
  for (long i = 1; i < n; ++i) {
    const double h = a[i] * b[i];
    const double r = fma(a[i], b[i], -h);
    const double t = p + h;
    const double z = t - p;
    const double q = (p - (t - z)) + (h - z);
    p = t;
    s += q + r;
  }
  return p + s;
}

static double dotm(int mode, long n, const double *a, const double *b) {
  return mode == 1 ? dot2(n, a, b) : dot(n, a, b);
}

/* The inner product of or_solve's dot_mode (0 serial, 1 Dot2), exported so
   that the tests can pin it. */
double or_dot(int mode, long n, const double *a, const double *b) { return dotm(mode, n, a, b); }

/* Full solve: assemble f, set up the preconditioner, run PCG (Saad Alg. 9.1
   in the split form of the footnote to eq. prec_lin_system_general), then
   remove the mean of u per component and compute sigma_bar.

   stop_mode 0: stop when ||r_k||_2 <= tol ||f||_2 (recursive residual);
   stop_mode 1: stop when ||r_k||_2^2 <= tol (the absolute rule of Sec. 4).
   iters receives the number of updates of u.  The histories (length hist_len,
   each optional) receive alpha_k, beta_k and ||r_k||_2 for k = 1.. .
   timing (optional, 3 entries) receives wall seconds of setup, PCG loop, post.
   f_in (optional) replaces the assembled right-hand side; project_rhs != 0
   subtracts its per-component mean.
   Returns OR_OK, OR_E_NOT_CONVERGED (iterate still written), OR_E_BREAKDOWN,
   OR_E_ODD_GRID or OR_E_INVALID. */
#include <time.h>
static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* Rounding-difference model for measuring how far the stopping iteration
   moves between two FP64 evaluations of the same method (two programs round
   every operator application differently): every entry of v moves by one
   unit in the last place, up or down.  The direction is the top bit of
   splitmix64 (Steele, Lea and Flood, 2014) applied to a counter built from
   the seed, the iteration, the operator and the entry index.  Zeros stay. */
static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

static void ulp_noise(double *v, long n, uint64_t seed, int iter, int op) {
  const uint64_t base = splitmix64(seed) ^ ((uint64_t)(unsigned)iter << 33) ^ ((uint64_t)op << 32);
  for (long i = 0; i < n; ++i) {
    if (v[i] == 0.0) continue;
    const uint64_t h = splitmix64(base + (uint64_t)i);
    v[i] = nextafter(v[i], (h >> 63) ? INFINITY : -INFINITY);
  }
}

int or_solve(int dim, const int *n, const double *len, double lam, double mu, const double *E,
             const double *macro, int pc, double lam_ref, double mu_ref, double void_value,
             double tol, int stop_mode, int maxit, const double *u0, double *u_out,
             double *sigma_bar, int *iters, double *relres_rec, double *relres_true,
             double *alpha_hist, double *beta_hist, double *res_hist, int hist_len,
             int remove_mean, double *timing, const double *f_in, int project_rhs,
             unsigned long long noise_seed, int dot_mode) {
  grid_t g;
  int st = grid_init(&g, dim, n, len);
  if (st) return st;
  if (!(tol > 0.0) || maxit < 0 || pc < PC_NONE || pc > PC_GREEN_JACOBI) return OR_E_INVALID;
  const long N = g.N;
  const int d = dim;
  const long nd = d * N;
  double t0 = now_s();
  for (long e = 0; e < N; ++e)
    if (!(E[e] >= 0.0) || !isfinite(E[e])) return OR_E_INVALID;
  if ((pc == PC_JACOBI || pc == PC_GREEN_JACOBI) && !all_even(&g)) return OR_E_ODD_GRID;

  double *f = (double *)malloc(sizeof(double) * nd);
  double *fabs_ = (double *)malloc(sizeof(double) * nd);
  double *r = (double *)malloc(sizeof(double) * nd);
  double *z = (double *)malloc(sizeof(double) * nd);
  double *p = (double *)malloc(sizeof(double) * nd);
  double *q = (double *)malloc(sizeof(double) * nd);
  double *diag = (double *)malloc(sizeof(double) * nd);
  double *Gre = NULL, *Gim = NULL;
  double complex *work = NULL;
  if (pc == PC_GREEN || pc == PC_GREEN_JACOBI) {
    Gre = (double *)malloc(sizeof(double) * d * d * N);
    Gim = (double *)malloc(sizeof(double) * d * d * N);
    work = (double complex *)malloc(sizeof(double complex) * 2 * nd);
  }
  if (!f || !fabs_ || !r || !z || !p || !q || !diag ||
      ((pc == PC_GREEN || pc == PC_GREEN_JACOBI) && (!Gre || !Gim || !work))) {
    st = OR_E_OOM;
    goto cleanup;
  }

  /* right-hand side; f is mean-free in exact arithmetic (the shape functions
     sum to one, so the columns of B^T sum to zero).  project_rhs removes the
     rounding-level mean per component; it is off by default because the
     projection writes rounding-level values into void dofs, where the void
     rule's replacement value would then amplify them (Sec. 3.2). */
  if (f_in) {
    /* caller-supplied right-hand side (used by the one-iteration test) */
    memcpy(f, f_in, sizeof(double) * nd);
    for (long i = 0; i < nd; ++i) fabs_[i] = fabs(f_in[i]);
  } else {
    or_rhs(dim, n, len, lam, mu, E, macro, f, fabs_);
  }
  if (project_rhs)
    for (int a = 0; a < d; ++a) {
      double m = 0.0;
      for (long i = 0; i < N; ++i) m += f[a * N + i];
      m /= (double)N;
      for (long i = 0; i < N; ++i) f[a * N + i] -= m;
    }
  double fnorm = sqrt(dotm(dot_mode, nd, f, f));
  double fabsnorm = sqrt(dotm(dot_mode, nd, fabs_, fabs_));

  /* preconditioner set-up */
  if (pc == PC_JACOBI || pc == PC_GREEN_JACOBI) {
    st = or_jacobi_diag(dim, n, len, lam, mu, E, diag, NULL);
    if (st) goto cleanup;
    void_rule(nd, diag, void_value);
  }
  if (pc == PC_GREEN || pc == PC_GREEN_JACOBI) {
    st = or_green(dim, n, len, lam_ref, mu_ref, Gre, Gim);
    if (st) goto cleanup;
  }
  double t1 = now_s();

  /* start vector */
  if (u0) {
    memcpy(u_out, u0, sizeof(double) * nd);
    stiffness_apply(&g, lam, mu, E, u_out, q);
    for (long i = 0; i < nd; ++i) r[i] = f[i] - q[i];
  } else {
    memset(u_out, 0, sizeof(double) * nd);
    memcpy(r, f, sizeof(double) * nd);
  }
  int k = 0;
  double rnorm = sqrt(dotm(dot_mode, nd, r, r));
  int converged;
  if (stop_mode == 0)
    converged = (fnorm <= 1e-13 * fabsnorm) || (rnorm <= tol * fnorm);
  else
    converged = (rnorm * rnorm <= tol);
  if (fnorm <= 1e-13 * fabsnorm) {
    /* homogeneous material: the exact fluctuation is zero */
    memset(u_out, 0, sizeof(double) * nd);
    rnorm = 0.0;
  }
  st = OR_OK;
  if (!converged) {
    st = precond_apply(&g, pc, diag, Gre, Gim, r, z, NULL, work);
    if (st) goto cleanup;
    if (noise_seed) ulp_noise(z, nd, noise_seed, 0, 1);
    memcpy(p, z, sizeof(double) * nd);
    double rz = dotm(dot_mode, nd, r, z);
    for (;;) {
      if (k >= maxit) {
        st = OR_E_NOT_CONVERGED;
        break;
      }
      stiffness_apply(&g, lam, mu, E, p, q);
      if (noise_seed) ulp_noise(q, nd, noise_seed, k + 1, 0);
      double pq = dotm(dot_mode, nd, p, q);
      double alpha = rz / pq;
      if (!(pq > 0.0) || !isfinite(alpha)) {
        st = OR_E_BREAKDOWN;
        break;
      }
      for (long i = 0; i < nd; ++i) u_out[i] += alpha * p[i];
      for (long i = 0; i < nd; ++i) r[i] -= alpha * q[i];
      ++k;
      rnorm = sqrt(dotm(dot_mode, nd, r, r));
      if (alpha_hist && k <= hist_len) alpha_hist[k - 1] = alpha;
      if (res_hist && k <= hist_len) res_hist[k - 1] = rnorm;
      if (stop_mode == 0 ? (rnorm <= tol * fnorm) : (rnorm * rnorm <= tol)) break;
      if (k >= maxit) {
        st = OR_E_NOT_CONVERGED;
        break;
      }
      st = precond_apply(&g, pc, diag, Gre, Gim, r, z, NULL, work);
      if (st) goto cleanup;
      if (noise_seed) ulp_noise(z, nd, noise_seed, k, 1);
      double rz_new = dotm(dot_mode, nd, r, z);
      double beta = rz_new / rz;
      if (!isfinite(beta)) {
        st = OR_E_BREAKDOWN;
        break;
      }
      if (beta_hist && k <= hist_len) beta_hist[k - 1] = beta;
      rz = rz_new;
      for (long i = 0; i < nd; ++i) p[i] = z[i] + beta * p[i];
    }
  }
  double t2 = now_s();
  if (iters) *iters = k;
  if (relres_rec) *relres_rec = (fnorm > 0.0) ? rnorm / fnorm : 0.0;

  /* true residual of the returned iterate */
  stiffness_apply(&g, lam, mu, E, u_out, q);
  for (long i = 0; i < nd; ++i) q[i] = f[i] - q[i];
  if (relres_true) *relres_true = (fnorm > 0.0) ? sqrt(dotm(dot_mode, nd, q, q)) / fnorm : 0.0;

  /* zero-mean fluctuation (Sec. 5 on mean shifts) and homogenised stress */
  if (remove_mean)
    for (int a = 0; a < d; ++a) {
      double m = 0.0;
      for (long i = 0; i < N; ++i) m += u_out[a * N + i];
      m /= (double)N;
      for (long i = 0; i < N; ++i) u_out[a * N + i] -= m;
    }
  if (sigma_bar) or_stress(dim, n, len, lam, mu, E, macro, u_out, NULL, sigma_bar);
  if (timing) {
    timing[0] = t1 - t0;
    timing[1] = t2 - t1;
    timing[2] = now_s() - t2;
  }

cleanup:
  free(f);
  free(fabs_);
  free(r);
  free(z);
  free(p);
  free(q);
  free(diag);
  free(Gre);
  free(Gim);
  free(work);
  return st;
}

/* One timed sample of the PCG loop body for the CPU baseline: given a grid,
   material and preconditioner, run set-up then exactly `iters` iterations of
   PCG from u0 = 0 (no stopping test), returning wall seconds of set-up and of
   the iterations.  Used to time the oracle on a bounded sample of a large
   workload. */
int or_time_iterations(int dim, const int *n, const double *len, double lam, double mu,
                       const double *E, const double *macro, int pc, double lam_ref,
                       double mu_ref, int iters, double *timing) {
  grid_t g;
  int st = grid_init(&g, dim, n, len);
  if (st) return st;
  const long N = g.N;
  const int d = dim;
  const long nd = d * N;
  double t0 = now_s();
  double *u = (double *)calloc(nd, sizeof(double));
  double *r = (double *)malloc(sizeof(double) * nd);
  double *z = (double *)malloc(sizeof(double) * nd);
  double *p = (double *)malloc(sizeof(double) * nd);
  double *q = (double *)malloc(sizeof(double) * nd);
  double *diag = (double *)malloc(sizeof(double) * nd);
  double *Gre = (double *)malloc(sizeof(double) * d * d * N);
  double *Gim = (double *)malloc(sizeof(double) * d * d * N);
  double complex *work = (double complex *)malloc(sizeof(double complex) * 2 * nd);
  if (!u || !r || !z || !p || !q || !diag || !Gre || !Gim || !work) {
    st = OR_E_OOM;
    goto out;
  }
  or_rhs(dim, n, len, lam, mu, E, macro, r, NULL);
  if (pc == PC_JACOBI || pc == PC_GREEN_JACOBI) {
    st = or_jacobi_diag(dim, n, len, lam, mu, E, diag, NULL);
    if (st) goto out;
    void_rule(nd, diag, 1.0);
  }
  if (pc == PC_GREEN || pc == PC_GREEN_JACOBI) {
    st = or_green(dim, n, len, lam_ref, mu_ref, Gre, Gim);
    if (st) goto out;
  }
  double t1 = now_s();
  st = precond_apply(&g, pc, diag, Gre, Gim, r, z, NULL, work);
  if (st) goto out;
  memcpy(p, z, sizeof(double) * nd);
  double rz = dot(nd, r, z);
  double t2 = now_s();
  for (int k = 0; k < iters; ++k) {
    stiffness_apply(&g, lam, mu, E, p, q);
    double alpha = rz / dot(nd, p, q);
    for (long i = 0; i < nd; ++i) u[i] += alpha * p[i];
    for (long i = 0; i < nd; ++i) r[i] -= alpha * q[i];
    (void)sqrt(dot(nd, r, r));
    st = precond_apply(&g, pc, diag, Gre, Gim, r, z, NULL, work);
    if (st) goto out;
    double rz_new = dot(nd, r, z);
    double beta = rz_new / rz;
    rz = rz_new;
    for (long i = 0; i < nd; ++i) p[i] = z[i] + beta * p[i];
  }
  double t3 = now_s();
  timing[0] = t1 - t0;
  timing[1] = t3 - t2;
  timing[2] = t2 - t1;
out:
  free(u);
  free(r);
  free(z);
  free(p);
  free(q);
  free(diag);
  free(Gre);
  free(Gim);
  free(work);
  return st;
}

int or_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
