// Matrix-free stiffness K = B^T W C(E) B for Q1 quads / hexes on a periodic
// grid (Sec. 2.1, eq. disc_wf and eq. lin_system_exp; matrix-free operator of
// Sec. 3.1).  Element data: u at the 2^d corners, strain at the 2^d Gauss
// points by sum factorisation (difference along the derivative axis,
// two-point interpolation along the others), isotropic stress
// sigma = E w (lambda tr(eps) I + 2 mu eps), and the transposed
// factorisation back to the corners.
//
// Kernels are halo-tiled: a block owns a tile of output nodes in the x-y
// plane (16 x 16 in 2D, 16 x 14 in 3D), evaluates every element that touches
// the tile (17 x 17, resp. 17 x 15, about 13% redundant halo work, no atomics,
// deterministic), keeps the node values of the input vector in LDS and sums
// the corner contributions of the four x-y neighbouring elements from LDS.
// The 3D kernel marches along z through a chunk of planes with a ring of node
// planes in LDS; the z neighbour's contribution is carried in registers to
// the next layer.
#pragma once
#include "jfft_common.h"

namespace jfft {

constexpr int TILE = 16;           // output nodes per tile edge
constexpr int ETILE = TILE + 1;    // elements per tile edge (with halo)
constexpr int NTILE = TILE + 2;    // nodes per tile edge (with halo)
constexpr int STENCIL_THREADS = 384;  // 6 wavefronts (2D kernel)
// Default shape of a 2D block (the tiles2d codes of the tunables: 1 = 16 x
// 16 output nodes, 2 = 16 wide x 32, 3 = 32 wide x 16, 4 = 32 x 32): in FP32
// one row of 32 x 16 (whole 128-byte rows; 5-7 % faster than 16 x 32 on the
// 512^2 groups, which beat 16 x 16 by 13 %), in FP64 16 x 16 (a larger FP64
// block's LDS cuts occupancy to 3 blocks per CU, 8 % slower).
template <typename Real>
constexpr int default_tiles2d() {
  return sizeof(Real) == 8 ? 1 : 3;
}
template <typename Real>
constexpr int ty2() {  // rows of the default block
  return TILE;
}
// 3D block shapes (the tiles3d codes of the tunables), both on four
// wavefronts.  Code 1: 16 x 14 output nodes, 17 x 15 elements, 18 x 16 node
// planes.  Code 2: 32 x 6 output nodes, 33 x 7 elements, 34 x 8
// node planes, so that a row of output nodes is one whole 128-byte line: a
// wavefront's load or store of a plane touches two whole lines instead of
// four halves, which more than pays for the larger halo (measured at 256^3:
// 0.44 ms per launch for code 1, 0.35 for code 2; a 32 x 10 block on six
// wavefronts took 0.51).  Rows start on 64-byte boundaries (code 1, FP32;
// 128 in FP64) or 128-byte ones (code 2), so every store covers whole
// sectors and no sector is written by two blocks.  A block has one thread
// per node of columns 1..TX of a node plane (TX x NY = threads) and at
// least one per element; columns 0 and NX - 1 are loaded by 2 NY further
// threads.
template <int SHAPE>
struct Geo3 {
  static constexpr int TX = SHAPE == 2 ? 32 : 16, TY = SHAPE == 2 ? 6 : 14;
  static constexpr int EX = TX + 1, EY = TY + 1;
  static constexpr int NX = TX + 2, NY = TY + 2;
  static constexpr int NELEM = EX * EY;  // 255 or 231
  static constexpr int NNODE = NX * NY;  // 288 or 272
  static constexpr int NT = TX * NY;     // 256 threads
  static constexpr int NSTRIP = NNODE - NT;
  static_assert(NSTRIP == 2 * NY && NELEM <= NT && NT == 256 && (TX & (TX - 1)) == 0,
                "four wavefronts: one thread per node of columns 1..TX, one per element");
};
constexpr int STENCIL3_THREADS = 256;
// Default 3D block shape of the precision.
template <typename Real>
constexpr int default_tiles3d() {
  return sizeof(Real) == 4 ? 2 : 1;
}
// Register budget of the 3D kernel (waves per SIMD = blocks per CU): three
// blocks per CU in FP32 (<= 168 VGPRs; at 128 it spills), one in FP64 (at
// 256 VGPRs it spills, which costs more than the second block gains).
// The power-law tangent (MAT = 1) holds two gradient sets: two blocks per CU
// in FP32, one in FP64.
template <typename Real, int MAT = 0>
constexpr int stencil3_waves_per_simd() {
  return MAT ? (sizeof(Real) == 4 ? 2 : 1) : (sizeof(Real) == 4 ? 3 : 1);
}

// Gauss-point interpolation weights of the linear shape functions:
// N_0(xi_g) = {A, B}, N_1(xi_g) = {B, A} for xi_g = 1/2 -+ 1/(2 sqrt 3).
template <typename Real>
__device__ __forceinline__ Real gA() { return (Real)0.78867513459481288225457439025098; }
template <typename Real>
__device__ __forceinline__ Real gB() { return (Real)0.21132486540518711774542560974902; }

// Two-point interpolation (and its transpose, the same matrix).
template <typename Real>
__device__ __forceinline__ void interp2(Real v0, Real v1, Real &o0, Real &o1) {
  o0 = gA<Real>() * v0 + gB<Real>() * v1;
  o1 = gB<Real>() * v0 + gA<Real>() * v1;
}

enum StencilMode { SM_APPLY = 0, SM_CG = 1, SM_COMB = 2 };

// Power-law matrix and linear inclusion of the nonlinear example (Sec. 4):
// matrix sigma = K tr(eps) I + g(eps_eq) e, g(s) = gcoef s^(n-1) with
// gcoef = sigma0 (2/3) / eps0^n, e = dev(eps), eps_eq = sqrt(2/3 e.e);
// inclusion sigma = Ki tr(eps) I + 2 mui e.  macro: the macroscopic strain
// (Mandel), added to the strain of the Newton iterate.
struct PowerLawArgs {
  double K, gcoef, n;
  double Ki, mui;
  double macro[6];
  int ipow;  // n - 1 when it is a whole number in [0, 64] (powers by squaring), else -1
};

// g = gcoef s^k and h = g k / (e.e) (k = n - 1, s = eps_eq, e.e = 1.5 s^2)
// from e.e.  A whole k takes products of s^2 (and one sqrt for odd k), and
// for k >= 2, h = (2/3) k gcoef s^(k-2) without a division; otherwise pow.
// g(0) = h(0) = 0 for n > 1.
template <typename Real>
__device__ __forceinline__ void powerlaw_gh(Real ee, const PowerLawArgs &m, Real &g, Real &h) {
  const Real s2 = (Real)(2.0 / 3.0) * ee, gc = (Real)m.gcoef;
  const int k = m.ipow;
  if (k == 0) {
    g = gc;
    h = (Real)0;
  } else if (k >= 2) {
    // t = s^(k - 2)
    Real t = (Real)1, b = s2;
    for (int e = (k - 2) >> 1; e; e >>= 1) {
      if (e & 1) t *= b;
      b *= b;
    }
    if (k & 1) t *= sqrt(s2);
    g = gc * t * s2;
    h = (Real)(2.0 / 3.0) * (Real)k * gc * t;
  } else {
    const Real s = sqrt(s2), kn = (Real)m.n - (Real)1;
    g = s > (Real)0 ? (k == 1 ? gc * s : gc * pow(s, kn)) : (Real)0;
    h = ee > (Real)0 ? g * kn / ee : (Real)0;
  }
}

template <typename Real>
struct StencilArgs {
  const Real *in;        // APPLY: vector to multiply; CG: p_old
  const Real *zin;       // CG: preconditioned residual z
  Real *pout;            // CG: p_new = z + beta p_old (owned nodes)
  Real *u;               // CG: u += alpha_prev * p_old (owned nodes)
  const Real *E;         // element moduli
  Real *out;             // q = K p (APPLY / CG)
  double *partial;       // CG: per-block partial of p_new . q
  const CgState *st;     // CG: scalars
  CgState *ctl;          // CG: the same state when the alpha step is fused (else NULL)
  History h;             // CG: history arrays of the fused step
  int parity;            // CG: buffer parity of p_new (fused alpha step)
  Real *diag;            // COMB: diag(K) output
  int comb_comp, comb_off;  // COMB: component and sub-grid offset bits (x, y, z)
  int tz;                // z planes per block (3D)
  int nbz;               // z blocks per cell (3D); gridDim.z = nbz * cells
  long long cs;          // bytes between the cells of a batch
  Real lam, mu;          // Lame constants of C^ times the Gauss weight
  Real ihx, ihy, ihz;
  Real clam[3], cmu[3];  // cubic elements: half of lam, mu times k_c^2 (see elem_hex_modes_cubic)
  int nx, ny, nz;
  long long N;
  // tangent of the power-law problem (power-law kernel variant only)
  const Real *uk;        // Newton iterate u^(i) [3][N]; E holds the phase (1 = matrix)
  PowerLawArgs pl;
  Real w;                // Gauss weight (element volume / 8)
};

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// XCD-aware tile order.  The dispatcher sends workgroup b to XCD b % 8; each
// XCD has its own L2.  Re-map b so that XCD k receives one contiguous range of
// logical tiles (x fastest), so neighbouring tiles, which share halo rows and
// cache lines, run on the same L2.  A bijection for any grid size.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_logical_block(int b, int total) {
  const int q = total / kNumXcd, r = total % kNumXcd;
  const int k = b % kNumXcd, j = b / kNumXcd;
  return k * q + min(k, r) + j;
}

template <typename Real>
__device__ __forceinline__ void shift_args(StencilArgs<Real> &a, int cell) {
  a.in = cshift(a.in, cell, a.cs);
  a.zin = cshift(a.zin, cell, a.cs);
  a.pout = cshift(a.pout, cell, a.cs);
  a.u = cshift(a.u, cell, a.cs);
  a.E = cshift(a.E, cell, a.cs);
  a.out = cshift(a.out, cell, a.cs);
  a.partial = cshift(a.partial, cell, a.cs);
  a.st = cshift(a.st, cell, a.cs);
  a.ctl = cshift(a.ctl, cell, a.cs);
  a.diag = cshift(a.diag, cell, a.cs);
}

// ----------------------------------------------------------------- 3D ----
// Strain pieces of one component from the 8 corner values (corner c = cx + 2 cy + 4 cz):
// dX[gy][gz] = d/dx at Gauss points (independent of gx), likewise dY[gx][gz], dZ[gx][gy].
template <typename Real>
__device__ __forceinline__ void grad_hex(const Real (&u)[8], Real ihx, Real ihy, Real ihz,
                                         Real (&dX)[2][2], Real (&dY)[2][2], Real (&dZ)[2][2]) {
  Real T[2][2];
  // x: differences at (cy, cz), interpolate along y then z
#pragma unroll
  for (int cz = 0; cz < 2; ++cz) {
    Real d0 = u[1 + 4 * cz] - u[0 + 4 * cz];
    Real d1 = u[3 + 4 * cz] - u[2 + 4 * cz];
    interp2(d0, d1, T[0][cz], T[1][cz]);  // T[gy][cz]
  }
#pragma unroll
  for (int gy = 0; gy < 2; ++gy) {
    Real o0, o1;
    interp2(T[gy][0], T[gy][1], o0, o1);
    dX[gy][0] = o0 * ihx;
    dX[gy][1] = o1 * ihx;
  }
  // y: differences at (cx, cz), interpolate along x then z
#pragma unroll
  for (int cz = 0; cz < 2; ++cz) {
    Real d0 = u[2 + 4 * cz] - u[0 + 4 * cz];
    Real d1 = u[3 + 4 * cz] - u[1 + 4 * cz];
    interp2(d0, d1, T[0][cz], T[1][cz]);  // T[gx][cz]
  }
#pragma unroll
  for (int gx = 0; gx < 2; ++gx) {
    Real o0, o1;
    interp2(T[gx][0], T[gx][1], o0, o1);
    dY[gx][0] = o0 * ihy;
    dY[gx][1] = o1 * ihy;
  }
  // z: differences at (cx, cy), interpolate along x then y
#pragma unroll
  for (int cy = 0; cy < 2; ++cy) {
    Real d0 = u[4 + 2 * cy] - u[0 + 2 * cy];
    Real d1 = u[5 + 2 * cy] - u[1 + 2 * cy];
    interp2(d0, d1, T[0][cy], T[1][cy]);  // T[gx][cy]
  }
#pragma unroll
  for (int gx = 0; gx < 2; ++gx) {
    Real o0, o1;
    interp2(T[gx][0], T[gx][1], o0, o1);
    dZ[gx][0] = o0 * ihz;
    dZ[gx][1] = o1 * ihz;
  }
}

// Transposed factorisation: corner forces of one component from the
// Gauss-point sums SX[gy][gz] = sum_gx sigma_ix, SY[gx][gz], SZ[gx][gy].
template <typename Real>
__device__ __forceinline__ void force_hex(const Real (&SX)[2][2], const Real (&SY)[2][2],
                                          const Real (&SZ)[2][2], Real ihx, Real ihy, Real ihz,
                                          Real (&y)[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) y[c] = (Real)0;
  Real U[2][2], R0, R1;
  // x part: interpolate^T along z then y, difference^T along x
#pragma unroll
  for (int gy = 0; gy < 2; ++gy) interp2(SX[gy][0], SX[gy][1], U[gy][0], U[gy][1]);  // U[gy][cz]
#pragma unroll
  for (int cz = 0; cz < 2; ++cz) {
    interp2(U[0][cz], U[1][cz], R0, R1);  // cy = 0, 1
    R0 *= ihx;
    R1 *= ihx;
    y[1 + 4 * cz] += R0;
    y[0 + 4 * cz] -= R0;
    y[3 + 4 * cz] += R1;
    y[2 + 4 * cz] -= R1;
  }
  // y part
#pragma unroll
  for (int gx = 0; gx < 2; ++gx) interp2(SY[gx][0], SY[gx][1], U[gx][0], U[gx][1]);  // U[gx][cz]
#pragma unroll
  for (int cz = 0; cz < 2; ++cz) {
    interp2(U[0][cz], U[1][cz], R0, R1);  // cx = 0, 1
    R0 *= ihy;
    R1 *= ihy;
    y[2 + 4 * cz] += R0;
    y[0 + 4 * cz] -= R0;
    y[3 + 4 * cz] += R1;
    y[1 + 4 * cz] -= R1;
  }
  // z part
#pragma unroll
  for (int gx = 0; gx < 2; ++gx) interp2(SZ[gx][0], SZ[gx][1], U[gx][0], U[gx][1]);  // U[gx][cy]
#pragma unroll
  for (int cy = 0; cy < 2; ++cy) {
    interp2(U[0][cy], U[1][cy], R0, R1);  // cx = 0, 1
    R0 *= ihz;
    R1 *= ihz;
    y[4 + 2 * cy] += R0;
    y[0 + 2 * cy] -= R0;
    y[5 + 2 * cy] += R1;
    y[1 + 2 * cy] -= R1;
  }
}

// Element force y = E w B^T C^ B u for a hex (lam, mu already carry w).
// With ENERGY, en += u . y = sum_q w sigma_q : eps_q (the element energy).
template <typename Real, bool ENERGY = false>
__device__ __forceinline__ void elem_hex(const Real (&u)[3][8], Real Elam, Real Emu, Real ihx,
                                         Real ihy, Real ihz, Real (&y)[3][8], double &en) {
  Real dX[3][2][2], dY[3][2][2], dZ[3][2][2];
#pragma unroll
  for (int i = 0; i < 3; ++i) grad_hex(u[i], ihx, ihy, ihz, dX[i], dY[i], dZ[i]);
  Real SX[3][2][2], SY[3][2][2], SZ[3][2][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) SX[i][a][b] = SY[i][a][b] = SZ[i][a][b] = (Real)0;
  const Real m2 = Emu + Emu;
#pragma unroll
  for (int gx = 0; gx < 2; ++gx)
#pragma unroll
    for (int gy = 0; gy < 2; ++gy)
#pragma unroll
      for (int gz = 0; gz < 2; ++gz) {
        const Real e11 = dX[0][gy][gz], e22 = dY[1][gx][gz], e33 = dZ[2][gx][gy];
        const Real g23 = dY[2][gx][gz] + dZ[1][gx][gy];
        const Real g13 = dX[2][gy][gz] + dZ[0][gx][gy];
        const Real g12 = dX[1][gy][gz] + dY[0][gx][gz];
        const Real lt = Elam * (e11 + e22 + e33);
        const Real s11 = lt + m2 * e11, s22 = lt + m2 * e22, s33 = lt + m2 * e33;
        const Real s23 = Emu * g23, s13 = Emu * g13, s12 = Emu * g12;
        if (ENERGY)
          en += (double)(s11 * e11 + s22 * e22 + s33 * e33 + s23 * g23 + s13 * g13 + s12 * g12);
        SX[0][gy][gz] += s11;
        SY[0][gx][gz] += s12;
        SZ[0][gx][gy] += s13;
        SX[1][gy][gz] += s12;
        SY[1][gx][gz] += s22;
        SZ[1][gx][gy] += s23;
        SX[2][gy][gz] += s13;
        SY[2][gx][gz] += s23;
        SZ[2][gx][gy] += s33;
      }
#pragma unroll
  for (int i = 0; i < 3; ++i) force_hex(SX[i], SY[i], SZ[i], ihx, ihy, ihz, y[i]);
}

// ---- hex element with the power-law tangent ---------------------------------
// Tangent of the law above at the strain eps of a Gauss point, applied to a
// strain increment d (both Mandel): for the matrix
//   C d = K tr(d) I + g dev(d) + h (e.d) e,  h = g (n - 1) / (e.e),
// (dg/ds = g (n-1)/s and d eps_eq = (2/3) e.d / eps_eq), for the inclusion
// C d = Ki tr(d) I + 2 mui dev(d); g(0) = 0 for n > 1.
template <typename Real>
__device__ __forceinline__ void powerlaw_tangent(const Real (&eps)[6], const Real (&d)[6],
                                                 bool matrix, const PowerLawArgs &m,
                                                 Real (&sg)[6]) {
  const Real dtr = d[0] + d[1] + d[2];
  if (matrix) {
    const Real tr3 = (eps[0] + eps[1] + eps[2]) / (Real)3;
    Real e[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) e[k] = eps[k] - (k < 3 ? tr3 : (Real)0);
    Real ee = 0, ed = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      ee += e[k] * e[k];
      ed += e[k] * d[k];
    }
    Real g, h;
    powerlaw_gh(ee, m, g, h);
    const Real kt = (Real)m.K * dtr, g3 = g * dtr / (Real)3, he = h * ed;
#pragma unroll
    for (int k = 0; k < 6; ++k) sg[k] = g * d[k] + he * e[k] + (k < 3 ? kt - g3 : (Real)0);
  } else {
    const Real m2 = (Real)(2.0 * m.mui), kt = (Real)m.Ki * dtr, m3 = m2 * dtr / (Real)3;
#pragma unroll
    for (int k = 0; k < 6; ++k) sg[k] = m2 * d[k] + (k < 3 ? kt - m3 : (Real)0);
  }
}

// Mandel strain at Gauss point (gx, gy, gz) from the factorised gradients.
template <typename Real>
__device__ __forceinline__ void mandel_strain(const Real (&X)[3][2][2], const Real (&Y)[3][2][2],
                                              const Real (&Z)[3][2][2], int gx, int gy, int gz,
                                              Real (&eps)[6]) {
  const Real r2 = (Real)0.70710678118654752440084436210485;  // 1/sqrt2
  eps[0] = X[0][gy][gz];
  eps[1] = Y[1][gx][gz];
  eps[2] = Z[2][gx][gy];
  eps[3] = (Y[2][gx][gz] + Z[1][gx][gy]) * r2;  // 23
  eps[4] = (X[2][gy][gz] + Z[0][gx][gy]) * r2;  // 13
  eps[5] = (X[1][gy][gz] + Y[0][gx][gz]) * r2;  // 12
}

// Element force y = w B^T C(E + B uk) B u of the power-law tangent at the
// Newton iterate uk (Gauss-point loop on the factorised gradients).  With
// ENERGY, en += u . y.
template <typename Real, bool ENERGY>
__device__ __forceinline__ void elem_hex_tangent(const Real (&uk)[3][8], const Real (&u)[3][8],
                                                 bool matrix, const PowerLawArgs &m, Real w,
                                                 Real ihx, Real ihy, Real ihz, Real (&y)[3][8],
                                                 double &en) {
  Real kX[3][2][2], kY[3][2][2], kZ[3][2][2];
  Real dX[3][2][2], dY[3][2][2], dZ[3][2][2];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    grad_hex(uk[i], ihx, ihy, ihz, kX[i], kY[i], kZ[i]);
    grad_hex(u[i], ihx, ihy, ihz, dX[i], dY[i], dZ[i]);
  }
  Real SX[3][2][2], SY[3][2][2], SZ[3][2][2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) SX[i][a][b] = SY[i][a][b] = SZ[i][a][b] = (Real)0;
  const Real r2 = (Real)0.70710678118654752440084436210485;
  Real e = 0;
#pragma unroll
  for (int gx = 0; gx < 2; ++gx)
#pragma unroll
    for (int gy = 0; gy < 2; ++gy)
#pragma unroll
      for (int gz = 0; gz < 2; ++gz) {
        Real es[6], de[6], sg[6];
        mandel_strain(kX, kY, kZ, gx, gy, gz, es);
#pragma unroll
        for (int k = 0; k < 6; ++k) es[k] += (Real)m.macro[k];
        mandel_strain(dX, dY, dZ, gx, gy, gz, de);
        powerlaw_tangent(es, de, matrix, m, sg);
#pragma unroll
        for (int k = 0; k < 6; ++k) sg[k] *= w;
        if (ENERGY) {
#pragma unroll
          for (int k = 0; k < 6; ++k) e += sg[k] * de[k];
        }
        const Real s23 = sg[3] * r2, s13 = sg[4] * r2, s12 = sg[5] * r2;
        SX[0][gy][gz] += sg[0];
        SY[0][gx][gz] += s12;
        SZ[0][gx][gy] += s13;
        SX[1][gy][gz] += s12;
        SY[1][gx][gz] += sg[1];
        SZ[1][gx][gy] += s23;
        SX[2][gy][gz] += s13;
        SY[2][gx][gz] += s23;
        SZ[2][gx][gy] += sg[2];
      }
#pragma unroll
  for (int i = 0; i < 3; ++i) force_hex(SX[i], SY[i], SZ[i], ihx, ihy, ihz, y[i]);
  if (ENERGY) en += (double)e;
}

// ---- hex element in Hadamard modes of the Gauss points -------------------
// The two-point interpolation matrix of the linear shape functions at the
// Gauss points is M = (1/2) H diag(1, 1/sqrt3) H with H = [[1, 1], [1, -1]].
// Writing Gauss-point fields in the Hadamard basis of the 2 x 2 x 2 points
// (mode m in {0,1}^3) makes the strain and force steps cheap:
//   * d/dx u_i lives on the modes with m_x = 0 only (it is constant in x_g),
//     its four mode values are H2(u[1,:,:] - u[0,:,:]) scaled by s^|m| / h_x;
//   * the isotropic stress is the same linear map in every mode;
//   * the x force on corner c is sign(c_x) / h_x times H2 of the m_x = 0
//     stress modes scaled by s^|m|, and likewise for y and z;
// with s = 1/sqrt3.  Only the stress modes the forces use are formed.  The
// element energy u.y = sum_q w sigma:eps is the sum of stress times strain
// modes.  Same operator as grad_hex / force_hex, about 40% fewer operations.

// h[m1][m2] = sum_{a,b} (-1)^(a m1 + b m2) v[a][b]
template <typename Real>
__device__ __forceinline__ void had2(Real v00, Real v01, Real v10, Real v11, Real (&h)[2][2]) {
  const Real p0 = v00 + v10, p1 = v01 + v11, d0 = v00 - v10, d1 = v01 - v11;
  h[0][0] = p0 + p1;
  h[0][1] = p0 - p1;
  h[1][0] = d0 + d1;
  h[1][1] = d0 - d1;
}

// lam, mu: Lame constants times E_e and half the Gauss weight.
template <typename Real, bool ENERGY>
__device__ __forceinline__ void elem_hex_modes(const Real (&u)[3][8], Real lam, Real mu,
                                               Real ihx, Real ihy, Real ihz, Real (&y)[3][8],
                                               double &en) {
  const Real s1 = (Real)0.57735026918962576450914878050196;  // 1/sqrt3
  const Real s2 = (Real)(1.0 / 3.0);
  // strain modes: X[i][my][mz] = d_x u_i, Y[i][mx][mz] = d_y u_i, Z[i][mx][my] = d_z u_i
  Real X[3][2][2], Y[3][2][2], Z[3][2][2];
  const Real kx[3] = {ihx, s1 * ihx, s2 * ihx};
  const Real ky[3] = {ihy, s1 * ihy, s2 * ihy};
  const Real kz[3] = {ihz, s1 * ihz, s2 * ihz};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const Real *v = u[i];
    Real h[2][2];
    had2(v[1] - v[0], v[5] - v[4], v[3] - v[2], v[7] - v[6], h);  // D[cy][cz]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) X[i][a][b] = h[a][b] * kx[a + b];
    had2(v[2] - v[0], v[6] - v[4], v[3] - v[1], v[7] - v[5], h);  // D[cx][cz]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) Y[i][a][b] = h[a][b] * ky[a + b];
    had2(v[4] - v[0], v[6] - v[2], v[5] - v[1], v[7] - v[3], h);  // D[cx][cy]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) Z[i][a][b] = h[a][b] * kz[a + b];
  }
  const Real m2 = mu + mu;
  Real e = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 8; ++c) y[i][c] = (Real)0;
  // One family of modes at a time: the x family (modes with m_x = 0) carries
  // the stresses sigma_1j that the x forces of all three components need, etc.
  // x family: modes (0, my = a, mz = b)
  {
    Real S[3][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const Real tr = X[0][a][b] + (a == 0 ? Y[1][0][b] : (Real)0) + (b == 0 ? Z[2][0][a] : (Real)0);
        const Real g12 = X[1][a][b] + (a == 0 ? Y[0][0][b] : (Real)0);
        const Real g13 = X[2][a][b] + (b == 0 ? Z[0][0][a] : (Real)0);
        S[0][a][b] = lam * tr + m2 * X[0][a][b];
        S[1][a][b] = mu * g12;
        S[2][a][b] = mu * g13;
        if (ENERGY) e += S[0][a][b] * X[0][a][b] + S[1][a][b] * g12 + S[2][a][b] * g13;
      }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Real R[2][2];  // R[cy][cz]
      had2(S[i][0][0] * kx[0], S[i][0][1] * kx[1], S[i][1][0] * kx[1], S[i][1][1] * kx[2], R);
      y[i][1] += R[0][0];
      y[i][0] -= R[0][0];
      y[i][5] += R[0][1];
      y[i][4] -= R[0][1];
      y[i][3] += R[1][0];
      y[i][2] -= R[1][0];
      y[i][7] += R[1][1];
      y[i][6] -= R[1][1];
    }
  }
  // y family: modes (mx = a, 0, mz = b); components sigma_21, sigma_22, sigma_23
  {
    Real S[3][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const Real tr = Y[1][a][b] + (a == 0 ? X[0][0][b] : (Real)0) + (b == 0 ? Z[2][a][0] : (Real)0);
        const Real g12 = Y[0][a][b] + (a == 0 ? X[1][0][b] : (Real)0);
        const Real g23 = Y[2][a][b] + (b == 0 ? Z[1][a][0] : (Real)0);
        S[0][a][b] = mu * g12;
        S[1][a][b] = lam * tr + m2 * Y[1][a][b];
        S[2][a][b] = mu * g23;
        if (ENERGY) {
          e += S[1][a][b] * Y[1][a][b] + S[2][a][b] * g23;
          if (a == 1) e += S[0][a][b] * g12;  // modes (1, 0, mz); (0, 0, mz) counted in x
        }
      }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Real R[2][2];  // R[cx][cz]
      had2(S[i][0][0] * ky[0], S[i][0][1] * ky[1], S[i][1][0] * ky[1], S[i][1][1] * ky[2], R);
      y[i][2] += R[0][0];
      y[i][0] -= R[0][0];
      y[i][6] += R[0][1];
      y[i][4] -= R[0][1];
      y[i][3] += R[1][0];
      y[i][1] -= R[1][0];
      y[i][7] += R[1][1];
      y[i][5] -= R[1][1];
    }
  }
  // z family: modes (mx = a, my = b, 0); components sigma_31, sigma_32, sigma_33
  {
    Real S[3][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const Real tr = Z[2][a][b] + (a == 0 ? X[0][b][0] : (Real)0) + (b == 0 ? Y[1][a][0] : (Real)0);
        const Real g13 = Z[0][a][b] + (a == 0 ? X[2][b][0] : (Real)0);
        const Real g23 = Z[1][a][b] + (b == 0 ? Y[2][a][0] : (Real)0);
        S[0][a][b] = mu * g13;
        S[1][a][b] = mu * g23;
        S[2][a][b] = lam * tr + m2 * Z[2][a][b];
        if (ENERGY) {
          e += S[2][a][b] * Z[2][a][b];
          if (a == 1) e += S[0][a][b] * g13;  // modes (1, my, 0); (0, my, 0) counted in x
          if (b == 1) e += S[1][a][b] * g23;  // modes (mx, 1, 0); (mx, 0, 0) counted in y
        }
      }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Real R[2][2];  // R[cx][cy]
      had2(S[i][0][0] * kz[0], S[i][0][1] * kz[1], S[i][1][0] * kz[1], S[i][1][1] * kz[2], R);
      y[i][4] += R[0][0];
      y[i][0] -= R[0][0];
      y[i][6] += R[0][1];
      y[i][2] -= R[0][1];
      y[i][5] += R[1][0];
      y[i][1] -= R[1][0];
      y[i][7] += R[1][1];
      y[i][3] -= R[1][1];
    }
  }
  if (ENERGY) en += (double)e;
}

// Cubic elements (h_x = h_y = h_z = h): every term of strain mode m carries
// the same factor k_|m| = s^|m| / h, so the stress of mode m is k_|m| times
// the stress of the unscaled modes and the forces take k_|m|^2 times it.
// Folding k_|m|^2 into the Lame constants of each class |m| = 0, 1, 2
// (clam[c] = lam k_c^2, cmu[c] = mu k_c^2, without E_e) leaves no scaling
// multiply: the unscaled difference modes go in, forces come out, and the
// element energy is the sum of the folded stress times the unscaled strain.
// Same operator as elem_hex_modes on cubic elements.
template <typename Real, bool ENERGY>
__device__ __forceinline__ void stress_force_cubic(const Real (&X)[3][2][2],
                                                   const Real (&Y)[3][2][2],
                                                   const Real (&Z)[3][2][2], Real Ee,
                                                   const Real (&clam)[3], const Real (&cmu)[3],
                                                   Real (&y)[3][8], double &en);

template <typename Real, bool ENERGY>
__device__ __forceinline__ void elem_hex_modes_cubic(const Real (&u)[3][8], Real Ee,
                                                     const Real (&clam)[3], const Real (&cmu)[3],
                                                     Real (&y)[3][8], double &en) {
  // strain modes (unscaled): X[i][my][mz] = d_x u_i, Y[i][mx][mz], Z[i][mx][my]
  Real X[3][2][2], Y[3][2][2], Z[3][2][2];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const Real *v = u[i];
    Real h[2][2];
    had2(v[1] - v[0], v[5] - v[4], v[3] - v[2], v[7] - v[6], h);  // D[cy][cz]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) X[i][a][b] = h[a][b];
    had2(v[2] - v[0], v[6] - v[4], v[3] - v[1], v[7] - v[5], h);  // D[cx][cz]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) Y[i][a][b] = h[a][b];
    had2(v[4] - v[0], v[6] - v[2], v[5] - v[1], v[7] - v[3], h);  // D[cx][cy]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) Z[i][a][b] = h[a][b];
  }
  stress_force_cubic<Real, ENERGY>(X, Y, Z, Ee, clam, cmu, y, en);
}

// In-plane differences of one element face (4 nodes, index cx + 2 cy), per
// component: F[0] = sum over cy of the x differences, F[1] = their
// difference (cy = 0 minus cy = 1), F[2], F[3] the same for the y
// differences over cx.  The x and y strain modes of an element are
// X[my][mz] = F_bottom[my] +- F_top[my] (sign (-1)^mz) and likewise for y,
// so an element column marching in z reuses its top face's F as the next
// element's bottom face.
template <typename Real>
__device__ __forceinline__ void face_diffs(const Real (&v)[4], Real (&F)[4]) {
  const Real x0 = v[1] - v[0], x1 = v[3] - v[2];
  const Real y0 = v[2] - v[0], y1 = v[3] - v[1];
  F[0] = x0 + x1;
  F[1] = x0 - x1;
  F[2] = y0 + y1;
  F[3] = y0 - y1;
}

// elem_hex_modes_cubic with the bottom face given by its node values and
// in-plane differences (carried from the element below) and the top face by
// its node values; returns the top face's differences for the next element.
template <typename Real, bool ENERGY>
__device__ __forceinline__ void elem_hex_modes_cubic_faces(const Real (&bot)[3][4],
                                                           const Real (&botF)[3][4],
                                                           const Real (&top)[3][4],
                                                           Real (&topF)[3][4], Real Ee,
                                                           const Real (&clam)[3],
                                                           const Real (&cmu)[3],
                                                           Real (&y)[3][8], double &en) {
  Real X[3][2][2], Y[3][2][2], Z[3][2][2];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    face_diffs(top[i], topF[i]);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      X[i][a][0] = botF[i][a] + topF[i][a];
      X[i][a][1] = botF[i][a] - topF[i][a];
      Y[i][a][0] = botF[i][2 + a] + topF[i][2 + a];
      Y[i][a][1] = botF[i][2 + a] - topF[i][2 + a];
    }
    Real h[2][2];
    had2(top[i][0] - bot[i][0], top[i][2] - bot[i][2], top[i][1] - bot[i][1],
         top[i][3] - bot[i][3], h);  // D[cx][cy]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) Z[i][a][b] = h[a][b];
  }
  stress_force_cubic<Real, ENERGY>(X, Y, Z, Ee, clam, cmu, y, en);
}

template <typename Real, bool ENERGY>
__device__ __forceinline__ void stress_force_cubic(const Real (&X)[3][2][2],
                                                   const Real (&Y)[3][2][2],
                                                   const Real (&Z)[3][2][2], Real Ee,
                                                   const Real (&clam)[3], const Real (&cmu)[3],
                                                   Real (&y)[3][8], double &en) {
  Real lc[3], mc[3], m2c[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lc[c] = Ee * clam[c];
    mc[c] = Ee * cmu[c];
    m2c[c] = mc[c] + mc[c];
  }
  Real e = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 8; ++c) y[i][c] = (Real)0;
  // One family of modes at a time: the x family (modes with m_x = 0) carries
  // the stresses sigma_1j that the x forces of all three components need, etc.
  // x family: modes (0, my = a, mz = b)
  {
    Real S[3][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const Real tr = X[0][a][b] + (a == 0 ? Y[1][0][b] : (Real)0) + (b == 0 ? Z[2][0][a] : (Real)0);
        const Real g12 = X[1][a][b] + (a == 0 ? Y[0][0][b] : (Real)0);
        const Real g13 = X[2][a][b] + (b == 0 ? Z[0][0][a] : (Real)0);
        S[0][a][b] = lc[a + b] * tr + m2c[a + b] * X[0][a][b];
        S[1][a][b] = mc[a + b] * g12;
        S[2][a][b] = mc[a + b] * g13;
        if (ENERGY) e += S[0][a][b] * X[0][a][b] + S[1][a][b] * g12 + S[2][a][b] * g13;
      }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Real R[2][2];  // R[cy][cz]
      had2(S[i][0][0], S[i][0][1], S[i][1][0], S[i][1][1], R);
      y[i][1] += R[0][0];
      y[i][0] -= R[0][0];
      y[i][5] += R[0][1];
      y[i][4] -= R[0][1];
      y[i][3] += R[1][0];
      y[i][2] -= R[1][0];
      y[i][7] += R[1][1];
      y[i][6] -= R[1][1];
    }
  }
  // y family: modes (mx = a, 0, mz = b); components sigma_21, sigma_22, sigma_23
  {
    Real S[3][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const Real tr = Y[1][a][b] + (a == 0 ? X[0][0][b] : (Real)0) + (b == 0 ? Z[2][a][0] : (Real)0);
        const Real g12 = Y[0][a][b] + (a == 0 ? X[1][0][b] : (Real)0);
        const Real g23 = Y[2][a][b] + (b == 0 ? Z[1][a][0] : (Real)0);
        S[0][a][b] = mc[a + b] * g12;
        S[1][a][b] = lc[a + b] * tr + m2c[a + b] * Y[1][a][b];
        S[2][a][b] = mc[a + b] * g23;
        if (ENERGY) {
          e += S[1][a][b] * Y[1][a][b] + S[2][a][b] * g23;
          if (a == 1) e += S[0][a][b] * g12;  // modes (1, 0, mz); (0, 0, mz) counted in x
        }
      }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Real R[2][2];  // R[cx][cz]
      had2(S[i][0][0], S[i][0][1], S[i][1][0], S[i][1][1], R);
      y[i][2] += R[0][0];
      y[i][0] -= R[0][0];
      y[i][6] += R[0][1];
      y[i][4] -= R[0][1];
      y[i][3] += R[1][0];
      y[i][1] -= R[1][0];
      y[i][7] += R[1][1];
      y[i][5] -= R[1][1];
    }
  }
  // z family: modes (mx = a, my = b, 0); components sigma_31, sigma_32, sigma_33
  {
    Real S[3][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const Real tr = Z[2][a][b] + (a == 0 ? X[0][b][0] : (Real)0) + (b == 0 ? Y[1][a][0] : (Real)0);
        const Real g13 = Z[0][a][b] + (a == 0 ? X[2][b][0] : (Real)0);
        const Real g23 = Z[1][a][b] + (b == 0 ? Y[2][a][0] : (Real)0);
        S[0][a][b] = mc[a + b] * g13;
        S[1][a][b] = mc[a + b] * g23;
        S[2][a][b] = lc[a + b] * tr + m2c[a + b] * Z[2][a][b];
        if (ENERGY) {
          e += S[2][a][b] * Z[2][a][b];
          if (a == 1) e += S[0][a][b] * g13;  // modes (1, my, 0); (0, my, 0) counted in x
          if (b == 1) e += S[1][a][b] * g23;  // modes (mx, 1, 0); (mx, 0, 0) counted in y
        }
      }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Real R[2][2];  // R[cx][cy]
      had2(S[i][0][0], S[i][0][1], S[i][1][0], S[i][1][1], R);
      y[i][4] += R[0][0];
      y[i][0] -= R[0][0];
      y[i][6] += R[0][1];
      y[i][2] -= R[0][1];
      y[i][5] += R[1][0];
      y[i][1] -= R[1][0];
      y[i][7] += R[1][1];
      y[i][3] -= R[1][1];
    }
  }
  if (ENERGY) en += (double)e;
}

// Block reduction of one double per thread; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sm) {
  // wavefront reduction (fixed order), then across wavefronts in LDS
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (NT + 63) / 64; ++i) r += sm[i];
  }
  return r;
}

// ------------------------------------------------------ CG control steps
// The scalar steps of a PCG iteration (Sec. 3.3): alpha after p.q, the
// update count and stopping test after ||r||^2, beta after r.z.  Run by
// thread 0 of a single-block control kernel (cg.h), or fused into the
// kernel that produces the step's partial sums: every block of a cell
// writes its partial, makes it visible (device-scope fence) and counts its
// arrival on the cell's counter; the block that arrives last (fence again)
// sums the partials in a fixed order, runs the step and resets the counter.
// Which block is last does not change the result.

// alpha_k = (r.z) / (p.q); breakdown if p.q <= 0 or alpha not finite.
// parity: which of the two search-direction buffers holds p_k.
__device__ __forceinline__ void cg_alpha_step(CgState *st, double pq, const History &h, int parity) {
  st->pq = pq;
  st->parity = parity;
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

// ||r_{k+1}||^2; count the update of u; stop on tolerance or maxit.
__device__ __forceinline__ void cg_rr_step(CgState *st, double rr, const History &h) {
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
  // the last iteration forms no beta: its history entry is NaN
  if (st->done && h.beta && st->iter - 1 < st->hist_cap) h.beta[st->iter - 1] = __builtin_nan("");
}

// beta_k = (r.z)_new / (r.z)_old.
__device__ __forceinline__ void cg_beta_step(CgState *st, double rz, const History &h) {
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

// Fixed-order sum of n partials by the NT threads of a block (thread 0
// gets the result).
template <int NT>
__device__ __forceinline__ double block_fixed_sum(const double *p, long long n, double *sm) {
  double v = 0.0;
  long long i = threadIdx.x;
  for (; i + 7LL * NT < n; i += 8LL * NT) {
    double t[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) t[k] = p[i + (long long)k * NT];
#pragma unroll
    for (int k = 0; k < 8; ++k) v += t[k];
  }
  for (; i < n; i += NT) v += p[i];
  return block_sum<NT>(v, sm);
}

enum CtrlStep { CTRL_ALPHA = 0, CTRL_RR = 1, CTRL_BETA = 2 };

// Called by every thread of every block of the cell after thread 0 stored
// the block's partial: the last block to arrive sums the `total` partials
// and runs the step.
template <int NT, int STEP>
__device__ __forceinline__ void fused_ctrl(CgState *st, const double *part, int total,
                                           History h, int cell, long long cs, int parity,
                                           double *sm) {
  __shared__ int last;
  if (threadIdx.x == 0) {
    __threadfence();  // this block's partial before its arrival
    last = atomicAdd(&st->arrive[STEP], 1) == total - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();  // every other block's partial before the sum
  const double v = block_fixed_sum<NT>(part, total, sm);
  if (threadIdx.x == 0) {
    shift_hist(h, cell, cs);
    if (STEP == CTRL_ALPHA) cg_alpha_step(st, v, h, parity);
    if (STEP == CTRL_RR) cg_rr_step(st, v, h);
    if (STEP == CTRL_BETA) cg_beta_step(st, v, h);
    st->arrive[STEP] = 0;
  }
}

// Software-pipelined layer march: while the elements of layer ez are
// evaluated from node planes ez and ez + 1 (LDS), the global loads of plane
// ez + 2 and of the next element moduli are in flight in registers; they are
// committed to the third slot of the plane ring after the element work.  Two
// barriers per layer.  In CG mode p.q is accumulated as the element energies
// u_e . K_e u_e of the elements the block owns (= p^T K p).
//
// Geometry (Geo3<SHAPE>): a block owns TX x TY output nodes and evaluates
// the EX x EY elements that touch them, one element per thread (threads past
// the last element repeat it and discard it).  A block is exactly four
// wavefronts: one per SIMD, and every SIMD of a CU carries the same element
// work at any occupancy.  Thread t also
// holds node (t % TX) + 1, t / TX of each NX x NY node plane (columns 1..TX,
// which hold every owned node) and, if t < TX TY, output node (t % TX) + 1,
// t / TX + 1.  Columns 0 and NX - 1 of a plane are loaded by threads
// 0 .. 2 NY - 1.
// MAT = 1: the tangent of the power-law problem at the Newton iterate a.uk
// (E holds the phase); a second ring of node planes holds the iterate.
template <typename Real, int MODE, bool CUBIC = false, int MAT = 0, int SHAPE = 1>
__global__ void __launch_bounds__(Geo3<SHAPE>::NT, (stencil3_waves_per_simd<Real, MAT>()))
    k_stiffness3d(StencilArgs<Real> a) {
  using G = Geo3<SHAPE>;
  constexpr int NT = G::NT, TX = G::TX, TY = G::TY, EX = G::EX, NX = G::NX, NY = G::NY;
  __shared__ Real P[3][3][G::NNODE];               // ring of three node planes of the input vector
  __shared__ Real U[MAT ? 3 : 1][3][MAT ? G::NNODE : 1];  // MAT: ring of the Newton iterate
  __shared__ Real Y[24][NT];                       // corner contributions of one element layer
  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  const int nbx = gridDim.x, nby = gridDim.y;
  const int per_cell = nbx * nby * a.nbz;
  const int lbg = xcd_logical_block(blockIdx.x + nbx * (blockIdx.y + nby * blockIdx.z),
                                    nbx * nby * gridDim.z);
  const int cell = lbg / per_cell;
  const int lb = lbg - cell * per_cell;
  shift_args(a, cell);
  if (MODE == SM_CG && a.st->done) return;
  const int bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
  const int x0 = bx * TX, y0 = by * TY;
  const int z0 = bz * a.tz;
  const int zend = min(z0 + a.tz, a.nz);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long N = a.N;
  // Addresses: a uniform base per array and component, held in scalar
  // registers, plus a 32-bit byte offset per node (a cell holds at most
  // 512^3 nodes, so offsets stay below 2^32 even in FP64): every access is a
  // scalar-base load or store with one vector offset shared by the arrays,
  // instead of a 64-bit address per array and component.  The empty asm
  // keeps each base opaque, so that the compiler does not fold the component
  // stride back into the vector address.
  const unsigned uplane = (unsigned)nx * (unsigned)ny;
  typedef __attribute__((address_space(1))) char gchar;  // global memory
  struct Bases {
    gchar *p[3];
  };
  auto bases = [&](const Real *p) {
    Bases b;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gchar *q = (gchar *)(const_cast<Real *>(p) + (long long)c * N);
      asm volatile("" : "+s"(q));
      b.p[c] = q;
    }
    return b;
  };
  auto ld = [&](const Bases &b, int c, unsigned off) -> Real {
    return *reinterpret_cast<const __attribute__((address_space(1))) Real *>(b.p[c] + off);
  };
  auto st = [&](const Bases &b, int c, unsigned off, Real v) {
    __builtin_nontemporal_store(v, reinterpret_cast<__attribute__((address_space(1))) Real *>(b.p[c] + off));
  };

  bool first = false;
  Real beta = 0, alpha_prev = 0;
  if (MODE == SM_CG) {
    first = a.st->first != 0;
    beta = (Real)a.st->beta;
    alpha_prev = (Real)a.st->alpha;
  }

  // element (halo-extended layer; beyond the grid: E = 0)
  const int te = min(tid, G::NELEM - 1);
  const int exl = te % EX, eyl = te / EX;
  const int gex = x0 - 1 + exl, gey = y0 - 1 + eyl;
  const bool elem_valid = gex < nx && gey < ny;
  const bool elem_owned = elem_valid && exl >= 1 && eyl >= 1 && tid < G::NELEM;
  const unsigned exy_b = ((unsigned)wrapi(gex, nx) + (unsigned)nx * (unsigned)wrapi(gey, ny)) *
                        (unsigned)sizeof(Real);
  const int lie = eyl * NX + exl;  // corner (0, 0) of the element in a node plane
  // output node (ox + 1, oy + 1); its x-y neighbouring elements are e00,
  // e00 + 1, e00 + EX and e00 + EX + 1
  const int ox = tid % TX, oy = tid / TX;
  const int e00 = oy * EX + ox;
  const int gnx = x0 + ox, gny = y0 + oy;
  const bool node_valid = oy < TY && gnx < nx && gny < ny;
  // node slot 0: node (ox + 1, oy) of the plane, global (x0 + ox, y0 - 1 + oy)
  const int li0 = oy * NX + ox + 1;
  const int w0x = wrapi(x0 + ox, nx), w0y = wrapi(y0 - 1 + oy, ny);
  const unsigned n0xy = (unsigned)w0x + (unsigned)nx * (unsigned)w0y;
  const bool own0 = oy >= 1 && oy <= TY && x0 + ox < nx && y0 - 1 + oy < ny;
  const int par0 = (w0x & 1) | ((w0y & 1) << 1);
  // u is read for every slot-0 node (so that the loads need no branch); a
  // halo row reads its owned neighbour row instead, and discards the value
  const unsigned u0xy =
      (unsigned)w0x + (unsigned)nx * (unsigned)wrapi(y0 - 1 + min(max(oy, 1), TY), ny);
  // node slot 1 (threads 0 .. 2 NY - 1): column 0, then column NX - 1; the
  // other threads load node (0, 0) again (one cache line per wavefront) and
  // discard it
  const bool has1 = tid < G::NSTRIP;
  const int s1x = (has1 && tid >= NY) ? NX - 1 : 0;
  const int s1y = has1 ? tid % NY : 0;
  const int li1 = s1y * NX + s1x;
  const int w1x = wrapi(x0 - 1 + s1x, nx), w1y = wrapi(y0 - 1 + s1y, ny);
  const unsigned n1xy = (unsigned)w1x + (unsigned)nx * (unsigned)w1y;
  const int par1 = (w1x & 1) | ((w1y & 1) << 1);

  // One prefetched plane in registers (z or the APPLY input, p_old and u
  // for slot 0; z and p_old for slot 1), committed at the top of the next
  // layer.  Slot 0 is refilled right after its commit; slot 1 only after the
  // element work, so that its registers are free while the element is
  // evaluated (its loads then hide behind the node sums).  Every load is
  // issued unconditionally at a valid address and masked at the commit: with
  // no load under a branch the compiler knows the exact number of memory
  // operations in flight and waits only for the ones a value needs.
  const Bases b_in = bases(a.in), b_zin = bases(MODE == SM_CG ? a.zin : a.in);
  const Bases b_u = bases(MODE == SM_CG ? a.u : a.in), b_pout = bases(MODE == SM_CG ? a.pout : a.in);
  const Bases b_out = bases(MODE == SM_COMB ? a.in : a.out), b_uk = bases(MAT ? a.uk : a.in);
  const Bases b_E = bases(a.E);
  Real fz[3], fp[3], fu[3], hz[3], hp[3], ku[3], kh[3];
  auto fetch0 = [&](int zp) {
    const unsigned o0 = ((unsigned)wrapi(zp, nz) * uplane + n0xy) * (unsigned)sizeof(Real);
    // owned u lies in planes z0 .. zend - 1 (< nz, no wrap)
    const unsigned ou =
        ((unsigned)min(max(zp, z0), zend - 1) * uplane + u0xy) * (unsigned)sizeof(Real);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (MODE == SM_APPLY) {
        fz[c] = ld(b_in, c, o0);
      } else if (MODE == SM_CG) {
        fz[c] = ld(b_zin, c, o0);
        fp[c] = ld(b_in, c, o0);
        fu[c] = ld(b_u, c, ou);
      }
      if (MAT) ku[c] = ld(b_uk, c, o0);
    }
  };
  auto fetch1 = [&](int zp) {
    const unsigned o1 = ((unsigned)wrapi(zp, nz) * uplane + n1xy) * (unsigned)sizeof(Real);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (MODE == SM_APPLY) {
        hz[c] = ld(b_in, c, o1);
      } else if (MODE == SM_CG) {
        hz[c] = ld(b_zin, c, o1);
        hp[c] = ld(b_in, c, o1);
      }
      if (MAT) kh[c] = ld(b_uk, c, o1);
    }
  };
  auto fetch = [&](int zp) {
    fetch0(zp);
    fetch1(zp);
  };
  auto commit = [&](int zp, int slot) {
    const int wz = wrapi(zp, nz);
    const unsigned o0 = ((unsigned)wz * uplane + n0xy) * (unsigned)sizeof(Real);
    const bool owned = (zp >= z0) && (zp < zend) && own0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Real v, w;
      if (MODE == SM_APPLY) {
        v = fz[c];
        w = hz[c];
      } else if (MODE == SM_COMB) {
        const int zb = (wz & 1) << 2;
        v = (c == a.comb_comp && (par0 | zb) == a.comb_off) ? (Real)1 : (Real)0;
        w = (c == a.comb_comp && (par1 | zb) == a.comb_off) ? (Real)1 : (Real)0;
      } else {
        // p_old and u hold no data before the first iteration: select, not multiply
        v = first ? fz[c] : fz[c] + beta * fp[c];
        w = first ? hz[c] : hz[c] + beta * hp[c];
        if (owned) {
          if (!first) st(b_u, c, o0, fu[c] + alpha_prev * fp[c]);
          st(b_pout, c, o0, v);
        }
      }
      P[slot][c][li0] = v;
      if (has1) P[slot][c][li1] = w;
      if (MAT) {
        U[slot][c][li0] = ku[c];
        if (has1) U[slot][c][li1] = kh[c];
      }
    }
  };
  auto ring = [&](int zp) { return (zp - z0 + 1) % 3; };

  // Loop order: every value loaded in one layer is first used at the top of
  // the next one, after which the layer's new loads are issued; stores of
  // the finished plane are also issued at the top.  The single wait on
  // memory per layer thus comes after a whole layer of work.
  double acc = 0.0;
  Real carry[3] = {0, 0, 0};
  Real qpend[3] = {0, 0, 0};
  // cubic elements: the bottom face of the next element (its node values and
  // in-plane differences) is this element's top face, carried in registers
  Real fbot[3][4], fbotF[3][4];
  // pending output node (stored at the next layer's top): its index, valid
  // while qpending
  unsigned qnode = 0;
  bool qpending = false;
  fetch(z0 - 1);
  commit(z0 - 1, ring(z0 - 1));
  fetch(z0);
  commit(z0, ring(z0));
  fetch(z0 + 1);  // layer z0 always exists and reads plane z0 + 1
  // the modulus is loaded for every thread and layer (the wrapped address is
  // always valid) and masked at use, so no register is conditionally loaded
  Real Enext = ld(b_E, 0, (unsigned)wrapi(z0 - 1, nz) * uplane * (unsigned)sizeof(Real) + exy_b);
  const Real emask = elem_valid ? (Real)1 : (Real)0;
  __syncthreads();
  auto flush_q = [&]() {
    if (!qpending) return;
    if (MODE == SM_COMB) {
      a.diag[a.comb_comp * N + qnode] = qpend[0];
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) st(b_out, i, qnode * (unsigned)sizeof(Real), qpend[i]);
    }
    qpending = false;
  };
  for (int ez = z0 - 1; ez < zend; ++ez) {
    const int s0 = ring(ez), s1 = ring(ez + 1);
    const bool more = ez + 1 < zend;   // layer ez + 1 exists and needs plane ez + 2
    const bool more2 = ez + 2 < zend;  // layer ez + 2 exists and needs plane ez + 3
    // Everything loaded during the last layer is consumed first (the modulus
    // and plane ez + 2); only then are this layer's stores and loads issued,
    // so no wait below can fall on a load issued in this layer.
    Real Ecur = Enext * emask;
    asm volatile("" : "+v"(Ecur)::"memory");
    if (more) commit(ez + 2, ring(ez + 2));  // plane ez + 2, in flight since the last layer
    flush_q();
    if (more2) {
      fetch0(ez + 3);
      if (sizeof(Real) == 4) fetch1(ez + 3);  // FP32: the strip one layer ahead as well
    }
    Enext = ld(b_E, 0, (unsigned)wrapi(ez + 1, nz) * uplane * (unsigned)sizeof(Real) + exy_b);
    if constexpr (CUBIC && MAT == 0 && sizeof(Real) == 4) {
      // (FP32 only: in FP64 the 24 carried registers would halve occupancy)
      Real top[3][4], topF[3][4], yv[3][8];
      if (ez == z0 - 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int i = 0; i < 3; ++i) fbot[i][k] = P[s0][i][lie + (k >> 1) * NX + (k & 1)];
#pragma unroll
        for (int i = 0; i < 3; ++i) face_diffs(fbot[i], fbotF[i]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) top[i][k] = P[s1][i][lie + (k >> 1) * NX + (k & 1)];
      double en = 0.0;
      // a.lam, a.mu carry the full Gauss weight; the mode form takes half
      elem_hex_modes_cubic_faces<Real, MODE == SM_CG>(fbot, fbotF, top, topF, Ecur, a.clam, a.cmu,
                                                      yv, en);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          fbot[i][k] = top[i][k];
          fbotF[i][k] = topF[i][k];
        }
      if (elem_owned && ez >= z0) acc += en;
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) Y[c * 3 + i][tid] = yv[i][c];
    } else {
      Real uv[3][8], yv[3][8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
        const int li = lie + cy * NX + cx;
#pragma unroll
        for (int i = 0; i < 3; ++i) uv[i][c] = P[cz ? s1 : s0][i][li];
      }
      double en = 0.0;
      if constexpr (MAT == 1) {
        Real kv[3][8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
          const int li = lie + cy * NX + cx;
#pragma unroll
          for (int i = 0; i < 3; ++i) kv[i][c] = U[cz ? s1 : s0][i][li];
        }
        // Ecur is the phase (0 beyond the grid, where the result is masked)
        elem_hex_tangent<Real, MODE == SM_CG>(kv, uv, Ecur > (Real)0.5, a.pl, a.w, a.ihx, a.ihy,
                                              a.ihz, yv, en);
#pragma unroll
        for (int c = 0; c < 8; ++c)
#pragma unroll
          for (int i = 0; i < 3; ++i) yv[i][c] *= emask;
      } else if constexpr (CUBIC) {
        // a.lam, a.mu carry the full Gauss weight; the mode form takes half
        elem_hex_modes_cubic<Real, MODE == SM_CG>(uv, Ecur, a.clam, a.cmu, yv, en);
      } else {
        elem_hex_modes<Real, MODE == SM_CG>(uv, Ecur * a.lam * (Real)0.5, Ecur * a.mu * (Real)0.5,
                                            a.ihx, a.ihy, a.ihz, yv, en);
      }
      if (elem_owned && ez >= z0) acc += en;
#pragma unroll
      for (int c = 0; c < 8; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) Y[c * 3 + i][tid] = yv[i][c];
    }
    if (sizeof(Real) == 8 && more2) fetch1(ez + 3);  // FP64: after the element (registers)
    __syncthreads();
    if (node_valid) {
      // corners (1,1), (0,1), (1,0), (0,0) of the four x-y neighbouring elements
      if (ez >= z0) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
          qpend[i] = carry[i] + Y[3 * 3 + i][e00] + Y[2 * 3 + i][e00 + 1] +
                     Y[1 * 3 + i][e00 + EX] + Y[0 * 3 + i][e00 + EX + 1];
        const unsigned node = (unsigned)ez * uplane + (unsigned)gny * (unsigned)nx + (unsigned)gnx;
        if (MODE == SM_COMB) {
          const int par = (gnx & 1) | ((gny & 1) << 1) | ((ez & 1) << 2);
          if (par == a.comb_off) {
            qpend[0] = qpend[a.comb_comp];
            qnode = node;
            qpending = true;
          }
        } else {
          qnode = node;
          qpending = true;
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
        carry[i] = Y[7 * 3 + i][e00] + Y[6 * 3 + i][e00 + 1] + Y[5 * 3 + i][e00 + EX] +
                   Y[4 * 3 + i][e00 + EX + 1];
    }
    __syncthreads();
  }
  flush_q();
  if (MODE == SM_CG) {
    const double s = block_sum<NT>(acc, red);
    if (tid == 0) a.partial[lb] = s;
    if (a.ctl)
      fused_ctrl<NT, CTRL_ALPHA>(a.ctl, a.partial, per_cell, a.h, cell, a.cs,
                                               a.parity, red);
  }
}

// ----------------------------------------------------------------- 2D ----
// Quad (plane strain): corner c = cx + 2 cy.
template <typename Real>
__device__ __forceinline__ void elem_quad(const Real (&u)[2][4], Real Elam, Real Emu, Real ihx,
                                          Real ihy, Real (&y)[2][4]) {
  // dX[i][gy], dY[i][gx]
  Real dX[2][2], dY[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    interp2(u[i][1] - u[i][0], u[i][3] - u[i][2], dX[i][0], dX[i][1]);
    interp2(u[i][2] - u[i][0], u[i][3] - u[i][1], dY[i][0], dY[i][1]);
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      dX[i][g] *= ihx;
      dY[i][g] *= ihy;
    }
  }
  Real SX[2][2] = {{0, 0}, {0, 0}}, SY[2][2] = {{0, 0}, {0, 0}};  // [comp][g]
  const Real m2 = Emu + Emu;
#pragma unroll
  for (int gx = 0; gx < 2; ++gx)
#pragma unroll
    for (int gy = 0; gy < 2; ++gy) {
      const Real e11 = dX[0][gy], e22 = dY[1][gx];
      const Real g12 = dX[1][gy] + dY[0][gx];
      const Real lt = Elam * (e11 + e22);
      const Real s11 = lt + m2 * e11, s22 = lt + m2 * e22, s12 = Emu * g12;
      SX[0][gy] += s11;
      SY[0][gx] += s12;
      SX[1][gy] += s12;
      SY[1][gx] += s22;
    }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    Real R0, R1;
    interp2(SX[i][0], SX[i][1], R0, R1);  // cy = 0, 1
    R0 *= ihx;
    R1 *= ihx;
    y[i][1] = R0;
    y[i][0] = -R0;
    y[i][3] = R1;
    y[i][2] = -R1;
    interp2(SY[i][0], SY[i][1], R0, R1);  // cx = 0, 1
    R0 *= ihy;
    R1 *= ihy;
    y[i][2] += R0;
    y[i][0] -= R0;
    y[i][3] += R1;
    y[i][1] -= R1;
  }
}

// Two linear triangles per pixel (the alternative 2D element): the pixel is
// split along its anti-diagonal into T0 = corners (0, 1, 2) and T1 =
// corners (3, 2, 1).  The strain is constant on each, so one point of weight
// A = hx hy / 2 integrates exactly; Elam, Emu carry E and A.
template <typename Real>
__device__ __forceinline__ void elem_tri2(const Real (&u)[2][4], Real Elam, Real Emu, Real ihx,
                                          Real ihy, Real (&y)[2][4]) {
  const Real m2 = Emu + Emu;
  {  // T0: grad N_0 = (-1/hx, -1/hy), grad N_1 = (1/hx, 0), grad N_2 = (0, 1/hy)
    const Real e11 = (u[0][1] - u[0][0]) * ihx, e22 = (u[1][2] - u[1][0]) * ihy;
    const Real g12 = (u[0][2] - u[0][0]) * ihy + (u[1][1] - u[1][0]) * ihx;
    const Real lt = Elam * (e11 + e22);
    const Real s11 = lt + m2 * e11, s22 = lt + m2 * e22, s12 = Emu * g12;
    const Real ax = s11 * ihx, ay = s12 * ihy, bx = s12 * ihx, by = s22 * ihy;
    y[0][0] = -ax - ay;
    y[1][0] = -bx - by;
    y[0][1] = ax;
    y[1][1] = bx;
    y[0][2] = ay;
    y[1][2] = by;
  }
  {  // T1: grad N_3 = (1/hx, 1/hy), grad N_2 = (-1/hx, 0), grad N_1 = (0, -1/hy)
    const Real e11 = (u[0][3] - u[0][2]) * ihx, e22 = (u[1][3] - u[1][1]) * ihy;
    const Real g12 = (u[0][3] - u[0][1]) * ihy + (u[1][3] - u[1][2]) * ihx;
    const Real lt = Elam * (e11 + e22);
    const Real s11 = lt + m2 * e11, s22 = lt + m2 * e22, s12 = Emu * g12;
    const Real ax = s11 * ihx, ay = s12 * ihy, bx = s12 * ihx, by = s22 * ihy;
    y[0][3] = ax + ay;
    y[1][3] = bx + by;
    y[0][2] -= ax;
    y[1][2] -= bx;
    y[0][1] -= ay;
    y[1][1] -= by;
  }
}

// One block: TX x TY2 output nodes (TX 16 or 32 wide, TY2 one or two 16-node
// rows of tiles, which then share a halo row), 384 threads; every thread owns up to R
// nodes of the halo-extended tile, R elements and R outputs (index tid +
// r * 384).  All loads of its nodes (and element moduli) are issued before
// any store, so a thread keeps up to a dozen loads in flight.  Loads use clamped,
// valid addresses and are masked where the value is committed.
// TRI: the pixel is two linear triangles (elem_tri2) instead of a bilinear
// quadrilateral.
template <typename Real, int MODE, bool TRI = false, int TT = 1, int TX = TILE>
__global__ void __launch_bounds__(STENCIL_THREADS)
    k_stiffness2d(StencilArgs<Real> a) {
  // TT rows of 16-node tiles, TX (16 or 32) nodes wide: a tunable tile shape
  // (32-wide rows are whole 128-byte lines in FP32)
  constexpr int TY2 = TT * TILE;
  constexpr int ETX = TX + 1, NTX = TX + 2;  // elements / nodes per row with halo
  constexpr int NNODE2 = NTX * (TY2 + 2);  // nodes with halo
  constexpr int NELEM2 = ETX * (TY2 + 1);  // elements with halo
  constexpr int NOUT2 = TX * TY2;          // outputs
  __shared__ Real P[2][NNODE2];
  __shared__ Real Y[8][NELEM2];
  __shared__ double red[8];
  const int tid = threadIdx.x;
  const int per_cell = gridDim.x * gridDim.y;
  const int lbg = xcd_logical_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                    per_cell * gridDim.z);
  const int cell = lbg / per_cell;
  const int lb = lbg - cell * per_cell;
  shift_args(a, cell);
  if (MODE == SM_CG && a.st->done) return;
  const int x0 = (lb % gridDim.x) * TX, y0 = (lb / gridDim.x) * TY2;
  const int nx = a.nx, ny = a.ny;
  const long long N = a.N;
  bool first = false;
  Real beta = 0, alpha_prev = 0;
  if (MODE == SM_CG) {
    first = a.st->first != 0;
    beta = (Real)a.st->beta;
    alpha_prev = (Real)a.st->alpha;
  }
  constexpr int R = (NNODE2 + STENCIL_THREADS - 1) / STENCIL_THREADS;  // items per thread
  static_assert(R * STENCIL_THREADS >= NNODE2 && R * STENCIL_THREADS >= NELEM2 &&
                    R * STENCIL_THREADS >= NOUT2,
                "R items per thread cover the tile");
  // element moduli (beyond the grid: 0)
  Real Ee[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = min(tid + r * STENCIL_THREADS, NELEM2 - 1);
    const int gex = x0 - 1 + e % ETX, gey = y0 - 1 + e / ETX;
    const Real v = a.E[(long long)wrapi(gex, nx) + (long long)nx * wrapi(gey, ny)];
    Ee[r] = (gex < nx && gey < ny) ? v : (Real)0;
  }
  // nodes: loads of both first
  long long node[R];
  bool owned[R], valid[R];
  int par[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int idx = tid + r * STENCIL_THREADS;
    valid[r] = idx < NNODE2;
    const int ci = min(idx, NNODE2 - 1);
    const int lx = ci % NTX, ly = ci / NTX;
    const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
    const int wx = wrapi(gx, nx), wy = wrapi(gy, ny);
    node[r] = (long long)wx + (long long)nx * wy;
    owned[r] = valid[r] && lx >= 1 && lx <= TX && ly >= 1 && ly <= TY2 && gx < nx && gy < ny;
    par[r] = (wx & 1) | ((wy & 1) << 1);
  }
  Real v[R][2];
  if (MODE == SM_APPLY) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) v[r][c] = a.in[c * N + node[r]];
  } else if (MODE == SM_COMB) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        v[r][c] = (c == a.comb_comp && par[r] == a.comb_off) ? (Real)1 : (Real)0;
  } else {
    Real z[R][2], po[R][2], uo[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        z[r][c] = a.zin[c * N + node[r]];
        po[r][c] = (Real)0;
        uo[r][c] = (Real)0;
      }
    if (!first) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          po[r][c] = a.in[c * N + node[r]];
          if (owned[r]) uo[r][c] = a.u[c * N + node[r]];  // u of owned nodes only
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) v[r][c] = first ? z[r][c] : z[r][c] + beta * po[r][c];
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (owned[r]) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (!first) a.u[c * N + node[r]] = uo[r][c] + alpha_prev * po[r][c];
          a.pout[c * N + node[r]] = v[r][c];
        }
      }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (valid[r]) {
      P[0][tid + r * STENCIL_THREADS] = v[r][0];
      P[1][tid + r * STENCIL_THREADS] = v[r][1];
    }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = tid + r * STENCIL_THREADS;
    if (e < NELEM2) {
      const int exl = e % ETX, eyl = e / ETX;
      Real uv[2][4], yv[2][4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int li = (eyl + (c >> 1)) * NTX + exl + (c & 1);
        uv[0][c] = P[0][li];
        uv[1][c] = P[1][li];
      }
      if constexpr (TRI)  // a.lam, a.mu carry the Gauss weight hx hy / 4; A is twice that
        elem_tri2(uv, (Real)2 * Ee[r] * a.lam, (Real)2 * Ee[r] * a.mu, a.ihx, a.ihy, yv);
      else
        elem_quad(uv, Ee[r] * a.lam, Ee[r] * a.mu, a.ihx, a.ihy, yv);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        Y[c * 2 + 0][e] = yv[0][c];
        Y[c * 2 + 1][e] = yv[1][c];
      }
    }
  }
  __syncthreads();
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int o = tid + r * STENCIL_THREADS;
    const int oxl = o % TX, oyl = o / TX;
    const int gnx = x0 + oxl, gny = y0 + oyl;
    if (o < NOUT2 && gnx < nx && gny < ny) {
      const int e00 = oyl * ETX + oxl;
      Real q[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        q[i] = Y[3 * 2 + i][e00] + Y[2 * 2 + i][e00 + 1] + Y[1 * 2 + i][e00 + ETX] +
               Y[0 * 2 + i][e00 + ETX + 1];
      const long long nd = (long long)gnx + (long long)nx * gny;
      const int li = (oyl + 1) * NTX + oxl + 1;
      if (MODE == SM_COMB) {
        const int pr = (gnx & 1) | ((gny & 1) << 1);
        if (pr == a.comb_off) a.diag[a.comb_comp * N + nd] = q[a.comb_comp];
      } else {
        a.out[nd] = q[0];
        a.out[N + nd] = q[1];
        if (MODE == SM_CG)
          acc += (double)P[0][li] * (double)q[0] + (double)P[1][li] * (double)q[1];
      }
    }
  }
  if (MODE == SM_CG) {
    const double s = block_sum<STENCIL_THREADS>(acc, red);
    if (tid == 0) a.partial[lb] = s;
    if (a.ctl)
      fused_ctrl<STENCIL_THREADS, CTRL_ALPHA>(a.ctl, a.partial, per_cell, a.h, cell, a.cs,
                                              a.parity, red);
  }
}

// ------------------------------------------------- right-hand side -------
// f(I) = -sum over the 2^d elements e containing I of E_e F[c(I,e)], with
// F = w sum_q B_q^T C^ macro the element force of a unit modulus (the same
// for every element on a regular grid).  Node-parallel gather: deterministic.
// fabs (optional) accumulates |E_e F| for the homogeneous-material test.
template <typename Real>
__global__ void k_rhs(const Real *E, const double *F /* [d][2^d] */, Real *f, Real *fabs_out,
                      int dim, int nx, int ny, int nz, long long N, long long cs) {
  const int cell = blockIdx.y;
  E = cshift(E, cell, cs);
  F = cshift(F, cell, cs);
  f = cshift(f, cell, cs);
  fabs_out = cshift(fabs_out, cell, cs);
  // 32-bit index arithmetic: a cell holds at most 512^3 nodes
  const unsigned node = blockIdx.x * blockDim.x + threadIdx.x;
  if ((long long)node >= N) return;
  const unsigned row = node / (unsigned)nx;
  const int ix = (int)(node - row * (unsigned)nx);
  const int iz = (int)(row / (unsigned)ny);
  const int iy = (int)(row - (unsigned)iz * (unsigned)ny);
  const int nloc = 1 << dim;
  double acc[3] = {0, 0, 0}, aab[3] = {0, 0, 0};
  for (int c = 0; c < nloc; ++c) {
    const int ex = wrapi(ix - (c & 1), nx), ey = wrapi(iy - ((c >> 1) & 1), ny);
    const int ez = dim == 3 ? wrapi(iz - ((c >> 2) & 1), nz) : 0;
    const double Ee = (double)E[(long long)ex + (long long)nx * (ey + (long long)ny * ez)];
    for (int i = 0; i < dim; ++i) {
      const double v = -Ee * F[i * nloc + c];
      acc[i] += v;
      aab[i] += fabs(v);
    }
  }
  for (int i = 0; i < dim; ++i) {
    f[i * N + node] = (Real)acc[i];
    if (fabs_out) fabs_out[i * N + node] = (Real)aab[i];
  }
}

// Element force of a unit modulus under a constant strain (Mandel macro):
// F[i][c] = w sum_q sum_j sigma0_ij dphi_c/dx_j, sigma0 = C^ macro.  One
// thread; evaluated with the same transposed factorisation as the stiffness.
// tri (2D): the two linear triangles of elem_tri2, weight A = 2 w each; the
// summed triangle gradients of corners 0..3 are (-ihx, -ihy), (ihx, -ihy),
// (-ihx, ihy), (ihx, ihy).
__global__ void k_unit_force(double *F, const double *macro, int dim, double lam, double mu,
                             double ihx, double ihy, double ihz, long long cs, int tri) {
  if (threadIdx.x != 0) return;
  F = cshift(F, blockIdx.x, cs);  // one block per cell
  macro = cshift(macro, blockIdx.x, cs);
  const double r2 = 0.70710678118654752440;  // Mandel shear -> tensor
  if (dim == 3) {
    const double e11 = macro[0], e22 = macro[1], e33 = macro[2];
    const double e23 = macro[3] * r2, e13 = macro[4] * r2, e12 = macro[5] * r2;
    const double lt = lam * (e11 + e22 + e33);
    double s[3][3];
    s[0][0] = lt + 2 * mu * e11;
    s[1][1] = lt + 2 * mu * e22;
    s[2][2] = lt + 2 * mu * e33;
    s[1][2] = s[2][1] = 2 * mu * e23;
    s[0][2] = s[2][0] = 2 * mu * e13;
    s[0][1] = s[1][0] = 2 * mu * e12;
    for (int i = 0; i < 3; ++i) {
      double SX[2][2], SY[2][2], SZ[2][2], y[8];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          SX[a][b] = 2 * s[i][0];  // sum over the two Gauss points of the derivative axis
          SY[a][b] = 2 * s[i][1];
          SZ[a][b] = 2 * s[i][2];
        }
      force_hex<double>(SX, SY, SZ, ihx, ihy, ihz, y);
      for (int c = 0; c < 8; ++c) F[i * 8 + c] = y[c];
    }
  } else if (tri) {
    const double e11 = macro[0], e22 = macro[1], e12 = macro[2] * r2;
    const double lt = lam * (e11 + e22);
    const double s11 = lt + 2 * mu * e11, s22 = lt + 2 * mu * e22, s12 = 2 * mu * e12;
    for (int c = 0; c < 4; ++c) {
      const double gx = 2.0 * ((c & 1) ? ihx : -ihx), gy = 2.0 * ((c >> 1) ? ihy : -ihy);
      F[0 * 4 + c] = s11 * gx + s12 * gy;  // 2.0: A = 2 w (lam, mu carry w)
      F[1 * 4 + c] = s12 * gx + s22 * gy;
    }
  } else {
    const double e11 = macro[0], e22 = macro[1], e12 = macro[2] * r2;
    const double lt = lam * (e11 + e22);
    const double s11 = lt + 2 * mu * e11, s22 = lt + 2 * mu * e22, s12 = 2 * mu * e12;
    double u[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, y[2][4];
    (void)u;
    const double sx[2] = {s11, s12}, sy[2] = {s12, s22};
    for (int i = 0; i < 2; ++i) {
      double R0, R1;
      interp2(2 * sx[i], 2 * sx[i], R0, R1);
      R0 *= ihx;
      R1 *= ihx;
      y[i][1] = R0;
      y[i][0] = -R0;
      y[i][3] = R1;
      y[i][2] = -R1;
      interp2(2 * sy[i], 2 * sy[i], R0, R1);
      R0 *= ihy;
      R1 *= ihy;
      y[i][2] += R0;
      y[i][0] -= R0;
      y[i][3] += R1;
      y[i][1] -= R1;
      for (int c = 0; c < 4; ++c) F[i * 4 + c] = y[i][c];
    }
  }
}

// ------------------------------------------------------- stresses --------
// sigma_q = E_e C^ (macro + B_q u_e) at every Gauss point, written in Mandel
// form to sig[r][q][e] when sig != NULL, and per-block partial sums of
// w sigma_q for the homogenised stress.  Element-parallel, one thread each.
template <typename Real>
__global__ void __launch_bounds__(256) k_stress(const Real *u, const Real *E, const double *macro, double lam, double mu,
                         double w, double ihx, double ihy, double ihz, int dim, int nx, int ny,
                         int nz, long long N, double *sig, double *partial /* [ds][nblocks] */,
                         long long cs, long long sig_cs, int tri) {
  __shared__ double red[8];
  const int cell = blockIdx.y;
  u = cshift(u, cell, cs);
  E = cshift(E, cell, cs);
  macro = cshift(macro, cell, cs);
  partial = cshift(partial, cell, cs);
  sig = cshift(sig, cell, sig_cs);
  // 32-bit index arithmetic (a cell holds at most 512^3 nodes); every loop
  // over corners, components and Gauss points is unrolled so that the
  // per-element arrays stay in registers
  const unsigned eu = blockIdx.x * blockDim.x + threadIdx.x;
  const long long e = eu;
  const int ds = dim == 3 ? 6 : 3;
  double loc[6] = {0, 0, 0, 0, 0, 0};
  const double r2 = 1.41421356237309504880;
  if (e < N) {
    const unsigned row = eu / (unsigned)nx;
    const int ix = (int)(eu - row * (unsigned)nx);
    const int iz = (int)(row / (unsigned)ny);
    const int iy = (int)(row - (unsigned)iz * (unsigned)ny);
    const double Ee = (double)E[e];
    if (dim == 3) {
      double uv[3][8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const long long nd = (long long)wrapi(ix + (c & 1), nx) +
                             (long long)nx * (wrapi(iy + ((c >> 1) & 1), ny) +
                                              (long long)ny * wrapi(iz + (c >> 2), nz));
#pragma unroll
        for (int i = 0; i < 3; ++i) uv[i][c] = u ? (double)u[i * N + nd] : 0.0;
      }
      double dX[3][2][2], dY[3][2][2], dZ[3][2][2];
#pragma unroll
      for (int i = 0; i < 3; ++i) grad_hex<double>(uv[i], ihx, ihy, ihz, dX[i], dY[i], dZ[i]);
      const double m11 = macro[0], m22 = macro[1], m33 = macro[2];
      const double m23 = macro[3] * r2, m13 = macro[4] * r2, m12 = macro[5] * r2;  // engineering
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int gx = q & 1, gy = (q >> 1) & 1, gz = q >> 2;
        const double e11 = m11 + dX[0][gy][gz], e22 = m22 + dY[1][gx][gz],
                     e33 = m33 + dZ[2][gx][gy];
        const double g23 = m23 + dY[2][gx][gz] + dZ[1][gx][gy];
        const double g13 = m13 + dX[2][gy][gz] + dZ[0][gx][gy];
        const double g12 = m12 + dX[1][gy][gz] + dY[0][gx][gz];
        const double lt = lam * (e11 + e22 + e33);
        double s[6];
        s[0] = Ee * (lt + 2 * mu * e11);
        s[1] = Ee * (lt + 2 * mu * e22);
        s[2] = Ee * (lt + 2 * mu * e33);
        s[3] = Ee * mu * g23 * r2;  // Mandel: sqrt2 sigma_23 = sqrt2 mu gamma_23
        s[4] = Ee * mu * g13 * r2;
        s[5] = Ee * mu * g12 * r2;
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          if (sig) sig[((long long)r * 8 + q) * N + e] = s[r];
          loc[r] += w * s[r];
        }
      }
    } else {
      double uv[2][4];
      for (int c = 0; c < 4; ++c) {
        const long long nd =
            (long long)wrapi(ix + (c & 1), nx) + (long long)nx * wrapi(iy + (c >> 1), ny);
        for (int i = 0; i < 2; ++i) uv[i][c] = u ? (double)u[i * N + nd] : 0.0;
      }
      if (tri) {
        // the two triangles of elem_tri2, one point each of weight 2 w:
        // sig[r][t][e], t = 0, 1
        const double ex[2] = {(uv[0][1] - uv[0][0]) * ihx, (uv[0][3] - uv[0][2]) * ihx};
        const double ey[2] = {(uv[1][2] - uv[1][0]) * ihy, (uv[1][3] - uv[1][1]) * ihy};
        const double gg[2] = {(uv[0][2] - uv[0][0]) * ihy + (uv[1][1] - uv[1][0]) * ihx,
                              (uv[0][3] - uv[0][1]) * ihy + (uv[1][3] - uv[1][2]) * ihx};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const double e11 = macro[0] + ex[t], e22 = macro[1] + ey[t];
          const double g12 = macro[2] * r2 + gg[t];
          const double lt = lam * (e11 + e22);
          double s[3];
          s[0] = Ee * (lt + 2 * mu * e11);
          s[1] = Ee * (lt + 2 * mu * e22);
          s[2] = Ee * mu * g12 * r2;
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            if (sig) sig[((long long)r * 2 + t) * N + e] = s[r];
            loc[r] += 2.0 * w * s[r];
          }
        }
      } else {
      double dX[2][2], dY[2][2];
      for (int i = 0; i < 2; ++i) {
        interp2(uv[i][1] - uv[i][0], uv[i][3] - uv[i][2], dX[i][0], dX[i][1]);
        interp2(uv[i][2] - uv[i][0], uv[i][3] - uv[i][1], dY[i][0], dY[i][1]);
        for (int g = 0; g < 2; ++g) {
          dX[i][g] *= ihx;
          dY[i][g] *= ihy;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gx = q & 1, gy = q >> 1;
        const double e11 = macro[0] + dX[0][gy], e22 = macro[1] + dY[1][gx];
        const double g12 = macro[2] * r2 + dX[1][gy] + dY[0][gx];
        const double lt = lam * (e11 + e22);
        double s[3];
        s[0] = Ee * (lt + 2 * mu * e11);
        s[1] = Ee * (lt + 2 * mu * e22);
        s[2] = Ee * mu * g12 * r2;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          if (sig) sig[((long long)r * 4 + q) * N + e] = s[r];
          loc[r] += w * s[r];
        }
      }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    if (r < ds) {  // uniform
      const double s = block_sum<256>(loc[r], red);
      if (threadIdx.x == 0) partial[(long long)r * gridDim.x + blockIdx.x] = s;
    }
  }
}

// ------------------------------------------- Algorithm 2 in closed form ----
// The diagonal that Algorithm 2 extracts by probing, for isotropic Q1
// elements with exact two-point Gauss integration: for corner c of an
// element, int (dN_c/dx_b)^2 dV = vol_e / (3^(d-1) h_b^2) =: g_b, so
//   K_e[alpha c, alpha c] = E_e (lam g_alpha + mu (g_alpha + sum_b g_b)) =: E_e k_alpha,
// the same for every corner, and diag_{alpha I} = k_alpha * (sum of the
// moduli of the 2^d elements around node I).  Element e is indexed by its
// lowest node, so the elements around node I are I - o, o in {0,1}^d
// (periodic).  Equal to the probing result up to rounding.
template <int DIM>
__global__ void __launch_bounds__(256)
    k_diag_closed(const double *E, double *diag, int nx, int ny, int nz, long long N, double k0,
                  double k1, double k2, long long cs) {
  E = cshift(E, blockIdx.y, cs);
  diag = cshift(diag, blockIdx.y, cs);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const long long plane = (long long)nx * ny;
    const int z = (int)(i / plane);
    const long long rem = i - (long long)z * plane;
    const int y = (int)(rem / nx), x = (int)(rem - (long long)y * nx);
    const int xm = x == 0 ? nx - 1 : x - 1, ym = y == 0 ? ny - 1 : y - 1;
    const long long r0 = (long long)y * nx, r1 = (long long)ym * nx;
    double s;
    if (DIM == 3) {
      const int zm = z == 0 ? nz - 1 : z - 1;
      const long long p0 = (long long)z * plane, p1 = (long long)zm * plane;
      s = ((E[p0 + r0 + x] + E[p0 + r0 + xm]) + (E[p0 + r1 + x] + E[p0 + r1 + xm])) +
          ((E[p1 + r0 + x] + E[p1 + r0 + xm]) + (E[p1 + r1 + x] + E[p1 + r1 + xm]));
    } else {
      s = (E[r0 + x] + E[r0 + xm]) + (E[r1 + x] + E[r1 + xm]);
    }
    diag[i] = k0 * s;
    diag[N + i] = k1 * s;
    if (DIM == 3) diag[2 * N + i] = k2 * s;
  }
}

// ----------------------------------------------- power-law Newton pieces ----
// Element corner values of the nodal field at the element with lowest node
// (ex, ey, ez) (periodic).
template <typename Real>
__device__ __forceinline__ void gather_hex(const Real *u, long long N, int nx, int ny, int nz,
                                           int ex, int ey, int ez, Real (&v)[3][8]) {
  const long long plane = (long long)nx * ny;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int x = ex + (c & 1), y = ey + ((c >> 1) & 1), z = ez + (c >> 2);
    const long long node = (long long)(x == nx ? 0 : x) + (long long)nx * (y == ny ? 0 : y) +
                           plane * (z == nz ? 0 : z);
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i][c] = u[i * N + node];
  }
}

// Moduli of the linearised law at a Gauss point with strain eps: sigma =
// kb tr(eps) I + g e and tangent C = kb I (x) I + g P_dev + h e (x) e, e =
// dev(eps) (inclusion: kb = Ki, g = 2 mui, h = 0).
template <typename Real>
__device__ __forceinline__ void powerlaw_point(const Real (&eps)[6], bool matrix,
                                               const PowerLawArgs &m, Real (&e)[6], Real &tr,
                                               Real &kb, Real &g, Real &h) {
  tr = eps[0] + eps[1] + eps[2];
  const Real tr3 = tr / (Real)3;
  Real ee = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    e[k] = eps[k] - (k < 3 ? tr3 : (Real)0);
    ee += e[k] * e[k];
  }
  if (matrix) {
    powerlaw_gh(ee, m, g, h);
    kb = (Real)m.K;
  } else {
    g = (Real)(2.0 * m.mui);
    h = (Real)0;
    kb = (Real)m.Ki;
  }
}

// Newton right-hand side f = -B^T W sigma(E + B uk) (eq. lin_system) and,
// with DIAG, the diagonal of the tangent K(uk) = B^T W C B, one thread per
// node.  The node is corner o of the elements node - o, o in {0,1}^3; at
// each of their Gauss points q the shape gradient b = grad N_o(q) gives the
// node's force w sigma(q) b and, for component a, the diagonal entry
// w beta_a^T C(q) beta_a of the unit strain beta_a = sym(e_a (x) b):
//   beta^T C beta = kb tr^2 + g (beta.beta - tr^2 / 3) + h (e.beta)^2
// (what Algorithm 2 returns, in one pass; no atomics, fixed order).
// part: per-block ||f||^2 partials.
template <typename Real, bool DIAG>
__global__ void __launch_bounds__(256)
    k_nl_force(const Real *uk, const Real *phase, Real *f, Real *diag, double *part,
               PowerLawArgs m, Real w, Real ihx, Real ihy, Real ihz, int nx, int ny, int nz,
               long long N) {
  __shared__ double red[4];
  const long long plane = (long long)nx * ny;
  const Real r2 = (Real)0.70710678118654752440084436210485;
  double ff = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const int z = (int)(i / plane);
    const long long rem = i - (long long)z * plane;
    const int y = (int)(rem / nx), x = (int)(rem - (long long)y * nx);
    Real acc[3] = {0, 0, 0}, dg[3] = {0, 0, 0};
    for (int o = 0; o < 8; ++o) {
      const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
      const int ex = x - ox < 0 ? nx - 1 : x - ox, ey = y - oy < 0 ? ny - 1 : y - oy,
                ez = z - oz < 0 ? nz - 1 : z - oz;
      Real v[3][8];
      gather_hex(uk, N, nx, ny, nz, ex, ey, ez, v);
      const bool matrix = phase[(long long)ex + (long long)nx * ey + plane * ez] > (Real)0.5;
      Real kX[3][2][2], kY[3][2][2], kZ[3][2][2];
#pragma unroll
      for (int c = 0; c < 3; ++c) grad_hex(v[c], ihx, ihy, ihz, kX[c], kY[c], kZ[c]);
#pragma unroll
      for (int gx = 0; gx < 2; ++gx)
#pragma unroll
        for (int gy = 0; gy < 2; ++gy)
#pragma unroll
          for (int gz = 0; gz < 2; ++gz) {
            Real es[6], e[6], tr, kb, g, h;
            mandel_strain(kX, kY, kZ, gx, gy, gz, es);
#pragma unroll
            for (int k = 0; k < 6; ++k) es[k] += (Real)m.macro[k];
            powerlaw_point(es, matrix, m, e, tr, kb, g, h);
            Real sg[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) sg[k] = g * e[k] + (k < 3 ? kb * tr : (Real)0);
            // grad N_o at the Gauss point
            const Real lx = gx == ox ? gA<Real>() : gB<Real>();
            const Real ly = gy == oy ? gA<Real>() : gB<Real>();
            const Real lz = gz == oz ? gA<Real>() : gB<Real>();
            const Real bx = (ox ? ihx : -ihx) * ly * lz;
            const Real by = (oy ? ihy : -ihy) * lx * lz;
            const Real bz = (oz ? ihz : -ihz) * lx * ly;
            acc[0] += sg[0] * bx + r2 * (sg[5] * by + sg[4] * bz);
            acc[1] += sg[1] * by + r2 * (sg[5] * bx + sg[3] * bz);
            acc[2] += sg[2] * bz + r2 * (sg[4] * bx + sg[3] * by);
            if (DIAG) {
              const Real b2x = bx * bx, b2y = by * by, b2z = bz * bz;
              const Real bb[3] = {b2x + (Real)0.5 * (b2y + b2z), b2y + (Real)0.5 * (b2x + b2z),
                                  b2z + (Real)0.5 * (b2x + b2y)};
              const Real t2[3] = {b2x, b2y, b2z};
              const Real eb[3] = {e[0] * bx + r2 * (e[5] * by + e[4] * bz),
                                  e[1] * by + r2 * (e[5] * bx + e[3] * bz),
                                  e[2] * bz + r2 * (e[4] * bx + e[3] * by)};
#pragma unroll
              for (int a = 0; a < 3; ++a)
                dg[a] += kb * t2[a] + g * (bb[a] - t2[a] / (Real)3) + h * eb[a] * eb[a];
            }
          }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const Real fc = -w * acc[c];
      f[c * N + i] = fc;
      ff += (double)fc * (double)fc;
      if (DIAG) diag[c * N + i] = w * dg[c];
    }
  }
  const double s = block_sum<256>(ff, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sum of the Gauss-point stresses sigma(E + B uk) per block, one element per
// thread: part[k * nblocks + block], k = 0..5 (the volume average is the
// total / (8 N)).
template <typename Real>
__global__ void __launch_bounds__(256)
    k_nl_stress_sum(const Real *uk, const Real *phase, double *part, PowerLawArgs m, Real ihx,
                    Real ihy, Real ihz, int nx, int ny, int nz, long long N) {
  __shared__ double red[4];
  const long long plane = (long long)nx * ny;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const int z = (int)(i / plane);
    const long long rem = i - (long long)z * plane;
    const int y = (int)(rem / nx), x = (int)(rem - (long long)y * nx);
    Real v[3][8];
    gather_hex(uk, N, nx, ny, nz, x, y, z, v);
    const bool matrix = phase[i] > (Real)0.5;
    Real kX[3][2][2], kY[3][2][2], kZ[3][2][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) grad_hex(v[c], ihx, ihy, ihz, kX[c], kY[c], kZ[c]);
#pragma unroll
    for (int gx = 0; gx < 2; ++gx)
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gz = 0; gz < 2; ++gz) {
          Real es[6], e[6], tr, kb, g, h;
          mandel_strain(kX, kY, kZ, gx, gy, gz, es);
#pragma unroll
          for (int k = 0; k < 6; ++k) es[k] += (Real)m.macro[k];
          powerlaw_point(es, matrix, m, e, tr, kb, g, h);
#pragma unroll
          for (int k = 0; k < 6; ++k) acc[k] += (double)(g * e[k] + (k < 3 ? kb * tr : (Real)0));
        }
  }
  for (int k = 0; k < 6; ++k) {
    const double s = block_sum<256>(acc[k], red);
    if (threadIdx.x == 0) part[(long long)k * gridDim.x + blockIdx.x] = s;
  }
}

// ------------------------------------- topology optimisation (2D triangles) ----
// Weights of the objective's gradient: W[g][a] = 2 (sigma_bar_g - t_g)_a / |Y|.
struct TopoW {
  double w[3][3];
};

// Gradient of f_sigma = sum_g ||sigma_bar_g - t_g||^2 (eq. aim_fun) in the
// pixel densities, for a group of three cells holding the unit load cases
// e_g on the same density (E = rho, C = rho C0).  By the mutual-energy
// identity, d (sigma_bar_g)_a / d rho_e = (1/|Y|) sum over the pixel's two
// triangles of A eps_a^T C0 eps_g with eps_g = e_g + B u_g, so no adjoint
// solve is needed: grad_e = sum_t A sum_g (sum_a W[g][a] eps_a)^T C0 eps_g.
// One thread per pixel; u of cell g at u + g * cs bytes.
__global__ void __launch_bounds__(256)
    k_topo_sens_tri(const double *u, long long cs, TopoW W, double lam, double mu, double A,
                    double ihx, double ihy, int nx, int ny, long long N, double *grad) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  const int x = (int)(e % nx), y = (int)(e / nx);
  const int x1 = x + 1 == nx ? 0 : x + 1, y1 = y + 1 == ny ? 0 : y + 1;
  const long long nd[4] = {(long long)x + (long long)nx * y, (long long)x1 + (long long)nx * y,
                           (long long)x + (long long)nx * y1, (long long)x1 + (long long)nx * y1};
  const double r2 = 0.70710678118654752440;
  double eps[3][2][3];  // [load case][triangle][Mandel]
  for (int g = 0; g < 3; ++g) {
    const double *ug = cshift(u, g, cs);
    double v[2][4];
    for (int c = 0; c < 4; ++c) {
      v[0][c] = ug[nd[c]];
      v[1][c] = ug[N + nd[c]];
    }
    // T0 = corners (0, 1, 2), T1 = corners (3, 2, 1) (elem_tri2)
    const double e11[2] = {(v[0][1] - v[0][0]) * ihx, (v[0][3] - v[0][2]) * ihx};
    const double e22[2] = {(v[1][2] - v[1][0]) * ihy, (v[1][3] - v[1][1]) * ihy};
    const double g12[2] = {(v[0][2] - v[0][0]) * ihy + (v[1][1] - v[1][0]) * ihx,
                           (v[0][3] - v[0][1]) * ihy + (v[1][3] - v[1][2]) * ihx};
    for (int t = 0; t < 2; ++t) {
      eps[g][t][0] = (g == 0 ? 1.0 : 0.0) + e11[t];
      eps[g][t][1] = (g == 1 ? 1.0 : 0.0) + e22[t];
      eps[g][t][2] = (g == 2 ? 1.0 : 0.0) + g12[t] * r2;
    }
  }
  double acc = 0.0;
  for (int t = 0; t < 2; ++t)
    for (int g = 0; g < 3; ++g) {
      double v[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) v[k] += W.w[g][a] * eps[a][t][k];
      const double *eg = eps[g][t];
      // v^T C0 eg, C0 = [[lam + 2 mu, lam, 0], [lam, lam + 2 mu, 0], [0, 0, 2 mu]] (Mandel)
      acc += v[0] * ((lam + 2 * mu) * eg[0] + lam * eg[1]) +
             v[1] * (lam * eg[0] + (lam + 2 * mu) * eg[1]) + v[2] * (2 * mu * eg[2]);
    }
  grad[e] = A * acc;
}

// Phase-field term f_pf = eta int |grad rho|^2 + (1/eta) int rho^2 (1 - rho)^2
// with rho linear on the triangles of elem_tri2 and the double well by
// nodal quadrature (one pixel area per node).  One thread per node I: its
// gradient entry (added to grad) sums the corner-o terms 2 eta A grad N_o .
// grad rho_T of the triangles T of the four pixels I - o; its energy share
// is pixel I's two triangles and node I's well.  part: per-block energy.
__global__ void __launch_bounds__(256)
    k_topo_pf_tri(const double *rho, double eta, double A, double cell, double ihx, double ihy,
                  int nx, int ny, long long N, double *grad, double *part) {
  __shared__ double red[4];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double en = 0.0;
  if (i < N) {
    const int x = (int)(i % nx), y = (int)(i / nx);
    double dg = 0.0;
    for (int o = 0; o < 4; ++o) {
      const int ox = o & 1, oy = o >> 1;
      const int ex = x - ox < 0 ? nx - 1 : x - ox, ey = y - oy < 0 ? ny - 1 : y - oy;
      const int ex1 = ex + 1 == nx ? 0 : ex + 1, ey1 = ey + 1 == ny ? 0 : ey + 1;
      const double r0 = rho[(long long)ex + (long long)nx * ey];
      const double r1 = rho[(long long)ex1 + (long long)nx * ey];
      const double r2v = rho[(long long)ex + (long long)nx * ey1];
      const double r3 = rho[(long long)ex1 + (long long)nx * ey1];
      const double t0x = (r1 - r0) * ihx, t0y = (r2v - r0) * ihy;  // T0 = (0, 1, 2)
      const double t1x = (r3 - r2v) * ihx, t1y = (r3 - r1) * ihy;  // T1 = (3, 2, 1)
      // grad N_o on T0 and T1 (zero where corner o is not a vertex)
      const double n0x[4] = {-ihx, ihx, 0.0, 0.0}, n0y[4] = {-ihy, 0.0, ihy, 0.0};
      const double n1x[4] = {0.0, 0.0, -ihx, ihx}, n1y[4] = {0.0, -ihy, 0.0, ihy};
      dg += 2.0 * eta * A * (n0x[o] * t0x + n0y[o] * t0y + n1x[o] * t1x + n1y[o] * t1y);
      if (o == 0) en = eta * A * (t0x * t0x + t0y * t0y + t1x * t1x + t1y * t1y);
    }
    const double r = rho[i];
    en += cell / eta * r * r * (1.0 - r) * (1.0 - r);
    grad[i] += dg + cell / eta * 2.0 * r * (1.0 - r) * (1.0 - 2.0 * r);
  }
  const double s = block_sum<256>(en, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}


}  // namespace jfft
