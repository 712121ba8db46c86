// Matrix-free stiffness K = B^T W C(E) B for Q1 quads / hexes on a periodic
// grid (Sec. 2.1, eq. disc_wf and eq. lin_system_exp; matrix-free operator of
// Sec. 3.1).  Element data: u at the 2^d corners, strain at the 2^d Gauss
// points by sum factorisation (difference along the derivative axis,
// two-point interpolation along the others), isotropic stress
// sigma = E w (lambda tr(eps) I + 2 mu eps), and the transposed
// factorisation back to the corners.
//
// Kernels are halo-tiled: a block owns a 16 x 16 tile of output nodes in the
// x-y plane and marches along z through a chunk of planes.  It evaluates the
// 17 x 17 elements that touch its tile per layer (13% redundant halo work,
// no atomics, deterministic), keeps two node planes of the input vector in
// LDS, and sums corner contributions of the four x-y neighbouring elements
// from LDS; the z neighbour's contribution is carried in registers to the
// next layer.
#pragma once
#include "jfft_common.h"

namespace jfft {

constexpr int TILE = 16;           // output nodes per tile edge
constexpr int ETILE = TILE + 1;    // elements per tile edge (with halo)
constexpr int NTILE = TILE + 2;    // nodes per tile edge (with halo)
constexpr int NELEM = ETILE * ETILE;  // 289
constexpr int NNODE = NTILE * NTILE;  // 324
constexpr int STENCIL_THREADS = 320;  // 5 wavefronts

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
  Real *diag;            // COMB: diag(K) output
  int comb_comp, comb_off;  // COMB: component and sub-grid offset bits (x, y, z)
  int tz;                // z planes per block (3D)
  Real lam, mu;          // Lame constants of C^ times the Gauss weight
  Real ihx, ihy, ihz;
  int nx, ny, nz;
  long long N;
};

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
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
template <typename Real>
__device__ __forceinline__ void elem_hex(const Real (&u)[3][8], Real Elam, Real Emu, Real ihx,
                                         Real ihy, Real ihz, Real (&y)[3][8]) {
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

template <typename Real, int MODE>
__global__ void __launch_bounds__(STENCIL_THREADS)
    k_stiffness3d(StencilArgs<Real> a) {
  if (MODE == SM_CG && a.st->done) return;
  __shared__ Real P[2][3][NNODE];    // two node planes of the input vector
  __shared__ Real Y[12][NELEM];      // corner contributions of one z level
  __shared__ double red[8];

  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TILE, y0 = blockIdx.y * TILE;
  const int z0 = blockIdx.z * a.tz;
  const int zend = min(z0 + a.tz, a.nz);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long N = a.N;

  bool first = false;
  Real beta = 0, alpha_prev = 0;
  if (MODE == SM_CG) {
    first = a.st->first != 0;
    beta = (Real)a.st->beta;
    alpha_prev = (Real)a.st->alpha;
  }

  // element owned by this thread in the x-y layer
  const bool is_elem = tid < NELEM;
  const int exl = tid % ETILE, eyl = tid / ETILE;
  const int gex = x0 - 1 + exl, gey = y0 - 1 + eyl;
  // elements beyond the grid only feed nodes beyond the grid: give them E = 0
  const bool elem_valid = is_elem && gex < nx && gey < ny;
  const int wex = wrapi(gex, nx), wey = wrapi(gey, ny);
  // output node owned by this thread
  const bool is_node = tid < TILE * TILE;
  const int oxl = tid % TILE, oyl = tid / TILE;
  const int gnx = x0 + oxl, gny = y0 + oyl;
  const bool node_valid = is_node && gnx < nx && gny < ny;

  auto load_plane = [&](int zp, int slot) {
    const int wz = wrapi(zp, nz);
    const bool owned_plane = (zp >= z0) && (zp < zend);
    for (int idx = tid; idx < NNODE; idx += STENCIL_THREADS) {
      const int lx = idx % NTILE, ly = idx / NTILE;
      const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
      const int wx = wrapi(gx, nx), wy = wrapi(gy, ny);
      const long long node = (long long)wx + (long long)nx * (wy + (long long)ny * wz);
      const bool owned = owned_plane && lx >= 1 && lx <= TILE && ly >= 1 && ly <= TILE && gx < nx &&
                         gy < ny;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Real v;
        if (MODE == SM_APPLY) {
          v = a.in[c * N + node];
        } else if (MODE == SM_COMB) {
          const int par = (wx & 1) | ((wy & 1) << 1) | ((wz & 1) << 2);
          v = (c == a.comb_comp && par == a.comb_off) ? (Real)1 : (Real)0;
        } else {
          const Real z = a.zin[c * N + node];
          if (first) {
            v = z;
          } else {
            const Real po = a.in[c * N + node];
            v = z + beta * po;
            if (owned) a.u[c * N + node] += alpha_prev * po;
          }
          if (owned) a.pout[c * N + node] = v;
        }
        P[slot][c][idx] = v;
      }
    }
  };

  double acc = 0.0;
  Real carry[3] = {0, 0, 0};
  load_plane(z0 - 1, 0);
  for (int ez = z0 - 1; ez < zend; ++ez) {
    const int slo = (ez - z0 + 1) & 1, shi = slo ^ 1;
    load_plane(ez + 1, shi);
    __syncthreads();
    Real yv[3][8];
    if (is_elem) {
      Real uv[3][8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
        const int li = (eyl + cy) * NTILE + exl + cx;
#pragma unroll
        for (int i = 0; i < 3; ++i) uv[i][c] = P[cz ? shi : slo][i][li];
      }
      Real Ee = (Real)0;
      if (elem_valid) {
        const int wez = wrapi(ez, nz);
        Ee = a.E[(long long)wex + (long long)nx * (wey + (long long)ny * wez)];
      }
      elem_hex(uv, Ee * a.lam, Ee * a.mu, a.ihx, a.ihy, a.ihz, yv);
    }
    // corners at cz = 0 complete plane ez
    if (ez >= z0) {
      if (is_elem) {
#pragma unroll
        for (int cxy = 0; cxy < 4; ++cxy)
#pragma unroll
          for (int i = 0; i < 3; ++i) Y[cxy * 3 + i][tid] = yv[i][cxy];
      }
      __syncthreads();
      if (node_valid) {
        const int e00 = oyl * ETILE + oxl;  // element (lx-1, ly-1) with lx = oxl+1
        Real q[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          q[i] = carry[i] + Y[3 * 3 + i][e00] + Y[2 * 3 + i][e00 + 1] + Y[1 * 3 + i][e00 + ETILE] +
                 Y[0 * 3 + i][e00 + ETILE + 1];
        }
        const long long node = (long long)gnx + (long long)nx * (gny + (long long)ny * ez);
        const int li = (oyl + 1) * NTILE + oxl + 1;
        if (MODE == SM_COMB) {
          const int par = (gnx & 1) | ((gny & 1) << 1) | ((ez & 1) << 2);
          if (par == a.comb_off) a.diag[a.comb_comp * N + node] = q[a.comb_comp];
        } else {
#pragma unroll
          for (int i = 0; i < 3; ++i) a.out[i * N + node] = q[i];
          if (MODE == SM_CG) {
#pragma unroll
            for (int i = 0; i < 3; ++i) acc += (double)P[slo][i][li] * (double)q[i];
          }
        }
      }
      __syncthreads();
    }
    // corners at cz = 1 start plane ez + 1
    if (is_elem) {
#pragma unroll
      for (int cxy = 0; cxy < 4; ++cxy)
#pragma unroll
        for (int i = 0; i < 3; ++i) Y[cxy * 3 + i][tid] = yv[i][4 + cxy];
    }
    __syncthreads();
    if (node_valid) {
      const int e00 = oyl * ETILE + oxl;
#pragma unroll
      for (int i = 0; i < 3; ++i)
        carry[i] = Y[3 * 3 + i][e00] + Y[2 * 3 + i][e00 + 1] + Y[1 * 3 + i][e00 + ETILE] +
                   Y[0 * 3 + i][e00 + ETILE + 1];
    }
    __syncthreads();
  }
  if (MODE == SM_CG) {
    const double s = block_sum<STENCIL_THREADS>(acc, red);
    if (tid == 0) {
      const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
      a.partial[bid] = s;
    }
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

template <typename Real, int MODE>
__global__ void __launch_bounds__(STENCIL_THREADS)
    k_stiffness2d(StencilArgs<Real> a) {
  if (MODE == SM_CG && a.st->done) return;
  __shared__ Real P[2][NNODE];
  __shared__ Real Y[8][NELEM];
  __shared__ double red[8];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TILE, y0 = blockIdx.y * TILE;
  const int nx = a.nx, ny = a.ny;
  const long long N = a.N;
  bool first = false;
  Real beta = 0, alpha_prev = 0;
  if (MODE == SM_CG) {
    first = a.st->first != 0;
    beta = (Real)a.st->beta;
    alpha_prev = (Real)a.st->alpha;
  }
  for (int idx = tid; idx < NNODE; idx += STENCIL_THREADS) {
    const int lx = idx % NTILE, ly = idx / NTILE;
    const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
    const int wx = wrapi(gx, nx), wy = wrapi(gy, ny);
    const long long node = (long long)wx + (long long)nx * wy;
    const bool owned = lx >= 1 && lx <= TILE && ly >= 1 && ly <= TILE && gx < nx && gy < ny;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      Real v;
      if (MODE == SM_APPLY) {
        v = a.in[c * N + node];
      } else if (MODE == SM_COMB) {
        const int par = (wx & 1) | ((wy & 1) << 1);
        v = (c == a.comb_comp && par == a.comb_off) ? (Real)1 : (Real)0;
      } else {
        const Real z = a.zin[c * N + node];
        if (first) {
          v = z;
        } else {
          const Real po = a.in[c * N + node];
          v = z + beta * po;
          if (owned) a.u[c * N + node] += alpha_prev * po;
        }
        if (owned) a.pout[c * N + node] = v;
      }
      P[c][idx] = v;
    }
  }
  __syncthreads();
  const int exl = tid % ETILE, eyl = tid / ETILE;
  if (tid < NELEM) {
    const int gex = x0 - 1 + exl, gey = y0 - 1 + eyl;
    Real uv[2][4], yv[2][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int li = (eyl + (c >> 1)) * NTILE + exl + (c & 1);
      uv[0][c] = P[0][li];
      uv[1][c] = P[1][li];
    }
    Real Ee = (Real)0;
    if (gex < nx && gey < ny) Ee = a.E[(long long)wrapi(gex, nx) + (long long)nx * wrapi(gey, ny)];
    elem_quad(uv, Ee * a.lam, Ee * a.mu, a.ihx, a.ihy, yv);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      Y[c * 2 + 0][tid] = yv[0][c];
      Y[c * 2 + 1][tid] = yv[1][c];
    }
  }
  __syncthreads();
  double acc = 0.0;
  const int oxl = tid % TILE, oyl = tid / TILE;
  const int gnx = x0 + oxl, gny = y0 + oyl;
  if (tid < TILE * TILE && gnx < nx && gny < ny) {
    const int e00 = oyl * ETILE + oxl;
    Real q[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      q[i] = Y[3 * 2 + i][e00] + Y[2 * 2 + i][e00 + 1] + Y[1 * 2 + i][e00 + ETILE] +
             Y[0 * 2 + i][e00 + ETILE + 1];
    const long long node = (long long)gnx + (long long)nx * gny;
    const int li = (oyl + 1) * NTILE + oxl + 1;
    if (MODE == SM_COMB) {
      const int par = (gnx & 1) | ((gny & 1) << 1);
      if (par == a.comb_off) a.diag[a.comb_comp * N + node] = q[a.comb_comp];
    } else {
      a.out[node] = q[0];
      a.out[N + node] = q[1];
      if (MODE == SM_CG) acc = (double)P[0][li] * (double)q[0] + (double)P[1][li] * (double)q[1];
    }
  }
  if (MODE == SM_CG) {
    const double s = block_sum<STENCIL_THREADS>(acc, red);
    if (tid == 0) a.partial[blockIdx.x + gridDim.x * blockIdx.y] = s;
  }
}

// ------------------------------------------------- right-hand side -------
// f(I) = -sum over the 2^d elements e containing I of E_e F[c(I,e)], with
// F = w sum_q B_q^T C^ macro the element force of a unit modulus (the same
// for every element on a regular grid).  Node-parallel gather: deterministic.
// fabs (optional) accumulates |E_e F| for the homogeneous-material test.
template <typename Real>
__global__ void k_rhs(const Real *E, const double *F /* [d][2^d] */, Real *f, Real *fabs_out,
                      int dim, int nx, int ny, int nz, long long N) {
  const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= N) return;
  const int ix = (int)(node % nx);
  const int iy = (int)((node / nx) % ny);
  const int iz = (int)(node / ((long long)nx * ny));
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
__global__ void k_unit_force(double *F, const double *macro, int dim, double lam, double mu,
                             double ihx, double ihy, double ihz) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
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
__global__ void k_stress(const Real *u, const Real *E, const double *macro, double lam, double mu,
                         double w, double ihx, double ihy, double ihz, int dim, int nx, int ny,
                         int nz, long long N, double *sig, double *partial /* [ds][nblocks] */) {
  __shared__ double red[8];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ds = dim == 3 ? 6 : 3;
  double loc[6] = {0, 0, 0, 0, 0, 0};
  const double r2 = 1.41421356237309504880;
  if (e < N) {
    const int ix = (int)(e % nx), iy = (int)((e / nx) % ny), iz = (int)(e / ((long long)nx * ny));
    const double Ee = (double)E[e];
    if (dim == 3) {
      double uv[3][8];
      for (int c = 0; c < 8; ++c) {
        const long long nd = (long long)wrapi(ix + (c & 1), nx) +
                             (long long)nx * (wrapi(iy + ((c >> 1) & 1), ny) +
                                              (long long)ny * wrapi(iz + (c >> 2), nz));
        for (int i = 0; i < 3; ++i) uv[i][c] = u ? (double)u[i * N + nd] : 0.0;
      }
      double dX[3][2][2], dY[3][2][2], dZ[3][2][2];
      for (int i = 0; i < 3; ++i) grad_hex<double>(uv[i], ihx, ihy, ihz, dX[i], dY[i], dZ[i]);
      const double m11 = macro[0], m22 = macro[1], m33 = macro[2];
      const double m23 = macro[3] * r2, m13 = macro[4] * r2, m12 = macro[5] * r2;  // engineering
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
      double dX[2][2], dY[2][2];
      for (int i = 0; i < 2; ++i) {
        interp2(uv[i][1] - uv[i][0], uv[i][3] - uv[i][2], dX[i][0], dX[i][1]);
        interp2(uv[i][2] - uv[i][0], uv[i][3] - uv[i][1], dY[i][0], dY[i][1]);
        for (int g = 0; g < 2; ++g) {
          dX[i][g] *= ihx;
          dY[i][g] *= ihy;
        }
      }
      for (int q = 0; q < 4; ++q) {
        const int gx = q & 1, gy = q >> 1;
        const double e11 = macro[0] + dX[0][gy], e22 = macro[1] + dY[1][gx];
        const double g12 = macro[2] * r2 + dX[1][gy] + dY[0][gx];
        const double lt = lam * (e11 + e22);
        double s[3];
        s[0] = Ee * (lt + 2 * mu * e11);
        s[1] = Ee * (lt + 2 * mu * e22);
        s[2] = Ee * mu * g12 * r2;
        for (int r = 0; r < 3; ++r) {
          if (sig) sig[((long long)r * 4 + q) * N + e] = s[r];
          loc[r] += w * s[r];
        }
      }
    }
  }
  for (int r = 0; r < ds; ++r) {
    const double s = block_sum<256>(loc[r], red);
    if (threadIdx.x == 0) partial[(long long)r * gridDim.x + blockIdx.x] = s;
  }
}

}  // namespace jfft
