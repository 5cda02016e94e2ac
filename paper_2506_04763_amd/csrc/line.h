// Line-block Jacobi along the last axis of a level (TPF_SMOOTH_LINE): the per-line
// block LU and the per-line solve, as __host__ __device__ bodies (one GPU thread per
// line).
//
// The lines of a level run along its last axis (z in 3D, y in 2D): line l, 0 <= l < S,
// holds the vertices v = l + k S, k = 0 .. n-1, with S = nx ny and n = nz in 3D, S = nx
// and n = ny in 2D.  The couplings of A inside a line form a block tridiagonal matrix
// A_L with L_k = A(k, k-1) (stencil offset -1 along the axis), D_k (the centre) and
// U_k = A(k, k+1) (offset +1); the blocks of neighbours outside the grid are stored as
// zeros, so L_0 = U_{n-1} = 0.  Its block LU without pivoting,
//   D'_0 = D_0,  D'_k = D_k - L_k D'_{k-1}^{-1} U_{k-1},
// is stored per vertex in the level's type as [3][N][4]: G_k = D'_k^{-1},
// V_k = G_k L_k and W_k = G_k U_k.  Then A_L z = r is
//   c_0 = G_0 r_0,  c_k = G_k r_k - V_k c_{k-1}   (forward),
//   z_{n-1} = c_{n-1},  z_k = c_k - W_k z_{k+1}    (backward).
// Consecutive lines are consecutive in x, so a wavefront's loads of one step k are
// contiguous.
#pragma once
#include "stencil.h"

namespace tpf {

struct LineGeo {
  long long S;  // number of lines = stride between consecutive vertices of a line
  int n;        // vertices per line
};

template <int DIM>
__host__ __device__ __forceinline__ LineGeo line_geo(const Geo &G) {
  return DIM == 3 ? LineGeo{(long long)G.nx * G.ny, G.nz} : LineGeo{(long long)G.nx, G.ny};
}

// Stencil offsets of the line couplings and of the centre (offset index
// ax + 3 ay + 9 az with a in {0, 1, 2} for {-1, 0, +1}).
template <int DIM>
struct LineOff {
  static constexpr int M = DIM == 3 ? 4 : 1;   // -1 along the last axis
  static constexpr int C = DIM == 3 ? 13 : 4;  // centre
  static constexpr int P = DIM == 3 ? 22 : 7;  // +1 along the last axis
};

__host__ __device__ __forceinline__ void mul22(const double (&a)[4], const double (&b)[4], double (&c)[4]) {
  c[0] = a[0] * b[0] + a[1] * b[2];
  c[1] = a[0] * b[1] + a[1] * b[3];
  c[2] = a[2] * b[0] + a[3] * b[2];
  c[3] = a[2] * b[1] + a[3] * b[3];
}

// Block LU of line l from the level's FP64 matrix A ([offset][vertex][4]) into lf.
// Returns false if a pivot block is singular or not finite (its G is then stored as
// computed, non-finite).
template <int DIM, typename TO>
__host__ __device__ inline bool line_factor(const Geo &G, const double *__restrict__ A, TO *__restrict__ lf,
                                            long long l) {
  const LineGeo lg = line_geo<DIM>(G);
  const long long N = G.N;
  double wp[4] = {0.0, 0.0, 0.0, 0.0};  // W_{k-1} in FP64
  bool ok = true;
  for (int k = 0; k < lg.n; ++k) {
    const long long v = l + (long long)k * lg.S;
    double d[4], lo[4], up[4], t[4], gi[4], vv[4], ww[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      d[i] = A[((long long)LineOff<DIM>::C * N + v) * 4 + i];
      lo[i] = A[((long long)LineOff<DIM>::M * N + v) * 4 + i];
      up[i] = A[((long long)LineOff<DIM>::P * N + v) * 4 + i];
    }
    mul22(lo, wp, t);  // L_k D'_{k-1}^{-1} U_{k-1}
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] -= t[i];
    const double det = d[0] * d[3] - d[1] * d[2];
    ok = ok && det != 0.0 && det - det == 0.0;
    gi[0] = d[3] / det;
    gi[1] = -d[1] / det;
    gi[2] = -d[2] / det;
    gi[3] = d[0] / det;
    mul22(gi, lo, vv);
    mul22(gi, up, ww);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      lf[v * 4 + i] = (TO)gi[i];
      lf[(N + v) * 4 + i] = (TO)vv[i];
      lf[(2 * N + v) * 4 + i] = (TO)ww[i];
      wp[i] = ww[i];
    }
  }
  return ok;
}

// One damped line sweep on line l: z = A_L^{-1} r with r = rin, then
// xo = xi + omega z (xi == nullptr: xo = omega z).  c is kept in cbuf, which may be rin
// itself (each chunk's entries are read before they are overwritten); xo is distinct
// from cbuf and xi.  Steps are taken in chunks of CH whose loads are all issued
// before the chunk's recurrence, so a thread keeps CH steps of loads in flight; the
// chunk past the end of the line re-reads its last vertex and stores nothing.
template <int DIM, typename T, typename TO, int CH>
__host__ __device__ inline void line_solve(const Geo &G, const T *__restrict__ lf, const T *rin, T *cbuf,
                                           const T *__restrict__ xi, TO *__restrict__ xo, const T omega,
                                           long long l) {
  const LineGeo lg = line_geo<DIM>(G);
  const long long N = G.N;
  const T *__restrict__ Gb = lf;
  const T *__restrict__ Vb = lf + 4 * N;
  const T *__restrict__ Wb = lf + 8 * N;
  T c0 = 0, c1 = 0;
  for (int k0 = 0; k0 < lg.n; k0 += CH) {
    T gk[CH][4], vk[CH][4], rk[CH][2];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int k = k0 + j < lg.n ? k0 + j : lg.n - 1;
      const long long v = l + (long long)k * lg.S;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gk[j][i] = Gb[v * 4 + i];
        vk[j][i] = Vb[v * 4 + i];
      }
      rk[j][0] = rin[2 * v];
      rk[j][1] = rin[2 * v + 1];
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (k0 + j < lg.n) {
        const long long v = l + (long long)(k0 + j) * lg.S;
        const T a0 = gk[j][0] * rk[j][0] + gk[j][1] * rk[j][1] - (vk[j][0] * c0 + vk[j][1] * c1);
        const T a1 = gk[j][2] * rk[j][0] + gk[j][3] * rk[j][1] - (vk[j][2] * c0 + vk[j][3] * c1);
        c0 = a0;
        c1 = a1;
        cbuf[2 * v] = c0;
        cbuf[2 * v + 1] = c1;
      }
    }
  }
  T z0 = 0, z1 = 0;
  for (int k1 = lg.n - 1; k1 >= 0; k1 -= CH) {
    T wk[CH][4], ck[CH][2], xk[CH][2];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int k = k1 - j >= 0 ? k1 - j : 0;
      const long long v = l + (long long)k * lg.S;
#pragma unroll
      for (int i = 0; i < 4; ++i) wk[j][i] = Wb[v * 4 + i];
      ck[j][0] = cbuf[2 * v];
      ck[j][1] = cbuf[2 * v + 1];
      xk[j][0] = xi ? xi[2 * v] : (T)0;
      xk[j][1] = xi ? xi[2 * v + 1] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (k1 - j >= 0) {
        const long long v = l + (long long)(k1 - j) * lg.S;
        const T a0 = ck[j][0] - (wk[j][0] * z0 + wk[j][1] * z1);
        const T a1 = ck[j][1] - (wk[j][2] * z0 + wk[j][3] * z1);
        z0 = a0;
        z1 = a1;
        xo[2 * v] = (TO)(xk[j][0] + omega * z0);
        xo[2 * v + 1] = (TO)(xk[j][1] + omega * z1);
      }
    }
  }
}

}  // namespace tpf
