// Line-block Jacobi along the last axis of a level (TPF_SMOOTH_LINE): the per-line
// block factorisation and the per-line solve, as __host__ __device__ bodies.
//
// The lines of a level run along its last axis (z in 3D, y in 2D): line l, 0 <= l < S,
// holds the vertices v = l + k S, k = 0 .. n-1, with S = nx ny and n = nz in 3D, S = nx
// and n = ny in 2D.  The couplings of A inside a line form a block tridiagonal matrix
// A_L with L_k = A(k, k-1) (stencil offset -1 along the axis), D_k (the centre) and
// U_k = A(k, k+1) (offset +1); the blocks of neighbours outside the grid are stored as
// zeros, so L_0 = U_{n-1} = 0.
//
// Twisted factorisation about the middle vertex m = n/2: the rows above m are
// eliminated downwards and the rows below m upwards, and the two meet at m.
//   top, k = 0 .. m-1:     D'_0 = D_0, D'_k = D_k - L_k W_{k-1},
//                          G_k = D'_k^{-1}, V_k = G_k L_k, W_k = G_k U_k;
//   bottom, k = n-1 .. m+1: D'_{n-1} = D_{n-1}, D'_k = D_k - U_k V_{k+1},
//                          G_k = D'_k^{-1}, V_k = G_k L_k, W_k = G_k U_k;
//   middle:                D'_m = D_m - L_m W_{m-1} - U_m V_{m+1}, G_m, V_m, W_m alike
// (a term is absent where its neighbour is).  Stored per vertex in the level's type
// as [3][N][4]: G, V, W.  Then A_L z = r is
//   top forward     c_k = G_k r_k - V_k c_{k-1}          (k = 0 .. m-1),
//   bottom forward  c_k = G_k r_k - W_k c_{k+1}          (k = n-1 .. m+1),
//   middle          z_m = G_m r_m - V_m c_{m-1} - W_m c_{m+1},
//   top backward    z_k = c_k - W_k z_{k+1}              (k = m-1 .. 0),
//   bottom backward z_k = c_k - V_k z_{k-1}              (k = m+1 .. n-1),
// so each line is two chains of about n/2 steps, one per thread of a pair.  Pairs are
// lanes l and l + 32 of one wavefront, which exchange c_{m-1} and c_{m+1} by a lane
// shuffle; the 32 lines of a wavefront are consecutive in x, so the loads of one step
// of each half-wavefront are contiguous.
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

// a b + c, rounded once: the factorisation and the recurrences below spell out every
// fused multiply-add, so that each kernel built from them (and the CPU build) rounds
// alike.
__host__ __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// (a0 x0 + a1 x1) for one row of a 2x2 block
template <typename T>
__host__ __device__ __forceinline__ T dot2(T a0, T a1, T x0, T x1) {
  return fma_(a1, x1, a0 * x0);
}

__host__ __device__ __forceinline__ void mul22(const double (&a)[4], const double (&b)[4], double (&c)[4]) {
  c[0] = dot2(a[0], a[1], b[0], b[2]);
  c[1] = dot2(a[0], a[1], b[1], b[3]);
  c[2] = dot2(a[2], a[3], b[0], b[2]);
  c[3] = dot2(a[2], a[3], b[1], b[3]);
}

// Pivot block d (FP64) of vertex v -> G, V = G L, W = G U stored in lf; returns false if d
// is singular or not finite.
template <int DIM, typename TO>
__host__ __device__ __forceinline__ bool line_store(const double (&d)[4], const double (&lo)[4],
                                                   const double (&up)[4], TO *__restrict__ lf, long long N,
                                                   long long v, double (&vv)[4], double (&ww)[4]) {
  const double det = fma_(d[0], d[3], -(d[1] * d[2]));
  double gi[4];
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
  }
  return det != 0.0 && det - det == 0.0;
}

template <int DIM>
__host__ __device__ __forceinline__ void line_blocks(const Geo &G, const double *__restrict__ A, long long v,
                                                    double (&d)[4], double (&lo)[4], double (&up)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    d[i] = A[((long long)LineOff<DIM>::C * G.N + v) * 4 + i];
    lo[i] = A[((long long)LineOff<DIM>::M * G.N + v) * 4 + i];
    up[i] = A[((long long)LineOff<DIM>::P * G.N + v) * 4 + i];
  }
}

// One half of the twisted factorisation of line l from the level's FP64 matrix A
// ([offset][vertex][4]) into lf: top (k = 0 .. m-1) or bottom (k = n-1 .. m+1).  Returns in
// cpl the coupling block the middle row needs (W_{m-1} of the top, V_{m+1} of the
// bottom; zero for an empty half), and false if a pivot block is singular or not finite.
// Steps are taken in chunks of CH whose loads are all issued before the chunk's
// recurrence (a chunk past the end of the half re-reads its last vertex).
template <int DIM, typename TO, int CH>
__host__ __device__ inline bool line_factor_half(const Geo &G, const double *__restrict__ A, TO *__restrict__ lf,
                                                 long long l, bool top, double (&cpl)[4]) {
  const LineGeo lg = line_geo<DIM>(G);
  const long long N = G.N;
  const int m = lg.n / 2;
  const int len = top ? m : lg.n - 1 - m;
  const int k0 = top ? 0 : lg.n - 1, dk = top ? 1 : -1;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 4; ++i) cpl[i] = 0.0;
  for (int j0 = 0; j0 < len; j0 += CH) {
    double d[CH][4], lo[CH][4], up[CH][4];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int jj = j0 + j < len ? j0 + j : len - 1;
      line_blocks<DIM>(G, A, l + (long long)(k0 + dk * jj) * lg.S, d[j], lo[j], up[j]);
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (j0 + j < len) {
        const long long v = l + (long long)(k0 + dk * (j0 + j)) * lg.S;
        double t[4], vv[4], ww[4];
        if (top)
          mul22(lo[j], cpl, t);  // L_k W_{k-1}
        else
          mul22(up[j], cpl, t);  // U_k V_{k+1}
#pragma unroll
        for (int i = 0; i < 4; ++i) d[j][i] -= t[i];
        ok = line_store<DIM, TO>(d[j], lo[j], up[j], lf, N, v, vv, ww) && ok;
#pragma unroll
        for (int i = 0; i < 4; ++i) cpl[i] = top ? ww[i] : vv[i];
      }
    }
  }
  return ok;
}

// The middle vertex of line l, eliminated from both sides with W_{m-1} (wtop) and
// V_{m+1} (vbot).
template <int DIM, typename TO>
__host__ __device__ inline bool line_factor_middle(const Geo &G, const double *__restrict__ A, TO *__restrict__ lf,
                                                   long long l, const double (&wtop)[4], const double (&vbot)[4]) {
  const LineGeo lg = line_geo<DIM>(G);
  const long long v = l + (long long)(lg.n / 2) * lg.S;
  double d[4], lo[4], up[4], t[4], t2[4], vv[4], ww[4];
  line_blocks<DIM>(G, A, v, d, lo, up);
  mul22(lo, wtop, t);
  mul22(up, vbot, t2);
#pragma unroll
  for (int i = 0; i < 4; ++i) d[i] -= t[i] + t2[i];
  return line_store<DIM, TO>(d, lo, up, lf, G.N, v, vv, ww);
}

// Twisted factorisation of line l by one thread (both halves in turn, then the middle).
// Returns false if a pivot block is singular or not finite.
template <int DIM, typename TO, int CH = 4>
__host__ __device__ inline bool line_factor(const Geo &G, const double *__restrict__ A, TO *__restrict__ lf,
                                            long long l) {
  double wtop[4], vbot[4];
  const bool ok_top = line_factor_half<DIM, TO, CH>(G, A, lf, l, true, wtop);
  const bool ok_bot = line_factor_half<DIM, TO, CH>(G, A, lf, l, false, vbot);
  return line_factor_middle<DIM, TO>(G, A, lf, l, wtop, vbot) && ok_top && ok_bot;
}

// Forward chain of one half of line l: top (k = 0 .. m-1, coupling block V) or bottom
// (k = n-1 .. m+1, coupling block W); c is written to cbuf, which may be rin itself
// (each chunk's entries are read before they are overwritten).  Returns the chain's
// last c (c_{m-1} or c_{m+1}; zero for an empty half).  Steps are taken in chunks of
// CH whose loads are all issued before the chunk's recurrence; a chunk past the end
// of the chain re-reads its last vertex and stores nothing.
template <int DIM, typename T, int CH>
__host__ __device__ inline void line_forward(const Geo &G, const T *__restrict__ lf, const T *rin, T *cbuf,
                                             long long l, bool top, T &c0, T &c1) {
  const LineGeo lg = line_geo<DIM>(G);
  const long long N = G.N;
  const int m = lg.n / 2;
  const int len = top ? m : lg.n - 1 - m;
  const int k0 = top ? 0 : lg.n - 1, dk = top ? 1 : -1;
  const T *__restrict__ Gb = lf;
  const T *__restrict__ Cb = lf + (top ? 4 : 8) * N;  // V (top) or W (bottom)
  c0 = 0;
  c1 = 0;
  for (int j0 = 0; j0 < len; j0 += CH) {
    T gk[CH][4], ck[CH][4], rk[CH][2];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int jj = j0 + j < len ? j0 + j : len - 1;
      const long long v = l + (long long)(k0 + dk * jj) * lg.S;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gk[j][i] = Gb[v * 4 + i];
        ck[j][i] = Cb[v * 4 + i];
      }
      rk[j][0] = rin[2 * v];
      rk[j][1] = rin[2 * v + 1];
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (j0 + j < len) {
        const long long v = l + (long long)(k0 + dk * (j0 + j)) * lg.S;
        const T a0 = dot2(gk[j][0], gk[j][1], rk[j][0], rk[j][1]) - dot2(ck[j][0], ck[j][1], c0, c1);
        const T a1 = dot2(gk[j][2], gk[j][3], rk[j][0], rk[j][1]) - dot2(ck[j][2], ck[j][3], c0, c1);
        c0 = a0;
        c1 = a1;
        cbuf[2 * v] = c0;
        cbuf[2 * v + 1] = c1;
      }
    }
  }
}

// z_m of line l from the middle row, given c_{m-1} (ct) and c_{m+1} (cb); r_m is read
// from rin, which neither half overwrites.
template <int DIM, typename T>
__host__ __device__ __forceinline__ void line_middle(const Geo &G, const T *__restrict__ lf, const T *rin,
                                                     long long l, T ct0, T ct1, T cb0, T cb1, T &z0, T &z1) {
  const LineGeo lg = line_geo<DIM>(G);
  const long long N = G.N;
  const long long v = l + (long long)(lg.n / 2) * lg.S;
  T g[4], vv[4], ww[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    g[i] = lf[v * 4 + i];
    vv[i] = lf[(N + v) * 4 + i];
    ww[i] = lf[(2 * N + v) * 4 + i];
  }
  const T r0 = rin[2 * v], r1 = rin[2 * v + 1];
  z0 = dot2(g[0], g[1], r0, r1) - dot2(vv[0], vv[1], ct0, ct1) - dot2(ww[0], ww[1], cb0, cb1);
  z1 = dot2(g[2], g[3], r0, r1) - dot2(vv[2], vv[3], ct0, ct1) - dot2(ww[2], ww[3], cb0, cb1);
}

// Backward chain of one half from z_m: top (k = m-1 .. 0, block W) or bottom
// (k = m+1 .. n-1, block V), writing xo = xi + omega z (xi == nullptr: xo = omega z); the
// top half also writes the middle vertex.  xo is distinct from cbuf and xi.
template <int DIM, typename T, typename TO, int CH>
__host__ __device__ inline void line_backward(const Geo &G, const T *__restrict__ lf, const T *cbuf,
                                              const T *__restrict__ xi, TO *__restrict__ xo, const T omega,
                                              long long l, bool top, T zm0, T zm1) {
  const LineGeo lg = line_geo<DIM>(G);
  const long long N = G.N;
  const int m = lg.n / 2;
  const int len = top ? m : lg.n - 1 - m;
  const int k0 = top ? m - 1 : m + 1, dk = top ? -1 : 1;
  const T *__restrict__ Cb = lf + (top ? 8 : 4) * N;  // W (top) or V (bottom)
  if (top) {
    const long long v = l + (long long)m * lg.S;
    xo[2 * v] = (TO)fma_(omega, zm0, xi ? xi[2 * v] : (T)0);
    xo[2 * v + 1] = (TO)fma_(omega, zm1, xi ? xi[2 * v + 1] : (T)0);
  }
  T z0 = zm0, z1 = zm1;
  for (int j0 = 0; j0 < len; j0 += CH) {
    T wk[CH][4], ck[CH][2], xk[CH][2];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int jj = j0 + j < len ? j0 + j : len - 1;
      const long long v = l + (long long)(k0 + dk * jj) * lg.S;
#pragma unroll
      for (int i = 0; i < 4; ++i) wk[j][i] = Cb[v * 4 + i];
      ck[j][0] = cbuf[2 * v];
      ck[j][1] = cbuf[2 * v + 1];
      xk[j][0] = xi ? xi[2 * v] : (T)0;
      xk[j][1] = xi ? xi[2 * v + 1] : (T)0;
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (j0 + j < len) {
        const long long v = l + (long long)(k0 + dk * (j0 + j)) * lg.S;
        const T a0 = ck[j][0] - dot2(wk[j][0], wk[j][1], z0, z1);
        const T a1 = ck[j][1] - dot2(wk[j][2], wk[j][3], z0, z1);
        z0 = a0;
        z1 = a1;
        xo[2 * v] = (TO)fma_(omega, z0, xk[j][0]);
        xo[2 * v + 1] = (TO)fma_(omega, z1, xk[j][1]);
      }
    }
  }
}

// The whole sweep of line l by one thread (both halves in turn): used where a line
// has no partner lane (the CPU build of the bodies).
template <int DIM, typename T, typename TO, int CH>
__host__ __device__ inline void line_solve(const Geo &G, const T *__restrict__ lf, const T *rin, T *cbuf,
                                           const T *__restrict__ xi, TO *__restrict__ xo, const T omega,
                                           long long l) {
  T t0, t1, b0, b1, z0, z1;
  line_forward<DIM, T, CH>(G, lf, rin, cbuf, l, true, t0, t1);
  line_forward<DIM, T, CH>(G, lf, rin, cbuf, l, false, b0, b1);
  line_middle<DIM, T>(G, lf, rin, l, t0, t1, b0, b1, z0, z1);
  line_backward<DIM, T, TO, CH>(G, lf, cbuf, xi, xo, omega, l, true, z0, z1);
  line_backward<DIM, T, TO, CH>(G, lf, cbuf, xi, xo, omega, l, false, z0, z1);
}

}  // namespace tpf
