// Geometric multigrid on structured vertex grids (gfx950): stencil SpMV, damped 2x2
// point-block Jacobi or line-block Jacobi smoothing (the per-line bodies in line.h),
// residual, restriction (P^T), prolongation, Galerkin coarse operators A_c = P^T A P,
// dense coarsest-level LU with partial pivoting and its inverse, and the V(nu1, nu2)
// cycle used as BiCGSTAB preconditioner.
//
// Matrices are 27-point (3D) / 9-point (2D) stencils of 2x2 blocks stored
// [offset][vertex][4]: for a fixed offset, consecutive lanes read consecutive 16-byte
// (FP32) or 32-byte (FP64) blocks, so every matrix load of a wave is one contiguous
// 1-2 KB segment.  Entries for neighbours outside the grid are stored as zeros and
// never dereference x.  P acts per component between vertex-halved grids: (bi/tri)
// linear interpolation of the pressure, piecewise-constant aggregation of the
// saturation; on the finest level its rows at Dirichlet components are zero.
#include <type_traits>
#include <utility>

#include "line.h"
#include "stencil.h"

namespace tpf {
namespace {

// Offsets per group of the branch-free row product: every matrix block and x value
// of a group is loaded before any of them is used, so a wave keeps a group's loads in
// flight together instead of waiting on each offset in turn.
#ifndef TPF_ROW_GROUP32
#define TPF_ROW_GROUP32 9
#endif
#ifndef TPF_ROW_GROUP64
#define TPF_ROW_GROUP64 9
#endif

typedef float tpf_f4 __attribute__((ext_vector_type(4)));
typedef double tpf_d2 __attribute__((ext_vector_type(2)));
typedef _Float16 tpf_h4 __attribute__((ext_vector_type(4)));

// One FP16-stored 2x2 block (raw entries, before the row scales), as floats.
__device__ __forceinline__ void load_block16(const uint16_t *p, float (&b)[4]) {
  const tpf_h4 a = *reinterpret_cast<const tpf_h4 *>(p);
  b[0] = (float)a.x; b[1] = (float)a.y; b[2] = (float)a.z; b[3] = (float)a.w;
}

// One 2x2 block; NT: non-temporal load for a matrix streamed once per sweep from HBM
// (the finest level), which leaves the caches to the x gathers.
template <typename T, bool NT>
__device__ __forceinline__ void load_block(const T *p, T (&b)[4]) {
  if constexpr (NT && sizeof(T) == 4) {
    const tpf_f4 a = __builtin_nontemporal_load(reinterpret_cast<const tpf_f4 *>(p));
    b[0] = a.x; b[1] = a.y; b[2] = a.z; b[3] = a.w;
  } else if constexpr (NT) {
    const tpf_d2 a = __builtin_nontemporal_load(reinterpret_cast<const tpf_d2 *>(p));
    const tpf_d2 c = __builtin_nontemporal_load(reinterpret_cast<const tpf_d2 *>(p) + 1);
    b[0] = a.x; b[1] = a.y; b[2] = c.x; b[3] = c.y;
  } else {
    Blk<T>::load(p, b);
  }
}

// y = A x (row-block product) accumulated in the matrix type T for one vertex.
// Returns (A x)_v; the centre block (and, if xc is given, the centre x value) is
// copied out for the smoother, which then needs no load after the row.  Neighbours
// outside the grid have zero blocks; their x value is read at the clamped (valid)
// position and masked to zero, so no load depends on a branch.
// SKIPLINE: the row of A - A_L, without the three blocks that couple the vertex with
// itself and its two neighbours along the last axis (the line part; no loads for them).
template <int DIM, typename T, typename TX, bool NT = false, bool TILED = false, int GROUP = 0, typename AS = T,
          bool SKIPLINE = false>
__device__ __forceinline__ void row_apply(const Geo &G, long long v, const AS *__restrict__ A,
                                          const TX *__restrict__ x, T &y0, T &y1, T (&dblk)[4],
                                          T *xc = nullptr) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  constexpr int CEN = DIM == 3 ? 13 : 4;
  constexpr int GRP0 = GROUP > 0 ? GROUP : (sizeof(T) == 4 ? TPF_ROW_GROUP32 : TPF_ROW_GROUP64);
  constexpr int GRP = GRP0 > NST ? NST : GRP0;
  static_assert(NST % GRP == 0, "group size must divide the stencil size");
  int ix, iy, iz;
  vcoords(v, G, ix, iy, iz);
  const long long sy = G.nx, sz = (long long)G.nx * G.ny;
  const bool okx[3] = {ix > 0, true, ix < G.nx - 1};
  const bool oky[3] = {iy > 0, true, iy < G.ny - 1};
  const bool okz[3] = {DIM == 3 && iz > 0, true, DIM == 3 && iz < G.nz - 1};
  const long long offx[3] = {okx[0] ? -1 : 0, 0, okx[2] ? 1 : 0};
  const long long offy[3] = {oky[0] ? -sy : 0, 0, oky[2] ? sy : 0};
  const long long offz[3] = {okz[0] ? -sz : 0, 0, okz[2] ? sz : 0};
  using X2 = typename Vec2<TX>::type;
  T a0 = 0, a1 = 0;
#pragma unroll
  for (int g0 = 0; g0 < NST; g0 += GRP) {
    T b[GRP][4];
    X2 xv[GRP];
#pragma unroll
    for (int k = 0; k < GRP; ++k) {
      const int o = g0 + k;
      const int ax = o % 3, ay = (o / 3) % 3, az = DIM == 3 ? o / 9 : 1;
      if (SKIPLINE && (DIM == 3 ? o % 9 == 4 : o % 3 == 1)) continue;
      if constexpr (sizeof(AS) == 2)
        load_block16(A + ((long long)o * G.N + v) * 4, b[k]);
      else
        load_block<T, NT>(A + (TILED ? tiled_block(o, v, NST) : (long long)o * G.N + v) * 4, b[k]);
      xv[k] = *reinterpret_cast<const X2 *>(x + 2 * (v + offx[ax] + offy[ay] + offz[az]));
    }
#pragma unroll
    for (int k = 0; k < GRP; ++k) {
      const int o = g0 + k;
      const int ax = o % 3, ay = (o / 3) % 3, az = DIM == 3 ? o / 9 : 1;
      if (SKIPLINE && (DIM == 3 ? o % 9 == 4 : o % 3 == 1)) continue;
      if (o == CEN) {
        dblk[0] = b[k][0]; dblk[1] = b[k][1]; dblk[2] = b[k][2]; dblk[3] = b[k][3];
        if (xc) {
          xc[0] = (T)xv[k].x;
          xc[1] = (T)xv[k].y;
        }
      }
      const bool ok = okx[ax] && oky[ay] && okz[az];
      const T x0 = ok ? (T)xv[k].x : (T)0, x1 = ok ? (T)xv[k].y : (T)0;
      a0 += b[k][0] * x0 + b[k][1] * x1;
      a1 += b[k][2] * x0 + b[k][3] * x1;
    }
  }
  y0 = a0;
  y1 = a1;
}

template <typename T>
__device__ __forceinline__ void solve2(const T (&d)[4], T r0, T r1, T &z0, T &z1) {
  const T det = d[0] * d[3] - d[1] * d[2];
  z0 = (d[3] * r0 - d[1] * r1) / det;
  z1 = (d[0] * r1 - d[2] * r0) / det;
}

// ---- block-level reduction helpers (deterministic: fixed tree) ------------------
template <int NDOT>
__device__ __forceinline__ void block_reduce_store(double (&val)[NDOT], double *__restrict__ part,
                                                   unsigned blk, unsigned nblk) {
  __shared__ double sm[NDOT][BS / 64];
#pragma unroll
  for (int k = 0; k < NDOT; ++k) {
    double s = val[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < NDOT) {
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < BS / 64; ++wv) s += sm[threadIdx.x][wv];
    part[(long long)threadIdx.x * nblk + blk] = s;
  }
}

// y = A x (FP64); optionally partial dots (d0, y) [MODE 1], (d0,y),(y,y) [MODE 2],
// or the residual y = b - A x with partial (y, y) [MODE 3].
template <int DIM, int MODE>
__global__ void __launch_bounds__(BS) k_spmv64(const Geo G, const double *__restrict__ A,
                                               const double *__restrict__ x, double *__restrict__ y,
                                               const double *__restrict__ d0, double *__restrict__ part) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long v = (long long)blk * BS + threadIdx.x;
  double acc[MODE == 2 ? 2 : 1];
  acc[0] = 0.0;
  if (MODE == 2) acc[MODE == 2 ? 1 : 0] = 0.0;
  if (v < G.N) {
    double y0, y1, dd[4];
    // the vector operand d0 (dot partner or right-hand side) is loaded before the
    // row, and all 27 blocks of the row are in flight at once (379 -> 374 us at 129^3)
    double2 w = make_double2(0.0, 0.0);
    if (MODE != 0) w = *reinterpret_cast<const double2 *>(d0 + 2 * v);
    row_apply<DIM, double, double, false, false, DIM == 3 ? 27 : 9>(G, v, A, x, y0, y1, dd);
    if (MODE == 3) {
      y0 = w.x - y0;
      y1 = w.y - y1;
    }
    *reinterpret_cast<double2 *>(y + 2 * v) = make_double2(y0, y1);
    if (MODE == 1 || MODE == 2) {
      acc[0] = w.x * y0 + w.y * y1;
      if (MODE == 2) acc[MODE == 2 ? 1 : 0] = y0 * y0 + y1 * y1;
    }
    if (MODE == 3) acc[0] = y0 * y0 + y1 * y1;
  }
  if (MODE != 0) block_reduce_store<MODE == 2 ? 2 : 1>(acc, part, blk, gridDim.x);
}

// Damped block Jacobi update of one vertex: xo = xi + omega D^{-1} (b - A xi);
// FIRST: xi = 0, so only the diagonal block is read.
// LAT (the small, latency-bound coarse levels): all loads of the row are issued
// together, before any is used, so a sweep costs one memory round trip.
template <int DIM, typename T, typename TO, bool FIRST, bool NT = false, bool TILED = false, bool LAT = false>
__device__ __forceinline__ void jacobi_vertex(const Geo &G, const T *__restrict__ A, const T *__restrict__ b,
                                              const T *__restrict__ xi, TO *__restrict__ xo, const T omega,
                                              long long v) {
  constexpr int CEN = DIM == 3 ? 13 : 4;
  constexpr int NST = DIM == 3 ? 27 : 9;
  T r0, r1, d[4], x0 = 0, x1 = 0;
  if (FIRST) {
    Blk<T>::load(A + (TILED ? tiled_block(CEN, v, DIM == 3 ? 27 : 9) : (long long)CEN * G.N + v) * 4, d);
    const auto bb = *reinterpret_cast<const typename Vec2<T>::type *>(b + 2 * v);
    r0 = bb.x;
    r1 = bb.y;
  } else if (LAT) {
    const auto bb = *reinterpret_cast<const typename Vec2<T>::type *>(b + 2 * v);
    const auto xx = *reinterpret_cast<const typename Vec2<T>::type *>(xi + 2 * v);
    T a0, a1;
    row_apply<DIM, T, T, NT, TILED, NST>(G, v, A, xi, a0, a1, d);
    x0 = xx.x;
    x1 = xx.y;
    r0 = bb.x - a0;
    r1 = bb.y - a1;
  } else {
    T a0, a1, xc[2];
    row_apply<DIM, T, T, NT, TILED>(G, v, A, xi, a0, a1, d, xc);  // centre x from the row's gather
    typename Vec2<T>::type bb;
    if constexpr (NT && TILED) {  // streaming sweep: b is read once
      bb.x = __builtin_nontemporal_load(b + 2 * v);
      bb.y = __builtin_nontemporal_load(b + 2 * v + 1);
    } else {
      bb = *reinterpret_cast<const typename Vec2<T>::type *>(b + 2 * v);
    }
    x0 = xc[0];
    x1 = xc[1];
    r0 = bb.x - a0;
    r1 = bb.y - a1;
  }
  T z0, z1;
  solve2<T>(d, r0, r1, z0, z1);
  if constexpr (NT && TILED) {  // streaming sweep: the result bypasses the caches
    __builtin_nontemporal_store((TO)(x0 + omega * z0), xo + 2 * v);
    __builtin_nontemporal_store((TO)(x1 + omega * z1), xo + 2 * v + 1);
  } else {
    typename Vec2<TO>::type out;
    out.x = (TO)(x0 + omega * z0);
    out.y = (TO)(x1 + omega * z1);
    *reinterpret_cast<typename Vec2<TO>::type *>(xo + 2 * v) = out;
  }
}

template <int DIM, typename T, typename TO, bool FIRST, bool NT = false, bool TILED = false, bool LAT = false>
__global__ void __launch_bounds__(BS) k_jacobi(const Geo G, const T *__restrict__ A,
                                               const T *__restrict__ b, const T *__restrict__ xi,
                                               TO *__restrict__ xo, const T omega) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long v = (long long)blk * BS + threadIdx.x;
  if (v >= G.N) return;
  jacobi_vertex<DIM, T, TO, FIRST, NT, TILED, LAT>(G, A, b, xi, xo, omega, v);
}

// The finest-level FP32 sweeps stream a matrix far larger than the caches: they
// use non-temporal matrix and right-hand-side loads and non-temporal stores of
// their result (measured: 185 -> 179 us per 129^3 sweep against plain stores), take
// the centre x from the row's own gather instead of loading it again after the row
// (179 -> 173 us: one memory round trip less per wavefront), and
// a register budget that keeps enough wavefronts per SIMD in flight to cover HBM
// latency.  The FP64 SpMV keeps cached loads: its [offset][vertex] matrix is 27
// separate streams, which non-temporal loads slow down (378 -> 466 us).
#ifndef TPF_STREAM_WAVES
#define TPF_STREAM_WAVES 0
#endif
#if TPF_STREAM_WAVES > 0
#define TPF_STREAM_ATTR __attribute__((amdgpu_waves_per_eu(TPF_STREAM_WAVES, 8)))
#else
#define TPF_STREAM_ATTR
#endif

template <int DIM, typename T, typename TO>
__global__ void __launch_bounds__(BS) TPF_STREAM_ATTR k_jacobi_stream(const Geo G, const T *__restrict__ A,
                                                                      const T *__restrict__ b,
                                                                      const T *__restrict__ xi,
                                                                      TO *__restrict__ xo, const T omega) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long v = (long long)blk * BS + threadIdx.x;
  if (v >= G.N) return;
  jacobi_vertex<DIM, T, TO, false, true, true>(G, A, b, xi, xo, omega, v);
}

// r = b - A x at one vertex of a level.  OFFLINE: r = bscale b - (A - A_L) x, which is
// b - A x for x = omega A_L^{-1} b and bscale = 1 - omega (A_L x = omega b): the
// residual after a line sweep from a zero guess, without the line blocks.
template <int DIM, typename T, bool NT = false, bool TILED = false, bool LAT = false, bool OFFLINE = false>
__device__ __forceinline__ void resid_vertex(const Geo &G, const T *__restrict__ A, const T *__restrict__ b,
                                             const T *__restrict__ x, T *__restrict__ r, long long v,
                                             T bscale = (T)1) {
  T a0, a1, d[4];
  typename Vec2<T>::type bb;
  if (LAT) bb = *reinterpret_cast<const typename Vec2<T>::type *>(b + 2 * v);
  row_apply<DIM, T, T, NT, TILED, LAT ? (DIM == 3 ? 27 : 9) : 0, T, OFFLINE>(G, v, A, x, a0, a1, d);
  if (!LAT) bb = *reinterpret_cast<const typename Vec2<T>::type *>(b + 2 * v);
  if constexpr (OFFLINE) {
    bb.x *= bscale;
    bb.y *= bscale;
  }
  if constexpr (NT && TILED) {  // streaming residual: the result bypasses the caches
    __builtin_nontemporal_store(bb.x - a0, r + 2 * v);
    __builtin_nontemporal_store(bb.y - a1, r + 2 * v + 1);
  } else {
    typename Vec2<T>::type o;
    o.x = bb.x - a0;
    o.y = bb.y - a1;
    *reinterpret_cast<typename Vec2<T>::type *>(r + 2 * v) = o;
  }
}

template <int DIM, typename T, bool OFFLINE = false>
__global__ void __launch_bounds__(BS) TPF_STREAM_ATTR k_resid_stream(const Geo G, const T *__restrict__ A,
                                                                     const T *__restrict__ b,
                                                                     const T *__restrict__ x, T *__restrict__ r,
                                                                     const T bscale);

template <int DIM, typename T, bool NT = false, bool LAT = false, bool OFFLINE = false>
__global__ void __launch_bounds__(BS) k_resid(const Geo G, const T *__restrict__ A, const T *__restrict__ b,
                                              const T *__restrict__ x, T *__restrict__ r, const T bscale) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long v = (long long)blk * BS + threadIdx.x;
  if (v >= G.N) return;
  resid_vertex<DIM, T, NT, false, LAT, OFFLINE>(G, A, b, x, r, v, bscale);
}

template <int DIM, typename T, bool OFFLINE>
__global__ void __launch_bounds__(BS) TPF_STREAM_ATTR k_resid_stream(const Geo G, const T *__restrict__ A,
                                                                     const T *__restrict__ b,
                                                                     const T *__restrict__ x, T *__restrict__ r,
                                                                     const T bscale) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long v = (long long)blk * BS + threadIdx.x;
  if (v >= G.N) return;
  resid_vertex<DIM, T, true, true, false, OFFLINE>(G, A, b, x, r, v, bscale);
}

// Coarse levels stored in FP16 with a scale per scalar row (TPF_MIXED16): the raw
// row product is multiplied by the row scales, and so is the diagonal block.
template <int DIM, bool FIRST>
__global__ void __launch_bounds__(BS) k_jacobi16(const Geo G, const uint16_t *__restrict__ A,
                                                 const float *__restrict__ sc, const float *__restrict__ b,
                                                 const float *__restrict__ xi, float *__restrict__ xo,
                                                 const float omega) {
  constexpr int CEN = DIM == 3 ? 13 : 4;
  constexpr int NST = DIM == 3 ? 27 : 9;
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long v = (long long)blk * BS + threadIdx.x;
  if (v >= G.N) return;
  const float2 s = *reinterpret_cast<const float2 *>(sc + 2 * v);
  const float2 bb = *reinterpret_cast<const float2 *>(b + 2 * v);
  float d[4], r0, r1, x0 = 0.f, x1 = 0.f;
  if (FIRST) {
    load_block16(A + ((long long)CEN * G.N + v) * 4, d);
    r0 = bb.x;
    r1 = bb.y;
  } else {
    const float2 xx = *reinterpret_cast<const float2 *>(xi + 2 * v);
    float a0, a1;
    row_apply<DIM, float, float, false, false, NST, uint16_t>(G, v, A, xi, a0, a1, d);
    x0 = xx.x;
    x1 = xx.y;
    r0 = bb.x - s.x * a0;
    r1 = bb.y - s.y * a1;
  }
  d[0] *= s.x; d[1] *= s.x; d[2] *= s.y; d[3] *= s.y;
  float z0, z1;
  solve2<float>(d, r0, r1, z0, z1);
  *reinterpret_cast<float2 *>(xo + 2 * v) = make_float2(x0 + omega * z0, x1 + omega * z1);
}

template <int DIM>
__global__ void __launch_bounds__(BS) k_resid16(const Geo G, const uint16_t *__restrict__ A,
                                                const float *__restrict__ sc, const float *__restrict__ b,
                                                const float *__restrict__ x, float *__restrict__ r) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long v = (long long)blk * BS + threadIdx.x;
  if (v >= G.N) return;
  const float2 s = *reinterpret_cast<const float2 *>(sc + 2 * v);
  const float2 bb = *reinterpret_cast<const float2 *>(b + 2 * v);
  float a0, a1, d[4];
  row_apply<DIM, float, float, false, false, NST, uint16_t>(G, v, A, x, a0, a1, d);
  *reinterpret_cast<float2 *>(r + 2 * v) = make_float2(bb.x - s.x * a0, bb.y - s.y * a1);
}

// FP64 level matrix -> FP16 blocks with one scale per scalar row (the row's largest
// magnitude, 1 for an all-zero row), one thread per vertex.
template <int DIM>
__global__ void __launch_bounds__(BS) k_to16(const Geo G, const double *__restrict__ A, uint16_t *__restrict__ A16,
                                             float *__restrict__ sc) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= G.N) return;
  double m0 = 0.0, m1 = 0.0;
  for (int o = 0; o < NST; ++o) {
    const double *p = A + ((long long)o * G.N + v) * 4;
    m0 = fmax(m0, fmax(fabs(p[0]), fabs(p[1])));
    m1 = fmax(m1, fmax(fabs(p[2]), fabs(p[3])));
  }
  const float s0 = m0 > 0.0 ? (float)m0 : 1.f, s1 = m1 > 0.0 ? (float)m1 : 1.f;
  *reinterpret_cast<float2 *>(sc + 2 * v) = make_float2(s0, s1);
  for (int o = 0; o < NST; ++o) {
    const double *p = A + ((long long)o * G.N + v) * 4;
    tpf_h4 h;
    h.x = (_Float16)(float)(p[0] / s0);
    h.y = (_Float16)(float)(p[1] / s0);
    h.z = (_Float16)(float)(p[2] / s1);
    h.w = (_Float16)(float)(p[3] / s1);
    *reinterpret_cast<tpf_h4 *>(A16 + ((long long)o * G.N + v) * 4) = h;
  }
}

// Stored FP16 entries times their row scales, [offset][vertex][4] floats.
__global__ void k_expand16(const uint16_t *__restrict__ A16, const float *__restrict__ sc, float *__restrict__ dst,
                           long long N, int nst) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nst * N) return;
  const long long v = t % N;
  float b[4];
  load_block16(A16 + t * 4, b);
  const float2 s = *reinterpret_cast<const float2 *>(sc + 2 * v);
  *reinterpret_cast<float4 *>(dst + t * 4) = make_float4(b[0] * s.x, b[1] * s.x, b[2] * s.y, b[3] * s.y);
}

// Restriction bc = P^T rf.  Pressure component: (bi/tri)linear weights
// (1/2)^{|d|_1} over the 3^d fine neighbours of vertex 2I.  Saturation component:
// piecewise-constant aggregation, the sum over fine vertices 2I + d, d in {-1, 0}^d.
// On the finest level (fmask given) Dirichlet components are excluded and the
// residual enters in the volume-balance form of the Galerkin product: at vertices
// without Dirichlet components the wetting entry becomes r_w + vr r_n.
template <int DIM, typename T>
__host__ __device__ __forceinline__ typename Vec2<T>::type restrict_vertex(long long I, const Geo &F, const Geo &C,
                                                                          const T *__restrict__ rf,
                                                                          const uint8_t *__restrict__ fmask,
                                                                          const T vr, T *__restrict__ bc) {
  // branch-free: all 3^d neighbours are loaded (out-of-grid ones at a clamped, valid
  // position, with weight 0) before any is used; summation order dz, dy, dx
  constexpr int NP = DIM == 3 ? 27 : 9;
  int cx, cy, cz;
  vcoords(I, C, cx, cy, cz);
  const int fx = 2 * cx, fy = 2 * cy, fz = DIM == 3 ? 2 * cz : 0;
  typename Vec2<T>::type rv[NP];
  uint8_t mk[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = DIM == 3 ? k / 9 - 1 : 0;
    const int xr = fx + dx, yr = fy + dy, zr = fz + dz;
    const int x = xr < 0 ? 0 : (xr >= F.nx ? F.nx - 1 : xr);
    const int y = yr < 0 ? 0 : (yr >= F.ny ? F.ny - 1 : yr);
    const int z = zr < 0 ? 0 : (zr >= F.nz ? F.nz - 1 : zr);
    const long long i = x + (long long)F.nx * (y + (long long)F.ny * z);
    rv[k] = *reinterpret_cast<const typename Vec2<T>::type *>(rf + 2 * i);
    mk[k] = fmask ? fmask[i] : (uint8_t)0;
  }
  T s0 = 0, s1 = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = DIM == 3 ? k / 9 - 1 : 0;
    const bool in = fx + dx >= 0 && fx + dx < F.nx && fy + dy >= 0 && fy + dy < F.ny && fz + dz >= 0 &&
                    fz + dz < F.nz;
    T r0 = rv[k].x, r1 = rv[k].y;
    if (fmask) {
      const uint8_t m = mk[k];
      if (!m) r0 += vr * r1;
      if (m & 1) r0 = 0;
      if (m & 2) r1 = 0;
    }
    const T wl = in ? (T)((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0)) : (T)0;
    const T wc = (in && dx <= 0 && dy <= 0 && dz <= 0) ? (T)1 : (T)0;
    s0 += wl * r0;
    s1 += wc * r1;
  }
  typename Vec2<T>::type o;
  o.x = s0;
  o.y = s1;
  *reinterpret_cast<typename Vec2<T>::type *>(bc + 2 * I) = o;
  return o;
}

template <int DIM, typename T>
__global__ void __launch_bounds__(BS) k_restrict(const Geo F, const Geo C, const T *__restrict__ rf,
                                                 const uint8_t *__restrict__ fmask, const T vr,
                                                 T *__restrict__ bc) {
  const long long I = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= C.N) return;
  restrict_vertex<DIM, T>(I, F, C, rf, fmask, vr, bc);
}

// Restriction followed by the coarse level's first sweep from a zero guess,
// xc = 0 + omega D_c^{-1} bc, which needs only the vertex's own restricted value and
// centre block: one launch instead of two on every level that is smoothed.  The
// arithmetic is that of the separate first sweep, so the results are identical.  On
// the small levels the finest level's streams have evicted the level's matrix from
// L2 since the last cycle; the kernel loads each vertex's whole row alongside its
// centre block (one cold round trip for both), with the sweeps' vertex-to-XCD mapping,
// so that the next, full sweep finds it in the same L2.
template <int DIM, typename T>
__global__ void __launch_bounds__(BS) k_restrict_first(const Geo F, const Geo C, const T *__restrict__ rf,
                                                       const uint8_t *__restrict__ fmask, const T vr,
                                                       T *__restrict__ bc, const T *__restrict__ Ac,
                                                       T *__restrict__ xc, const T omega) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);  // the sweeps' vertex-to-XCD mapping
  const long long I = (long long)blk * blockDim.x + threadIdx.x;
  if (I >= C.N) return;
  constexpr int CEN = DIM == 3 ? 13 : 4;
  constexpr int NST = DIM == 3 ? 27 : 9;
  T d[4];
  Blk<T>::load(Ac + ((long long)CEN * C.N + I) * 4, d);
  if (C.N <= 65536) {  // small level: bring the whole row into this XCD's L2 for the next sweep
    T q[NST][4];
#pragma unroll
    for (int o = 0; o < NST; ++o) Blk<T>::load(Ac + ((long long)o * C.N + I) * 4, q[o]);
    T touch = 0;
#pragma unroll
    for (int o = 0; o < NST; ++o) touch += q[o][0];
    // the loads exist only for their side effect on the cache: an empty asm statement
    // that takes their sum as an operand makes the compiler keep them
    asm volatile("" ::"v"(touch));
  }
  const auto o = restrict_vertex<DIM, T>(I, F, C, rf, fmask, vr, bc);
  T z0, z1;
  solve2<T>(d, o.x, o.y, z0, z1);
  const T x0 = 0, x1 = 0;
  typename Vec2<T>::type out;
  out.x = x0 + omega * z0;
  out.y = x1 + omega * z1;
  *reinterpret_cast<typename Vec2<T>::type *>(xc + 2 * I) = out;
}

// Prolongation and correction xf += P ec: linear interpolation of the pressure
// correction, injection from the aggregating coarse vertex ((i + 1) / 2 per axis)
// of the saturation correction.
template <int DIM, typename T>
__host__ __device__ __forceinline__ void prolong_vertex(long long i, const Geo &F, const Geo &C,
                                                       const T *__restrict__ ec,
                                                       const uint8_t *__restrict__ fmask, T *__restrict__ xf) {
  // branch-free: x and the mask first, then the 2^d coarse pressure values (an even
  // fine index takes the same coarse vertex twice, once with weight 0)
  auto xv = *reinterpret_cast<typename Vec2<T>::type *>(xf + 2 * i);
  const uint8_t m = fmask ? fmask[i] : (uint8_t)0;
  int x, y, z;
  vcoords(i, F, x, y, z);
  const int xl = x >> 1, xh = (x + 1) >> 1, yl = y >> 1, yh = (y + 1) >> 1;
  const int zl = DIM == 3 ? z >> 1 : 0, zh = DIM == 3 ? (z + 1) >> 1 : 0;
  // per axis: weight of the lower and the upper coarse vertex
  const T hx = (x & 1) ? (T)0.5 : (T)1, hy = (y & 1) ? (T)0.5 : (T)1;
  const T hz = (DIM == 3 && (z & 1)) ? (T)0.5 : (T)1;
  const T ox = (x & 1) ? (T)0.5 : (T)0, oy = (y & 1) ? (T)0.5 : (T)0;
  const T oz = (DIM == 3 && (z & 1)) ? (T)0.5 : (T)0;
  const long long sy = C.nx, sz = (long long)C.nx * C.ny;
  constexpr int NK = DIM == 3 ? 8 : 4;
  T v[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int X = (k & 1) ? xh : xl, Y = (k & 2) ? yh : yl, Z = (k & 4) ? zh : zl;
    v[k] = ec[2 * (X + sy * Y + sz * Z)];
  }
  T s1 = ec[2 * (xh + sy * yh + sz * zh) + 1];  // saturation: the aggregating coarse vertex
  T s0 = 0;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const T w = ((k & 1) ? ox : hx) * ((k & 2) ? oy : hy) * (DIM == 3 ? ((k & 4) ? oz : hz) : (T)1);
    s0 += w * v[k];
  }
  if (m & 1) s0 = 0;
  if (m & 2) s1 = 0;
  xv.x += s0;
  xv.y += s1;
  *reinterpret_cast<typename Vec2<T>::type *>(xf + 2 * i) = xv;
}

template <int DIM, typename T>
__global__ void __launch_bounds__(BS) k_prolong(const Geo F, const Geo C, const T *__restrict__ ec,
                                                const uint8_t *__restrict__ fmask, T *__restrict__ xf) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long i = (long long)blk * BS + threadIdx.x;
  if (i >= F.N) return;
  prolong_vertex<DIM, T>(i, F, C, ec, fmask, xf);
}

// Dense coarsest matrix (column-major n x n, n = 2 N) from the stencil rows.
template <int DIM>
__global__ void k_densify(const Geo G, const double *__restrict__ A, double *__restrict__ D, int n) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)NST * G.N) return;
  const int o = (int)(t / G.N);
  const long long v = t % G.N;
  const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = DIM == 3 ? o / 9 - 1 : 0;
  int ix, iy, iz;
  vcoords(v, G, ix, iy, iz);
  const int x = ix + dx, y = iy + dy, z = iz + dz;
  if (x < 0 || y < 0 || z < 0 || x >= G.nx || y >= G.ny || z >= G.nz) return;
  const long long j = x + (long long)G.nx * (y + (long long)G.ny * z);
  const double *b = A + ((long long)o * G.N + v) * 4;
  D[(2 * j) * (long long)n + 2 * v] = b[0];
  D[(2 * j + 1) * (long long)n + 2 * v] = b[1];
  D[(2 * j) * (long long)n + 2 * v + 1] = b[2];
  D[(2 * j + 1) * (long long)n + 2 * v + 1] = b[3];
}

__global__ void k_zero(double *p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void k_zero_int(int *p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Blocked right-looking LU with partial pivoting of the column-major n x n coarsest
// matrix (P A = L U, L unit lower, both factors in place), in panels of LU_NB
// columns: the panel is factored by one workgroup, its row interchanges are then
// applied to the other columns, the block row of U is solved with the panel's unit
// lower triangle and the trailing matrix updated by a tiled product.  The pivot of a
// column is its largest magnitude below the diagonal, ties going to the lowest row.
constexpr int LU_NB = 32;

__global__ void __launch_bounds__(1024) k_lu_panel(double *__restrict__ a, int n, int j0, int w,
                                                   int *__restrict__ piv) {
  __shared__ double wbest[16];
  __shared__ int wrow[16];
  __shared__ int sp;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int c = 0; c < w; ++c) {
    const int k = j0 + c;
    double *colk = a + (long long)k * n;
    double best = -1.0;
    int bi = k;  // a column without a comparable entry (NaN) keeps its own row
    for (int i = k + tid; i < n; i += 1024) {  // ascending rows: strict > keeps the lowest
      const double v = fabs(colk[i]);
      if (v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_down(best, off, 64);
      const int oi = __shfl_down(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { wbest[wv] = best; wrow[wv] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b0 = wbest[0];
      int r0 = wrow[0];
      for (int q = 1; q < 16; ++q)
        if (wbest[q] > b0 || (wbest[q] == b0 && wrow[q] < r0)) { b0 = wbest[q]; r0 = wrow[q]; }
      sp = r0;
      piv[k] = r0;
    }
    __syncthreads();
    const int p = sp;
    if (p != k && tid < w) {  // interchange rows k and p inside the panel
      double *col = a + (long long)(j0 + tid) * n;
      const double t = col[k];
      col[k] = col[p];
      col[p] = t;
    }
    __syncthreads();
    const double inv = 1.0 / colk[k];
    for (int i = k + 1 + tid; i < n; i += 1024) {
      const double l = colk[i] * inv;
      colk[i] = l;
      for (int cc = c + 1; cc < w; ++cc) {
        double *colj = a + (long long)(j0 + cc) * n;
        colj[i] -= l * colj[k];
      }
    }
    __syncthreads();
  }
}

// (best, bi) <- the larger of (best, bi) and (ob, oi): larger magnitude first, then the
// lower row (a total order, so any reduction order gives the same pivot)
__device__ __forceinline__ void amax_take(double &best, int &bi, double ob, int oi) {
  const bool take = (ob > best) | ((ob == best) & (oi < bi));
  best = take ? ob : best;
  bi = take ? oi : bi;
}

// One step of a prefix maximum within each 16-lane row: lane i meets lane i - K (DPP
// row shift; lanes without a source keep their own pair).
template <int K>
__device__ __forceinline__ void amax_row_step(double &best, int &bi) {
  constexpr int CTRL = 0x110 + K;  // row_shr:K
  const unsigned long long b = __builtin_bit_cast(unsigned long long, best);
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)b, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(b >> 32), (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf,
                                             false);
  const int oi = __builtin_amdgcn_update_dpp(bi, bi, CTRL, 0xf, 0xf, false);
  const double ob = __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
  amax_take(best, bi, ob, oi);
}

// The wavefront's maximum pair, in every lane: row prefix maxima by DPP (lanes 15, 31,
// 47 and 63 then hold their rows' maxima), combined from those lanes by readlane.  All
// 64 lanes must be active (the panel kernels launch whole wavefronts and call this with
// uniform control flow).
__device__ __forceinline__ void amax_wave(double &best, int &bi) {
  amax_row_step<1>(best, bi);
  amax_row_step<2>(best, bi);
  amax_row_step<4>(best, bi);
  amax_row_step<8>(best, bi);
  const unsigned long long b = __builtin_bit_cast(unsigned long long, best);
  const int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
  double wb[4];
  int wi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const unsigned l = (unsigned)__builtin_amdgcn_readlane(lo, 16 * k + 15);
    const unsigned h = (unsigned)__builtin_amdgcn_readlane(hi, 16 * k + 15);
    wb[k] = __builtin_bit_cast(double, ((unsigned long long)h << 32) | l);
    wi[k] = __builtin_amdgcn_readlane(bi, 16 * k + 15);
  }
  best = wb[0];
  bi = wi[0];
#pragma unroll
  for (int k = 1; k < 4; ++k) amax_take(best, bi, wb[k], wi[k]);
}

// One column step of k_lu_panel_reg, column C of the panel held in x (row r).
template <int ROWS, int C>
__device__ __forceinline__ void lu_panel_column(double (&x)[LU_NB], int r, int m, int j0, int w,
                                                int *__restrict__ piv, double (*prow)[LU_NB],
                                                double (*crow)[LU_NB], double (*wbest)[ROWS / 64],
                                                int (*wrow)[ROWS / 64]) {
  constexpr int NW = ROWS / 64, q = C & 1;
  if (C >= w) return;
  const int lane = r & 63, wv = r >> 6;
  const bool in = r < m;
  double best = -1.0;
  int bi = C;  // a column without a comparable entry (NaN) keeps its own row
  if (in && r >= C) {
    best = fabs(x[C]);
    bi = r;
  }
  amax_wave(best, bi);
  if (lane == 0) {
    wbest[q][wv] = best;
    wrow[q][wv] = bi;
  }
  __syncthreads();
  double wb[NW];
  int wi[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) {  // all loads first, then the comparisons
    wb[k] = wbest[q][k];
    wi[k] = wrow[q][k];
  }
  best = wb[0];
  bi = wi[0];
#pragma unroll
  for (int k = 1; k < NW; ++k) amax_take(best, bi, wb[k], wi[k]);
  const int p = __builtin_amdgcn_readfirstlane(bi);
  if (r == p) {
#pragma unroll
    for (int cc = 0; cc < LU_NB; ++cc) prow[q][cc] = x[cc];
  }
  if (r == C) {
#pragma unroll
    for (int cc = 0; cc < LU_NB; ++cc) crow[q][cc] = x[cc];
  }
  __syncthreads();
  if (r == 0) piv[j0 + C] = j0 + p;
  if (p != C && r == C) {
#pragma unroll
    for (int cc = 0; cc < LU_NB; ++cc) x[cc] = prow[q][cc];
  } else if (p != C && r == p) {
#pragma unroll
    for (int cc = 0; cc < LU_NB; ++cc) x[cc] = crow[q][cc];
  }
  const double inv = 1.0 / prow[q][C];
  if (in && r > C) {
    const double l = x[C] * inv;
#pragma unroll
    for (int cc = C + 1; cc < LU_NB; ++cc) x[cc] -= l * prow[q][cc];
    x[C] = l;
  }
}

template <int ROWS, int... C>
__device__ __forceinline__ void lu_panel_columns(std::integer_sequence<int, C...>, double (&x)[LU_NB], int r,
                                                 int m, int j0, int w, int *__restrict__ piv,
                                                 double (*prow)[LU_NB], double (*crow)[LU_NB],
                                                 double (*wbest)[ROWS / 64], int (*wrow)[ROWS / 64]) {
  (lu_panel_column<ROWS, C>(x, r, m, j0, w, piv, prow, crow, wbest, wrow), ...);
}

// The same panel factorisation for panels of at most ROWS rows (256 or 1024), with each
// row's LU_NB entries in the registers of one thread (one column step per compile-time
// column index, so the row needs no LDS or scratch).  A column step is a pivot search
// (DPP row steps and readlanes within each wavefront, then the wavefront maxima through
// LDS), the row interchange through LDS, and the rank-1 update of every thread's own row
// with the pivot row read from LDS: two barriers per column.  The LDS buffers alternate
// between columns, so a column's writes never meet the previous column's reads.  The
// arithmetic is that of the other panel kernels, entry for entry.
template <int ROWS>
__global__ void __launch_bounds__(ROWS) k_lu_panel_reg(double *__restrict__ a, int n, int j0, int w,
                                                       int *__restrict__ piv) {
  __shared__ double prow[2][LU_NB], crow[2][LU_NB], wbest[2][ROWS / 64];
  __shared__ int wrow[2][ROWS / 64];
  const int r = threadIdx.x;
  const int m = n - j0;  // rows of the panel, <= ROWS
  const bool in = r < m;
  double x[LU_NB];
#pragma unroll
  for (int c = 0; c < LU_NB; ++c) x[c] = (in && c < w) ? a[(long long)(j0 + c) * n + j0 + r] : 0.0;
  lu_panel_columns<ROWS>(std::make_integer_sequence<int, LU_NB>{}, x, r, m, j0, w, piv, prow, crow, wbest, wrow);
#pragma unroll
  for (int c = 0; c < LU_NB; ++c)
    if (in && c < w) a[(long long)(j0 + c) * n + j0 + r] = x[c];
}

// Row interchanges of panel j0..j0+w-1 applied, in order, to every column outside it.
__global__ void __launch_bounds__(256) k_lu_swap(double *__restrict__ a, int n, int j0, int w,
                                                 const int *__restrict__ piv) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n || (col >= j0 && col < j0 + w)) return;
  double *c = a + (long long)col * n;
  for (int q = 0; q < w; ++q) {
    const int k = j0 + q, p = piv[k];
    if (p != k) {
      const double t = c[k];
      c[k] = c[p];
      c[p] = t;
    }
  }
}

// U12 = L11^{-1} A12: forward substitution with the panel's unit lower triangle, one
// wavefront per column right of the panel (lane r holds row j0 + r).
__global__ void __launch_bounds__(256) k_lu_trsm(double *__restrict__ a, int n, int j0, int w) {
  __shared__ double L[LU_NB][LU_NB];
  for (int t = threadIdx.x; t < w * w; t += blockDim.x) {
    const int r = t % w, c = t / w;
    L[r][c] = a[(long long)(j0 + c) * n + j0 + r];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int col = j0 + w + blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (col >= n) return;  // the whole wavefront leaves together
  double *c = a + (long long)col * n + j0;
  double x = lane < w ? c[lane] : 0.0;
  for (int q = 0; q + 1 < w; ++q) {
    const double xq = __shfl(x, q, 64);
    if (lane > q && lane < w) x -= L[lane][q] * xq;
  }
  if (lane < w) c[lane] = x;
}

// A22 -= L21 U12 on the trailing matrix (rows and columns from j0 + w): 64 x 64
// tiles per workgroup, 4 x 4 entries per thread, both operand tiles staged in LDS.
__global__ void __launch_bounds__(256) k_lu_gemm(double *__restrict__ a, int n, int j0, int w) {
  __shared__ double Lt[LU_NB][64];  // Lt[c][r] = L21(i0 + r, c)
  __shared__ double Ut[LU_NB][64];  // Ut[c][q] = U12(c, jc0 + q)
  const int base = j0 + w;
  const int i0 = base + blockIdx.x * 64, jc0 = base + blockIdx.y * 64;
  for (int t = threadIdx.x; t < LU_NB * 64; t += 256) {
    const int c = t / 64, r = t % 64;
    const int i = i0 + r, j = jc0 + r;
    Lt[c][r] = (c < w && i < n) ? a[(long long)(j0 + c) * n + i] : 0.0;
    Ut[c][r] = (c < w && j < n) ? a[(long long)j * n + j0 + c] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int c = 0; c < w; ++c) {
    double l[4], u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      l[q] = Lt[c][tx * 4 + q];
      u[q] = Ut[c][ty * 4 + q];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[r][q] += l[r] * u[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = jc0 + ty * 4 + q;
    if (j >= n) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + tx * 4 + r;
      if (i < n) a[(long long)j * n + i] -= acc[r][q];
    }
  }
}

// Lane l's copy of register v of lane `src` (a wavefront-uniform index), for doubles.
__device__ __forceinline__ double readlane_d(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, src);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Column j of A^{-1} from the factors P A = L U, one 64-lane workgroup per column.
// Lane l holds rows l + 64 q of the column in registers (q < NB = ceil(n / 64) <=
// NBMAX).  Forward (L, unit lower) and back (U) substitution go in blocks of 64 rows:
// the block's 64 x 64 diagonal part of the factor is staged in LDS by one burst of
// independent loads, its 64 sequential steps broadcast the solved entry with a
// readlane, and each 64 x 64 block of the factor below (above) it is staged the same
// way for the update of the rows outside the block.  The updates of every entry come in the
// same order as in plain column-by-column substitution.  No load or update is
// conditional (a conditional load is issued and waited for on its own): rows and
// columns past n are read at clamped, valid positions, and the lanes of rows past n
// compute values that are never read or stored.  The result is stored in row-major
// order for the coarse solve.
template <int NBMAX>
__global__ void __launch_bounds__(64) k_lu_inverse(const double *__restrict__ lu, const int *__restrict__ piv,
                                                   int n, double *__restrict__ inv) {
  __shared__ double D[64 * 64];  // D[c * 64 + l] = factor entry (64 kb + l, 64 kb + c)
  __shared__ double E[64 * 64];  // the same for the block (64 q + l, 64 kb + c), q != kb
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  const int NB = (n + 63) >> 6;
  // P e_j: the unit entry moves with every interchange that touches it
  int pv[NBMAX];
#pragma unroll
  for (int q = 0; q < NBMAX; ++q) pv[q] = piv[min(64 * q + lane, n - 1)];
  int pos = j;
#pragma unroll
  for (int q = 0; q < NBMAX; ++q) {
    if (q >= NB) continue;  // (not break: a constant trip count unrolls fully)
    const int rmax = min(64, n - 64 * q);
    for (int r = 0; r < rmax; ++r) {
      const int k = 64 * q + r;
      const int pk = __builtin_amdgcn_readlane(pv[q], r);
      pos = pos == k ? pk : (pos == pk ? k : pos);
    }
  }
  double y[NBMAX];
#pragma unroll
  for (int q = 0; q < NBMAX; ++q) y[q] = (64 * q + lane == pos) ? 1.0 : 0.0;
  // L y = P e_j
#pragma unroll
  for (int kb = 0; kb < NBMAX; ++kb) {
    if (kb >= NB) continue;
    const int rc = min(64 * kb + lane, n - 1);
    const int cmax = min(64, n - 64 * kb);  // columns of this block inside the matrix
#pragma unroll 16
    for (int c = 0; c < 64; ++c) D[c * 64 + lane] = lu[(long long)min(64 * kb + c, n - 1) * n + rc];
    __syncthreads();
    for (int c = 0; c < cmax; ++c) {
      const double yk = readlane_d(y[kb], c);
      if (lane > c) y[kb] -= D[c * 64 + lane] * yk;
    }
    // the blocks below, each staged in LDS by one burst of loads
#pragma unroll
    for (int q = kb + 1; q < NBMAX; ++q) {
      if (q >= NB) continue;
      const int rq = min(64 * q + lane, n - 1);
#pragma unroll 16
      for (int c = 0; c < 64; ++c) E[c * 64 + lane] = lu[(long long)min(64 * kb + c, n - 1) * n + rq];
      __syncthreads();
      for (int c = 0; c < cmax; ++c) y[q] -= E[c * 64 + lane] * readlane_d(y[kb], c);
      __syncthreads();
    }
    __syncthreads();  // D is restaged for the next block
  }
  // U x = y
#pragma unroll
  for (int kb = NBMAX - 1; kb >= 0; --kb) {
    if (kb >= NB) continue;
    const int rc = min(64 * kb + lane, n - 1);
    const int cmax = min(64, n - 64 * kb);
#pragma unroll 16
    for (int c = 0; c < 64; ++c) D[c * 64 + lane] = lu[(long long)min(64 * kb + c, n - 1) * n + rc];
    __syncthreads();
    for (int c = cmax - 1; c >= 0; --c) {
      const double xk = readlane_d(y[kb], c) / D[c * 64 + c];
      if (lane == c) y[kb] = xk;
      if (lane < c) y[kb] -= D[c * 64 + lane] * xk;
    }
#pragma unroll
    for (int q = 0; q < kb; ++q) {  // the blocks above
#pragma unroll 16
      for (int c = 0; c < 64; ++c) E[c * 64 + lane] = lu[(long long)min(64 * kb + c, n - 1) * n + 64 * q + lane];
      __syncthreads();
      for (int c = cmax - 1; c >= 0; --c) y[q] -= E[c * 64 + lane] * readlane_d(y[kb], c);
      __syncthreads();
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NBMAX; ++q) {
    const int i = 64 * q + lane;
    if (q < NB && i < n) inv[(long long)i * n + j] = y[q];
  }
}

// Column j of A^{-1} from the LU factors (one 64-lane block per column), column by
// column with the vector in LDS: the inverse of coarsest levels above 1024 unknowns.
__global__ void __launch_bounds__(64) k_lu_inverse_cols(const double *__restrict__ lu, const int *__restrict__ piv,
                                                   int n, double *__restrict__ inv) {
  extern __shared__ double y[];
  const int j = blockIdx.x;
  const int lane = threadIdx.x;
  for (int i = lane; i < n; i += 64) y[i] = (i == j) ? 1.0 : 0.0;
  __syncthreads();
  if (lane == 0)
    for (int k = 0; k < n; ++k) {
      const int p = piv[k];
      if (p != k) { const double t = y[k]; y[k] = y[p]; y[p] = t; }
    }
  __syncthreads();
  for (int k = 0; k < n; ++k) {  // L y = P e_j (unit lower)
    const double yk = y[k];
    for (int i = k + 1 + lane; i < n; i += 64) y[i] -= lu[(long long)k * n + i] * yk;
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {  // U x = y
    if (lane == 0) y[k] = y[k] / lu[(long long)k * n + k];
    __syncthreads();
    const double xk = y[k];
    for (int i = lane; i < k; i += 64) y[i] -= lu[(long long)k * n + i] * xk;
    __syncthreads();
  }
  for (int i = lane; i < n; i += 64) inv[(long long)i * n + j] = y[i];  // row-major
}

// Row r of x = A^{-1} b on the coarsest level (row-major inverse), computed by one
// 64-lane wavefront: coalesced row reads and a fixed-order shuffle reduction.
template <typename T>
__device__ __forceinline__ void coarse_row(const double *__restrict__ inv, int n, const T *__restrict__ b,
                                           T *__restrict__ x, int r, int lane) {
  const double *row = inv + (long long)r * n;
  double s = 0.0;
  for (int c = lane; c < n; c += 64) s += row[c] * (double)b[c];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[r] = (T)s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_coarse_solve(const double *__restrict__ inv, int n,
                                                      const T *__restrict__ b, T *__restrict__ x) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;  // whole wavefront exits together
  coarse_row<T>(inv, n, b, x, r, threadIdx.x & 63);
}

template <typename TI, typename TO>
__global__ void k_cast(const TI *__restrict__ a, TO *__restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = (TO)a[i];
}

inline Geo geo(const Level &L) { return Geo{L.n[0], L.n[1], L.n[2], L.N}; }

// Tiled finest FP32 matrix -> [offset][vertex] layout, one thread per block.
__global__ void k_untile(const float *__restrict__ src, float *__restrict__ dst, long long N, int nst) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nst * N) return;
  const int o = (int)(t / N);
  const long long v = t % N;
  *reinterpret_cast<float4 *>(dst + t * 4) = *reinterpret_cast<const float4 *>(src + tiled_block(o, v, nst) * 4);
}

// Storage part of one level's operator moved to a new step: the centre block's S-column
// entries are (flux part) + mst, where mst is the level's storage M/h (fine level: the
// box-method storage, zero on Dirichlet rows; coarse levels: its lumped Galerkin image,
// linear in the fine storage).  The flux part of every level does not depend on h, so
// A(h') = A(h) - mst + ratio mst with ratio = h / h'.  The FP32 copy's centre block is
// rewritten from the new FP64 block (tiled on the finest level).
template <int DIM>
__global__ void __launch_bounds__(BS) k_rescale(const Geo G, double *__restrict__ A, float *__restrict__ A32,
                                                int tiled, double *__restrict__ mst, double ratio) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  constexpr int CEN = DIM == 3 ? 13 : 4;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= G.N) return;
  const double2 m = *reinterpret_cast<const double2 *>(mst + 2 * v);
  const double n0 = m.x * ratio, n1 = m.y * ratio;
  double2 *blk = reinterpret_cast<double2 *>(A + ((long long)CEN * G.N + v) * 4);
  double2 b01 = blk[0], b23 = blk[1];
  b01.y = (b01.y - m.x) + n0;
  b23.y = (b23.y - m.y) + n1;
  blk[0] = b01;
  blk[1] = b23;
  *reinterpret_cast<double2 *>(mst + 2 * v) = make_double2(n0, n1);
  if (A32) {
    const long long k = tiled ? tiled_block(CEN, v, NST) : (long long)CEN * G.N + v;
    *reinterpret_cast<float4 *>(A32 + k * 4) = make_float4((float)b01.x, (float)b01.y, (float)b23.x, (float)b23.y);
  }
}

// ---- V-cycle driver ----------------------------------------------------------
// TPF_MIXED16 coarse levels: sweep (first: zero initial guess) and residual with the
// FP16 matrix; return false where the level is not stored in FP16.
// ---- line-block Jacobi (TPF_SMOOTH_LINE): two threads per vertex line ------------
// The twisted factorisation splits every line at its middle: lanes l and l + 32 of a
// wavefront run the top and the bottom chain of the same line and exchange their edge
// values with a lane shuffle, so a wavefront covers 32 lines and each chain is half a
// line long (against one thread per line: 504 -> 282 us per sweep on 4097 lines of 2049
// vertices, 57 -> 46 us on 129^3).  Few threads walk long lines, so the launches use one wavefront per block
// to spread the lines over the compute units, and each thread keeps 16 steps of loads
// in flight (one thread per line, measured against 8, 24 and 32 steps: 718 -> 504 us
// per sweep on 4097 lines of 2049 vertices, 71 -> 57 us on 129^3).
constexpr int LINE_BS = 64;
constexpr int LINES_PER_BLOCK = 32;
#ifndef TPF_LINE_CHUNK
#define TPF_LINE_CHUNK 16
#endif
#ifndef TPF_LINE_FACTOR_CHUNK
#define TPF_LINE_FACTOR_CHUNK 4
#endif

template <int DIM, typename TO>
__global__ void __launch_bounds__(LINE_BS) k_line_factor(const Geo G, const double *__restrict__ A,
                                                         TO *__restrict__ lf, int *__restrict__ bad) {
  const long long l = (long long)blockIdx.x * LINE_BS + threadIdx.x;
  if (l >= line_geo<DIM>(G).S) return;
  if (!line_factor<DIM, TO, TPF_LINE_FACTOR_CHUNK>(G, A, lf, l)) atomicAdd(bad, 1);
}

// The same factorisation with the two halves of a line on lanes l and l + 32 of one
// wavefront (the layout of k_line), which exchange W_{m-1} and V_{m+1} for the middle
// row; the top lane stores the middle and counts the line if any of its pivots is bad.
template <int DIM, typename TO>
__global__ void __launch_bounds__(LINE_BS) k_line_factor2(const Geo G, const double *__restrict__ A,
                                                          TO *__restrict__ lf, int *__restrict__ bad) {
  const int lane = threadIdx.x;  // the block is one wavefront
  const bool top = lane < LINES_PER_BLOCK;
  const long long l = (long long)blockIdx.x * LINES_PER_BLOCK + (top ? lane : lane - LINES_PER_BLOCK);
  const bool valid = l < line_geo<DIM>(G).S;
  double cpl[4] = {0.0, 0.0, 0.0, 0.0};
  bool ok = true;
  if (valid) ok = line_factor_half<DIM, TO, TPF_LINE_FACTOR_CHUNK>(G, A, lf, l, top, cpl);
  double other[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) other[i] = __shfl_xor(cpl[i], LINES_PER_BLOCK, 64);
  const bool ok_other = __shfl_xor((int)ok, LINES_PER_BLOCK, 64) != 0;
  if (!valid || !top) return;
  ok = line_factor_middle<DIM, TO>(G, A, lf, l, cpl, other) && ok && ok_other;
  if (!ok) atomicAdd(bad, 1);
}

// Levels with at least g->line_pair_max lines (default TPF_LINE_PAIR_MAX_LINES) have
// parallelism enough with one thread per line (both chains in turn, the same operations
// in the same order), which reads each step's blocks as 1 KB segments instead of two
// 512 B ones: 257^3 (66049 lines) 328 us per sweep against 353 us with pairs.

template <int DIM, typename T, typename TO>
__global__ void __launch_bounds__(LINE_BS) k_line_single(const Geo G, const T *__restrict__ lf, const T *rin,
                                                         T *cbuf, const T *__restrict__ xi, TO *__restrict__ xo,
                                                         const T omega) {
  const long long l = (long long)blockIdx.x * LINE_BS + threadIdx.x;
  if (l >= line_geo<DIM>(G).S) return;
  line_solve<DIM, T, TO, TPF_LINE_CHUNK>(G, lf, rin, cbuf, xi, xo, omega, l);
}

template <int DIM, typename T, typename TO>
__global__ void __launch_bounds__(LINE_BS) k_line(const Geo G, const T *__restrict__ lf, const T *rin, T *cbuf,
                                                  const T *__restrict__ xi, TO *__restrict__ xo, const T omega) {
  const int lane = threadIdx.x;  // the block is one wavefront
  const bool top = lane < LINES_PER_BLOCK;
  const long long l = (long long)blockIdx.x * LINES_PER_BLOCK + (lane & (LINES_PER_BLOCK - 1));
  const bool valid = l < line_geo<DIM>(G).S;  // the same for both lanes of a pair
  T c0 = 0, c1 = 0;
  if (valid) line_forward<DIM, T, TPF_LINE_CHUNK>(G, lf, rin, cbuf, l, top, c0, c1);
  // every lane takes part in the exchange: c_{m-1} from the top lane, c_{m+1} from the bottom
  const T o0 = __shfl_xor(c0, LINES_PER_BLOCK, 64), o1 = __shfl_xor(c1, LINES_PER_BLOCK, 64);
  if (!valid) return;
  T z0, z1;
  line_middle<DIM, T>(G, lf, rin, l, top ? c0 : o0, top ? c1 : o1, top ? o0 : c0, top ? o1 : c1, z0, z1);
  line_backward<DIM, T, TO, TPF_LINE_CHUNK>(G, lf, cbuf, xi, xo, omega, l, top, z0, z1);
}

// Line LU of every level but the coarsest from its FP64 matrix, in the level type.
// Singular pivot blocks are counted into g->line_bad (a device int cleared here).
template <int DIM>
tpf_status line_factors_t(tpf_grid *g, hipStream_t s) {
  if (g->smoother != TPF_SMOOTH_LINE) return TPF_OK;
  k_zero_int<<<1, 64, 0, s>>>(g->line_bad, 1);
  TPF_LAUNCH_CHECK();
  for (int l = 0; l + 1 < g->L; ++l) {
    const Level &lv = g->lv[l];
    const long long nl = line_geo<DIM>(geo(lv)).S;
    const bool pairs = nl < g->line_pair_max;
    const unsigned nb = pairs ? blocks_for(nl, LINES_PER_BLOCK) : blocks_for(nl, LINE_BS);
    if (g->prec == TPF_FP64) {
      double *lf = reinterpret_cast<double *>(lv.lf);
      if (pairs)
        k_line_factor2<DIM, double><<<nb, LINE_BS, 0, s>>>(geo(lv), lv.A64, lf, g->line_bad);
      else
        k_line_factor<DIM, double><<<nb, LINE_BS, 0, s>>>(geo(lv), lv.A64, lf, g->line_bad);
    } else {
      float *lf = reinterpret_cast<float *>(lv.lf);
      if (pairs)
        k_line_factor2<DIM, float><<<nb, LINE_BS, 0, s>>>(geo(lv), lv.A64, lf, g->line_bad);
      else
        k_line_factor<DIM, float><<<nb, LINE_BS, 0, s>>>(geo(lv), lv.A64, lf, g->line_bad);
    }
    TPF_LAUNCH_CHECK();
  }
  g->line_unchecked = true;
  return TPF_OK;
}

template <int DIM, typename T>
bool sweep16(tpf_grid *g, int l, bool first, const T *b, const T *xi, T *xo, T om, hipStream_t s) {
  if constexpr (sizeof(T) != sizeof(float)) {
    return false;
  } else {
    if (g->prec != TPF_MIXED16 || l == 0) return false;
    const Level &lv = g->lv[l];
    const unsigned nb = blocks_for(lv.N);
    if (first)
      (void)launch(g, TPF_K_COARSE_LEVELS, k_jacobi16<DIM, true>, nb, BS, s, geo(lv), (const uint16_t *)lv.A16,
                   (const float *)lv.s16, b, (const T *)nullptr, xo, om);
    else
      (void)launch(g, TPF_K_COARSE_LEVELS, k_jacobi16<DIM, false>, nb, BS, s, geo(lv), (const uint16_t *)lv.A16,
                   (const float *)lv.s16, b, xi, xo, om);
    return true;
  }
}

template <int DIM, typename T>
bool resid16(tpf_grid *g, int l, const T *b, const T *x, T *r, hipStream_t s) {
  if constexpr (sizeof(T) != sizeof(float)) {
    return false;
  } else {
    if (g->prec != TPF_MIXED16 || l == 0) return false;
    const Level &lv = g->lv[l];
    (void)launch(g, TPF_K_COARSE_LEVELS, k_resid16<DIM>, blocks_for(lv.N), BS, s, geo(lv),
                 (const uint16_t *)lv.A16, (const float *)lv.s16, b, x, r);
    return true;
  }
}

// Levels up to this many vertices are latency-bound: their sweeps issue a row's
// loads all at once (LAT) instead of in register-friendly groups.
constexpr long long LAT_NMAX = 65536;

template <int DIM, typename T>
tpf_status vcycle_t(tpf_grid *g, const double *bin, double *xout, hipStream_t s, bool staged) {
  const int L = g->L;
  const T om = (T)g->omega;
  const T *b0;
  if (sizeof(T) == sizeof(double)) {
    b0 = reinterpret_cast<const T *>(bin);
  } else {
    if (!staged) {  // else the caller has written (T)bin to the level-0 right-hand side
      k_cast<double, T><<<1024, BS, 0, s>>>(bin, reinterpret_cast<T *>(g->lv[0].b), 2 * g->lv[0].N);
      TPF_LAUNCH_CHECK();
    }
    b0 = reinterpret_cast<const T *>(g->lv[0].b);
  }
  auto A_of = [&](int l) -> const T * {
    if (sizeof(T) == sizeof(double)) return reinterpret_cast<const T *>(g->lv[l].A64);
    return reinterpret_cast<const T *>(g->lv[l].A32);
  };
  constexpr bool NT0 = sizeof(T) == sizeof(float);  // finest FP32 matrix: streamed, non-temporal
  const T *const noT = nullptr;
  const uint8_t *const nomask = nullptr;
  if (L == 1) {  // single level: the dense solve is the whole cycle
    {
      const tpf_status st = lu_join(g, s);
      if (st != TPF_OK) return st;
    }
    Level &lc = g->lv[0];
    T *X = sizeof(T) == sizeof(double) ? reinterpret_cast<T *>(xout) : reinterpret_cast<T *>(lc.x);
    TPF_HIP(launch(g, TPF_K_COARSE_LEVELS, k_coarse_solve<T>, (unsigned)((g->nc + 3) / 4), 256u, s,
                   (const double *)g->ainv, g->nc, b0, X));
    if (sizeof(T) != sizeof(double)) {
      k_cast<T, double><<<1024, BS, 0, s>>>(X, xout, 2 * lc.N);
      TPF_LAUNCH_CHECK();
    }
    return TPF_OK;
  }
  const T *bl[MAXL];
  T *cur[MAXL];
  bl[0] = b0;
  // levels whose first sweep runs inside the restriction (not the FP16 levels)
  auto fused_first = [&](int l) {
    return l >= 1 && l < L - 1 && g->prec != TPF_MIXED16 && g->smoother == TPF_SMOOTH_POINT;
  };
  const bool line = g->smoother == TPF_SMOOTH_LINE;
  // r = b - A x on level l into R
  // r = b - A x; after_zero_sweep: x = omega A_L^{-1} b (one line sweep from a zero
  // guess), so r = (1 - omega) b - (A - A_L) x needs 24 of the 27 blocks of each row
  auto resid = [&](int l, const T *b, const T *x, T *R, hipStream_t s, bool after_zero_sweep = false) -> tpf_status {
    Level &lv = g->lv[l];
    const Geo G = geo(lv);
    const unsigned nb = blocks_for(lv.N);
    const int c_re = l == 0 ? TPF_K_RESID0 : TPF_K_COARSE_LEVELS;
    const T one = (T)1, bs = (T)1 - om;
    if (resid16<DIM, T>(g, l, b, x, R, s)) {
      TPF_LAUNCH_CHECK();
    } else if (l == 0 && NT0) {
      if (after_zero_sweep)
        TPF_HIP(launch(g, c_re, k_resid_stream<DIM, T, true>, nb, BS, s, G, A_of(l), b, x, R, bs));
      else
        TPF_HIP(launch(g, c_re, k_resid_stream<DIM, T, false>, nb, BS, s, G, A_of(l), b, x, R, one));
    } else if (lv.N > LAT_NMAX) {
      if (after_zero_sweep)
        TPF_HIP(launch(g, c_re, k_resid<DIM, T, false, false, true>, nb, BS, s, G, A_of(l), b, x, R, bs));
      else
        TPF_HIP(launch(g, c_re, k_resid<DIM, T>, nb, BS, s, G, A_of(l), b, x, R, one));
    } else {
      if (after_zero_sweep)
        TPF_HIP(launch(g, c_re, k_resid<DIM, T, false, true, true>, nb, BS, s, G, A_of(l), b, x, R, bs));
      else
        TPF_HIP(launch(g, c_re, k_resid<DIM, T, false, true>, nb, BS, s, G, A_of(l), b, x, R, one));
    }
    return TPF_OK;
  };
  // one line sweep on level l: xo = xi + omega A_L^{-1} (b - A xi) (xi == nullptr: a
  // zero guess, xo = omega A_L^{-1} b); the level's residual vector holds r and c
  auto line_sweep = [&](int l, const T *b, const T *xi, auto *xo, hipStream_t s) -> tpf_status {
    using TO = std::remove_pointer_t<decltype(xo)>;
    Level &lv = g->lv[l];
    T *R = reinterpret_cast<T *>(lv.r);
    const T *rin = b;
    if (xi) {
      const tpf_status st = resid(l, b, xi, R, s);
      if (st != TPF_OK) return st;
      rin = R;
    }
    const long long nl = line_geo<DIM>(geo(lv)).S;
    const int cls = l == 0 ? TPF_K_LINE0 : TPF_K_COARSE_LEVELS;
    if (nl < g->line_pair_max)
      TPF_HIP(launch(g, cls, k_line<DIM, T, TO>, blocks_for(nl, LINES_PER_BLOCK), (unsigned)LINE_BS, s, geo(lv),
                     (const T *)lv.lf, rin, R, xi, xo, om));
    else
      TPF_HIP(launch(g, cls, k_line_single<DIM, T, TO>, blocks_for(nl, LINE_BS), (unsigned)LINE_BS, s, geo(lv),
                     (const T *)lv.lf, rin, R, xi, xo, om));
    return TPF_OK;
  };
  // pre-smoothing, residual and restriction of level l (into l + 1, with l + 1's first
  // sweep when it is fused into the restriction)
  auto down = [&](int l, hipStream_t s) -> tpf_status {
    Level &lv = g->lv[l];
    const Geo G = geo(lv);
    const unsigned nb = blocks_for(lv.N);
    T *X = reinterpret_cast<T *>(lv.x), *Y = reinterpret_cast<T *>(lv.y);
    const int c_sm = l == 0 ? TPF_K_SMOOTH0 : TPF_K_COARSE_LEVELS;
    if (line) {
      tpf_status st = line_sweep(l, bl[l], (const T *)nullptr, X, s);
      for (int k = 1; k < g->nu_pre && st == TPF_OK; ++k) {
        st = line_sweep(l, bl[l], (const T *)X, Y, s);
        T *t = X; X = Y; Y = t;
      }
      if (st != TPF_OK) return st;
    } else if (fused_first(l)) {
      // X already holds the first sweep, written with the restriction into this level
    } else if (sweep16<DIM, T>(g, l, true, bl[l], nullptr, X, om, s)) {
      TPF_LAUNCH_CHECK();
    } else if (l == 0 && NT0) {
      TPF_HIP(launch(g, TPF_K_SMOOTH0_FIRST, k_jacobi<DIM, T, T, true, false, true>, nb, BS, s, G, A_of(l), bl[l],
                     noT, X, om));
    } else {
      TPF_HIP(launch(g, l == 0 ? TPF_K_SMOOTH0_FIRST : TPF_K_COARSE_LEVELS, k_jacobi<DIM, T, T, true>, nb, BS, s,
                     G, A_of(l), bl[l], noT, X, om));
    }
    for (int k = 1; k < g->nu_pre && !line; ++k) {
      if (sweep16<DIM, T>(g, l, false, bl[l], X, Y, om, s)) {
        TPF_LAUNCH_CHECK();
      } else if (l == 0 && NT0) {
        TPF_HIP(launch(g, c_sm, k_jacobi_stream<DIM, T, T>, nb, BS, s, G, A_of(l), bl[l], (const T *)X, Y, om));
      } else if (lv.N > LAT_NMAX) {
        TPF_HIP(launch(g, c_sm, k_jacobi<DIM, T, T, false>, nb, BS, s, G, A_of(l), bl[l], (const T *)X, Y, om));
      } else {
        TPF_HIP(launch(g, c_sm, k_jacobi<DIM, T, T, false, false, false, true>, nb, BS, s, G, A_of(l), bl[l],
                       (const T *)X, Y, om));
      }
      T *t = X; X = Y; Y = t;
    }
    cur[l] = X;
    T *R = reinterpret_cast<T *>(lv.r);
    {
      const tpf_status st = resid(l, bl[l], (const T *)X, R, s, line && g->nu_pre == 1);
      if (st != TPF_OK) return st;
    }
    Level &lc = g->lv[l + 1];
    T *bc = reinterpret_cast<T *>(lc.b);
    const int c_tr = l == 0 ? TPF_K_TRANSFER0 : TPF_K_COARSE_LEVELS;
    const uint8_t *fm = l == 0 ? (const uint8_t *)g->dmask : nomask;
    const T vr = (T)(g->P.rho_w / g->P.rho_n);
    if (fused_first(l + 1))
      TPF_HIP(launch(g, c_tr, k_restrict_first<DIM, T>, blocks_for(lc.N), BS, s, G, geo(lc), (const T *)R, fm, vr,
                     bc, A_of(l + 1), reinterpret_cast<T *>(lc.x), om));
    else
      TPF_HIP(launch(g, c_tr, k_restrict<DIM, T>, blocks_for(lc.N), BS, s, G, geo(lc), (const T *)R, fm, vr, bc));
    bl[l + 1] = bc;
    return TPF_OK;
  };
  // coarsest level: x = A^{-1} b, one wavefront per row of the inverse
  bool capturing = false;  // the tail is being recorded into the grid's graph
  auto coarsest = [&](hipStream_t s) -> tpf_status {
    if (!capturing) {  // (a captured tail is launched after a wait of its own)
      const tpf_status st = lu_join(g, s);
      if (st != TPF_OK) return st;
    }
    Level &lc = g->lv[L - 1];
    T *X = reinterpret_cast<T *>(lc.x);
    TPF_HIP(launch(g, TPF_K_COARSE_LEVELS, k_coarse_solve<T>, (unsigned)((g->nc + 3) / 4), 256u, s,
                   (const double *)g->ainv, g->nc, bl[L - 1], X));
    cur[L - 1] = X;
    return TPF_OK;
  };
  // prolongation from level l + 1 and post-smoothing of level l (the finest level's
  // last sweep writes the FP64 result)
  auto up = [&](int l, hipStream_t s) -> tpf_status {
    Level &lv = g->lv[l];
    const Geo G = geo(lv);
    const unsigned nb = blocks_for(lv.N);
    T *X = cur[l];
    T *Y = (X == reinterpret_cast<T *>(lv.x)) ? reinterpret_cast<T *>(lv.y) : reinterpret_cast<T *>(lv.x);
    const int c_sm = l == 0 ? TPF_K_SMOOTH0 : TPF_K_COARSE_LEVELS;
    TPF_HIP(launch(g, l == 0 ? TPF_K_TRANSFER0 : TPF_K_COARSE_LEVELS, k_prolong<DIM, T>, nb, BS, s, G,
                   geo(g->lv[l + 1]), (const T *)cur[l + 1], l == 0 ? (const uint8_t *)g->dmask : nomask, X));
    const int nu = g->nu_post;
    for (int k = 0; k < nu; ++k) {
      if (line) {
        const tpf_status st = (l == 0 && k == nu - 1) ? line_sweep(l, bl[l], (const T *)X, xout, s)
                                                       : line_sweep(l, bl[l], (const T *)X, Y, s);
        if (st != TPF_OK) return st;
        if (l == 0 && k == nu - 1) {
          X = nullptr;
          break;
        }
        T *t = X; X = Y; Y = t;
        continue;
      }
      if (l == 0 && k == nu - 1) {
        if (NT0)
          TPF_HIP(launch(g, c_sm, k_jacobi_stream<DIM, T, double>, nb, BS, s, G, A_of(l), bl[l], (const T *)X,
                         xout, om));
        else
          TPF_HIP(launch(g, c_sm, k_jacobi<DIM, T, double, false>, nb, BS, s, G, A_of(l), bl[l], (const T *)X,
                         xout, om));
        X = nullptr;
        break;
      }
      if (sweep16<DIM, T>(g, l, false, bl[l], X, Y, om, s)) {
        TPF_LAUNCH_CHECK();
      } else if (l == 0 && NT0) {
        TPF_HIP(launch(g, c_sm, k_jacobi_stream<DIM, T, T>, nb, BS, s, G, A_of(l), bl[l], (const T *)X, Y, om));
      } else if (lv.N > LAT_NMAX) {
        TPF_HIP(launch(g, c_sm, k_jacobi<DIM, T, T, false>, nb, BS, s, G, A_of(l), bl[l], (const T *)X, Y, om));
      } else {
        TPF_HIP(launch(g, c_sm, k_jacobi<DIM, T, T, false, false, false, true>, nb, BS, s, G, A_of(l), bl[l],
                       (const T *)X, Y, om));
      }
      T *t = X; X = Y; Y = t;
    }
    if (l == 0 && X != nullptr) {  // nu_post == 0
      k_cast<T, double><<<1024, BS, 0, s>>>(X, xout, 2 * lv.N);
      TPF_LAUNCH_CHECK();
    }
    cur[l] = X;
    return TPF_OK;
  };
  // the coarse tail: every level below the finest, down and up again; it reads level
  // 1's right-hand side and writes cur[1], both at addresses fixed for the grid
  auto tail = [&](hipStream_t s) -> tpf_status {
    for (int l = 1; l < L - 1; ++l) {
      const tpf_status st = down(l, s);
      if (st != TPF_OK) return st;
    }
    tpf_status st = coarsest(s);
    if (st != TPF_OK) return st;
    for (int l = L - 2; l >= 1; --l) {
      st = up(l, s);
      if (st != TPF_OK) return st;
    }
    return TPF_OK;
  };
  tpf_status st = down(0, s);
  if (st != TPF_OK) return st;
  // (the graph's launches carry no timing events: it is skipped while the coarse-level
  // class itself is being timed)
  const bool timing_coarse = g->prof.active && ((g->prof.mask >> TPF_K_COARSE_LEVELS) & 1u);
  if (g->coarse_graph && L >= 3 && !timing_coarse) {
    // the tail as one captured graph (recorded on the grid's capture stream the first
    // time; the same launches as below, replayed)
    if (!g->vgraph_exec) {
      if (!g->cap_stream) TPF_HIP(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
      TPF_HIP(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal));
      capturing = true;
      const tpf_status cst = tail(g->cap_stream);
      capturing = false;
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(g->cap_stream, &graph);
      if (cst != TPF_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (cst != TPF_OK) return cst;
        TPF_HIP(e);
      }
      const hipError_t ei = hipGraphInstantiate(&g->vgraph_exec, graph, nullptr, nullptr, 0);
      if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        g->vgraph_exec = nullptr;
        TPF_HIP(ei);
      }
      g->vgraph = graph;
      g->vgraph_cur1 = cur[1];
    }
    cur[1] = reinterpret_cast<T *>(g->vgraph_cur1);
    st = lu_join(g, s);
    if (st != TPF_OK) return st;
    TPF_HIP(hipGraphLaunch(g->vgraph_exec, s));
  } else {
    st = tail(s);
    if (st != TPF_OK) return st;
  }
  return up(0, s);
}

template <int DIM>
tpf_status coarse_factor_t(tpf_grid *g, hipStream_t s);

template <int DIM>
tpf_status hierarchy_t(tpf_grid *g, hipStream_t s) {
  {  // the Galerkin products overwrite the matrix a pending factorisation reads
    const tpf_status st = lu_join(g, s);
    if (st != TPF_OK) return st;
  }
  for (int l = 0; l + 1 < g->L; ++l) {
    const Level &f = g->lv[l];
    Level &c = g->lv[l + 1];
    float *c32 = g->prec == TPF_MIXED ? c.A32 : nullptr;
    const int ps = prof_begin(g, TPF_K_RAP, s);
    const tpf_status st = launch_rap(g->dim, l == 0, f.n, f.N, c.n, c.N, f.A64, l == 0 ? g->dmask : nullptr, f.mst,
                                     g->P.rho_w / g->P.rho_n, g->rapb, c.A64, c32, c.mst, s);
    if (st != TPF_OK) return st;
    if (g->prec == TPF_MIXED16) {
      k_to16<DIM><<<blocks_for(c.N), BS, 0, s>>>(geo(c), c.A64, c.A16, c.s16);
      TPF_LAUNCH_CHECK();
    }
    prof_end(g, ps, s);
  }
  {  // the coarsest factorisation, forked to the grid's own stream
    const tpf_status st = coarse_factor_t<DIM>(g, s);
    if (st != TPF_OK) return st;
  }
  if (g->smoother == TPF_SMOOTH_LINE) {  // the line LU, timed with the Galerkin products
    const int ps = prof_begin(g, TPF_K_RAP, s);
    const tpf_status st = line_factors_t<DIM>(g, s);
    if (st != TPF_OK) return st;
    prof_end(g, ps, s);
  }
  return TPF_OK;
}

// Dense LU with partial pivoting of the coarsest level and its inverse.  Its kernels
// occupy one or a few workgroups at a time, so outside stream capture they run on the
// grid's own stream, forked from s: the line LU, the solver's set-up and the first
// V-cycle's descent, queued on s meanwhile, fill the rest of the device, and s waits
// for the factors only where it first needs them (lu_join).
template <int DIM>
tpf_status coarse_factor_t(tpf_grid *g, hipStream_t s0) {
  {
    const tpf_status st = lu_join(g, s0);
    if (st != TPF_OK) return st;
  }
  hipStream_t s = s0;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  TPF_HIP(hipStreamIsCapturing(s0, &cs));
  if (cs == hipStreamCaptureStatusNone) {
    if (!g->lu_stream) {
      TPF_HIP(hipStreamCreateWithFlags(&g->lu_stream, hipStreamNonBlocking));
      TPF_HIP(hipEventCreateWithFlags(&g->lu_fork, hipEventDisableTiming));
      TPF_HIP(hipEventCreateWithFlags(&g->lu_done, hipEventDisableTiming));
    }
    TPF_HIP(hipEventRecord(g->lu_fork, s0));
    TPF_HIP(hipStreamWaitEvent(g->lu_stream, g->lu_fork, 0));
    s = g->lu_stream;
  }
  Level &lc = g->lv[g->L - 1];
  const int n = g->nc;
  const int pl = prof_begin(g, TPF_K_COARSE_LU, s);
  k_zero<<<256, BS, 0, s>>>(g->lu, (long long)n * n);
  TPF_LAUNCH_CHECK();
  constexpr int NST = DIM == 3 ? 27 : 9;
  k_densify<DIM><<<blocks_for((long long)NST * lc.N), BS, 0, s>>>(geo(lc), lc.A64, g->lu, n);
  TPF_LAUNCH_CHECK();
  for (int j0 = 0; j0 < n; j0 += LU_NB) {
    const int w = n - j0 < LU_NB ? n - j0 : LU_NB;
    if (n - j0 <= 256)
      k_lu_panel_reg<256><<<1, 256, 0, s>>>(g->lu, n, j0, w, g->piv);
    else if (n - j0 <= 1024)
      k_lu_panel_reg<1024><<<1, 1024, 0, s>>>(g->lu, n, j0, w, g->piv);
    else
      k_lu_panel<<<1, 1024, 0, s>>>(g->lu, n, j0, w, g->piv);
    TPF_LAUNCH_CHECK();
    k_lu_swap<<<blocks_for(n, 256), 256, 0, s>>>(g->lu, n, j0, w, g->piv);
    TPF_LAUNCH_CHECK();
    const int m = n - j0 - w;
    if (m > 0) {
      k_lu_trsm<<<(unsigned)((m + 3) / 4), 256, 0, s>>>(g->lu, n, j0, w);
      TPF_LAUNCH_CHECK();
      const unsigned t = (unsigned)((m + 63) / 64);
      k_lu_gemm<<<dim3(t, t), 256, 0, s>>>(g->lu, n, j0, w);
      TPF_LAUNCH_CHECK();
    }
  }
  {
    const int nb = (n + 63) / 64;
    if (nb <= 4)
      k_lu_inverse<4><<<n, 64, 0, s>>>(g->lu, g->piv, n, g->ainv);
    else if (nb <= 16)
      k_lu_inverse<16><<<n, 64, 0, s>>>(g->lu, g->piv, n, g->ainv);
    else  // more row blocks than registers comfortably hold
      k_lu_inverse_cols<<<n, 64, (size_t)n * sizeof(double), s>>>(g->lu, g->piv, n, g->ainv);
    TPF_LAUNCH_CHECK();
  }
  prof_end(g, pl, s);
  if (s != s0) {
    TPF_HIP(hipEventRecord(g->lu_done, s));
    g->lu_pending = true;
  }
  return TPF_OK;
}

template <int DIM>
tpf_status spmv_t(tpf_grid *g, int level, const double *x, double *y, hipStream_t s) {
  const Level &lv = g->lv[level];
  TPF_HIP(launch(g, level == 0 ? TPF_K_SPMV64 : TPF_K_COARSE_LEVELS, k_spmv64<DIM, 0>, blocks_for(lv.N), BS, s,
                 geo(lv), (const double *)lv.A64, x, y, (const double *)nullptr, (double *)nullptr));
  return TPF_OK;
}

// Every level's operator moved from the step h to h / ratio (storage parts scaled by
// ratio), the FP32 / FP16 copies refreshed, the coarsest level refactored.
template <int DIM>
tpf_status rescale_t(tpf_grid *g, double ratio, hipStream_t s) {
  {  // the rescaling overwrites the matrix a pending factorisation reads
    const tpf_status st = lu_join(g, s);
    if (st != TPF_OK) return st;
  }
  const int ps = prof_begin(g, TPF_K_ASSEMBLE, s);
  for (int l = 0; l < g->L; ++l) {
    Level &lv = g->lv[l];
    float *a32 = lv.A32;  // FP32 copy where one exists (finest tiled)
    k_rescale<DIM><<<blocks_for(lv.N), BS, 0, s>>>(geo(lv), lv.A64, a32, l == 0 ? 1 : 0, lv.mst, ratio);
    TPF_LAUNCH_CHECK();
    if (g->prec == TPF_MIXED16 && l > 0) {  // the row scales depend on the centre block
      k_to16<DIM><<<blocks_for(lv.N), BS, 0, s>>>(geo(lv), lv.A64, lv.A16, lv.s16);
      TPF_LAUNCH_CHECK();
    }
  }
  prof_end(g, ps, s);
  {
    const tpf_status st = coarse_factor_t<DIM>(g, s);
    if (st != TPF_OK) return st;
  }
  const int pl = prof_begin(g, TPF_K_ASSEMBLE, s);
  const tpf_status st = line_factors_t<DIM>(g, s);
  prof_end(g, pl, s);
  return st;
}

}  // namespace

tpf_status rescale_stage(tpf_grid *g, double ratio, hipStream_t s) {
  return g->dim == 3 ? rescale_t<3>(g, ratio, s) : rescale_t<2>(g, ratio, s);
}

tpf_status untile_matrix32(tpf_grid *g, float *dst, hipStream_t s) {
  const Level &lv = g->lv[0];
  const long long n = (long long)g->nst * lv.N;
  k_untile<<<blocks_for(n), BS, 0, s>>>(lv.A32, dst, lv.N, g->nst);
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

tpf_status expand_matrix16(tpf_grid *g, int level, float *dst, hipStream_t s) {
  const Level &lv = g->lv[level];
  const long long n = (long long)g->nst * lv.N;
  k_expand16<<<blocks_for(n), BS, 0, s>>>(lv.A16, lv.s16, dst, lv.N, g->nst);
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

tpf_status build_hierarchy(tpf_grid *g, hipStream_t s) {
  return g->dim == 3 ? hierarchy_t<3>(g, s) : hierarchy_t<2>(g, s);
}

tpf_status vcycle(tpf_grid *g, const double *b, double *x, hipStream_t s, bool staged) {
  if (g->prec != TPF_FP64)
    return g->dim == 3 ? vcycle_t<3, float>(g, b, x, s, staged) : vcycle_t<2, float>(g, b, x, s, staged);
  return g->dim == 3 ? vcycle_t<3, double>(g, b, x, s, staged) : vcycle_t<2, double>(g, b, x, s, staged);
}

tpf_status spmv64(tpf_grid *g, int level, const double *x, double *y, hipStream_t s) {
  return g->dim == 3 ? spmv_t<3>(g, level, x, y, s) : spmv_t<2>(g, level, x, y, s);
}

// Fused SpMV variants used by BiCGSTAB (declared in krylov.hip).
tpf_status spmv64_mode(tpf_grid *g, int mode, const double *x, double *y, const double *d0, double *part,
                       unsigned *nblk_out, hipStream_t s) {
  const Level &lv = g->lv[0];
  const unsigned nb = blocks_for(lv.N);
  *nblk_out = nb;
  const Geo G = geo(lv);
  auto go = [&](auto kern) {
    return launch(g, TPF_K_SPMV64, kern, nb, BS, s, G, (const double *)lv.A64, x, y, d0, part);
  };
  hipError_t e;
  if (g->dim == 3) {
    switch (mode) {
      case 1: e = go(k_spmv64<3, 1>); break;
      case 2: e = go(k_spmv64<3, 2>); break;
      case 3: e = go(k_spmv64<3, 3>); break;
      default: e = go(k_spmv64<3, 0>); break;
    }
  } else {
    switch (mode) {
      case 1: e = go(k_spmv64<2, 1>); break;
      case 2: e = go(k_spmv64<2, 2>); break;
      case 3: e = go(k_spmv64<2, 3>); break;
      default: e = go(k_spmv64<2, 0>); break;
    }
  }
  TPF_HIP(e);
  return TPF_OK;
}

}  // namespace tpf
