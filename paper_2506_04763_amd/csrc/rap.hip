// Coarse-level operators of the geometric multigrid hierarchy (gfx950).
//
//   A_c = P^T (A_f - S_f) P + S_c,   S_c = lumped P^T S_f P on the S_n column,
//
// S_f the storage part of the fine centre blocks.  P interpolates each component
// separately: (bi/tri)linearly for the pressure, by piecewise-constant aggregation
// (coarse I <- fine 2I-1, 2I per axis) for the saturation; on the finest level the
// rows of P at Dirichlet components are zero.  On the finest level the rows enter
// in volume-balance form: at a vertex without Dirichlet components the wetting
// row becomes itself plus vr = rho_w/rho_n times the non-wetting row (storage and
// flux parts alike), so that the row restricted by the linear P carries the
// total-mobility pressure Laplacian even where the wetting phase is immobile; the
// smoother is unaffected (block Jacobi is invariant under a block-diagonal row
// transform) and the restriction of the finest residual applies the same transform.
// The product is formed in two passes
// through a scratch array (A P first, then P^T (A P); see below).  A coarse unknown
// whose prolongation column is empty (an aggregate made only of Dirichlet
// components) is decoupled and gets a unit diagonal.
#include "stencil.h"

namespace tpf {
namespace {

// 1-D weights of P at fine row 2I + d for coarse I: linear and aggregation.
__host__ __device__ __forceinline__ double lin_row(int d) { return d ? 0.5 : 1.0; }
__host__ __device__ __forceinline__ double agg_row(int d) { return d <= 0 ? 1.0 : 0.0; }

// Lumped coarse storage of coarse vertex I, sum_i P_r(i, I) keep_S(i) S_f(i, r), and
// whether the prolongation columns of (I, p) and (I, S) carry any weight.
template <int DIM, bool MASK>
__host__ __device__ __forceinline__ void rap_storage(long long I, const Geo &F, const Geo &C,
                                                    const uint8_t *__restrict__ fmask,
                                                    const double *__restrict__ mf, double vr, double &ms0,
                                                    double &ms1, bool &live0, bool &live1) {
  int cx, cy, cz;
  vcoords(I, C, cx, cy, cz);
  const long long sy = F.nx, sz = (long long)F.nx * F.ny;
  ms0 = 0.0;
  ms1 = 0.0;
  live0 = false;
  live1 = false;
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int fx = 2 * cx + dx, fy = 2 * cy + dy, fz = (DIM == 3 ? 2 * cz : 0) + dz;
        if (fx < 0 || fy < 0 || fz < 0 || fx >= F.nx || fy >= F.ny || fz >= F.nz) continue;
        const long long i = fx + sy * fy + sz * fz;
        const double wl = lin_row(dx) * lin_row(dy) * (DIM == 3 ? lin_row(dz) : 1.0);
        const double wa = agg_row(dx) * agg_row(dy) * (DIM == 3 ? agg_row(dz) : 1.0);
        double k0 = 1.0, k1 = 1.0, s0 = mf[2 * i];
        if (MASK) {
          const uint8_t m = fmask[i];
          if (!m) s0 += vr * mf[2 * i + 1];   // volume-balance row
          if (m & 2) { k0 = 0.0; k1 = 0.0; }  // keep_S(i) = 0: no lumped storage at i
          if (m & 1) k0 = 0.0;                 // keep_p(i) = 0
          if (!(m & 1)) live0 = true;
          if (!(m & 2) && wa != 0.0) live1 = true;
        } else {
          live0 = true;
          if (wa != 0.0) live1 = true;
        }
        ms0 += wl * k0 * s0;
        ms1 += wa * k1 * mf[2 * i + 1];
      }
}

// 1-D weights of a column of P at fine coordinate j for coarse coordinate J: linear
// interpolation (pressure) and aggregation of fine j into coarse (j + 1) / 2 (saturation).
__host__ __device__ __forceinline__ double lin_w(int j, int J) {
  const int d = j - 2 * J;
  return d == 0 ? 1.0 : ((d == 1 || d == -1) ? 0.5 : 0.0);
}
__host__ __device__ __forceinline__ double agg_w(int j, int J) { return ((j + 1) >> 1) == J ? 1.0 : 0.0; }

// The product runs in two passes over a scratch array B of NST blocks per fine vertex.
// Pass 1 (fine vertex i, slot s): B(i, s) = sum_j (A_f - S_f)(i, j) P(j, J) for the
// coarse column J = (i >> 1) + s, s in {-1, 0, 1} per axis (the only coarse columns
// a fine row reaches); the p column of A is weighted by the linear P, the S column by
// the aggregation P, zero at fine Dirichlet components j.  Pass 2 (coarse block
// (I, O)): A_c(I, I + O) = sum_i P_r(i, I) B(i, I + O - (i >> 1)) over the fine rows
// i = 2I + d of the support of I.  Each fine matrix block is read once per slot it
// reaches instead of once per coarse block using it.
template <int DIM, bool MASK>
__host__ __device__ __forceinline__ void rap_ap_entry(long long i, int slot, const Geo &F, const Geo &C,
                                                     const double *__restrict__ Af,
                                                     const uint8_t *__restrict__ fmask,
                                                     const double *__restrict__ mf, double vr, double (&b)[4]) {
  constexpr int CEN = DIM == 3 ? 13 : 4;
  b[0] = b[1] = b[2] = b[3] = 0.0;
  int fx, fy, fz;
  vcoords(i, F, fx, fy, fz);
  const int Jx = (fx >> 1) + slot % 3 - 1, Jy = (fy >> 1) + (slot / 3) % 3 - 1;
  const int Jz = DIM == 3 ? (fz >> 1) + slot / 9 - 1 : 0;
  if (Jx < 0 || Jy < 0 || Jz < 0 || Jx >= C.nx || Jy >= C.ny || Jz >= C.nz) return;
  const long long sy = F.nx, sz = (long long)F.nx * F.ny;
  for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz) {
    const int jz = fz + oz;
    if (jz < 0 || jz >= F.nz) continue;
    const double lz = DIM == 3 ? lin_w(jz, Jz) : 1.0, az = DIM == 3 ? agg_w(jz, Jz) : 1.0;
    if (lz == 0.0 && az == 0.0) continue;
    for (int oy = -1; oy <= 1; ++oy) {
      const int jy = fy + oy;
      if (jy < 0 || jy >= F.ny) continue;
      const double ly = lin_w(jy, Jy) * lz, ay = agg_w(jy, Jy) * az;
      if (ly == 0.0 && ay == 0.0) continue;
      for (int ox = -1; ox <= 1; ++ox) {
        const int jx = fx + ox;
        if (jx < 0 || jx >= F.nx) continue;
        double wl = lin_w(jx, Jx) * ly, wa = agg_w(jx, Jx) * ay;
        if (wl == 0.0 && wa == 0.0) continue;
        if (MASK) {
          const uint8_t mj = fmask[jx + sy * jy + sz * jz];
          if (mj & 1) wl = 0.0;
          if (mj & 2) wa = 0.0;
        }
        const int o = DIM == 3 ? (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1) : (ox + 1) + 3 * (oy + 1);
        const double2 *bp = reinterpret_cast<const double2 *>(Af + ((long long)o * F.N + i) * 4);
        const double2 b01 = bp[0], b23 = bp[1];
        double e1 = b01.y, e3 = b23.y;
        if (o == CEN) {  // flux part only: remove the fine storage
          e1 -= mf[2 * i];
          e3 -= mf[2 * i + 1];
        }
        b[0] += b01.x * wl;
        b[1] += e1 * wa;
        b[2] += b23.x * wl;
        b[3] += e3 * wa;
      }
    }
  }
  if (MASK && !fmask[i]) {  // volume-balance row of a vertex without Dirichlet components
    b[0] += vr * b[2];
    b[1] += vr * b[3];
  }
}

template <int DIM, bool MASK>
__host__ __device__ __forceinline__ void rap_ptb_entry(long long I, int T, const Geo &F, const Geo &C,
                                                      const double *__restrict__ B,
                                                      const uint8_t *__restrict__ fmask, double (&a)[4]) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  a[0] = a[1] = a[2] = a[3] = 0.0;
  int cx, cy, cz;
  vcoords(I, C, cx, cy, cz);
  const int Jx = cx + T % 3 - 1, Jy = cy + (T / 3) % 3 - 1, Jz = DIM == 3 ? cz + T / 9 - 1 : 0;
  if (Jx < 0 || Jy < 0 || Jz < 0 || Jx >= C.nx || Jy >= C.ny || Jz >= C.nz) return;
  const long long sy = F.nx, sz = (long long)F.nx * F.ny;
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
    const int iz = (DIM == 3 ? 2 * cz : 0) + dz, qz = DIM == 3 ? Jz - (iz >> 1) : 0;
    if (iz < 0 || iz >= F.nz || qz < -1 || qz > 1) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int iy = 2 * cy + dy, qy = Jy - (iy >> 1);
      if (iy < 0 || iy >= F.ny || qy < -1 || qy > 1) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int ix = 2 * cx + dx, qx = Jx - (ix >> 1);
        if (ix < 0 || ix >= F.nx || qx < -1 || qx > 1) continue;
        double wl = lin_row(dx) * lin_row(dy) * (DIM == 3 ? lin_row(dz) : 1.0);  // P_p(i, I)
        double wa = agg_row(dx) * agg_row(dy) * (DIM == 3 ? agg_row(dz) : 1.0);  // P_S(i, I)
        const long long i = ix + sy * iy + sz * iz;
        if (MASK) {
          const uint8_t mi = fmask[i];
          if (mi & 1) wl = 0.0;
          if (mi & 2) wa = 0.0;
        }
        if (wl == 0.0 && wa == 0.0) continue;
        const int slot = DIM == 3 ? (qx + 1) + 3 * (qy + 1) + 9 * (qz + 1) : (qx + 1) + 3 * (qy + 1);
        const double2 *bp = reinterpret_cast<const double2 *>(B + ((long long)slot * F.N + i) * 4);
        const double2 b01 = bp[0], b23 = bp[1];
        a[0] += wl * b01.x;
        a[1] += wl * b01.y;
        a[2] += wa * b23.x;
        a[3] += wa * b23.y;
      }
    }
  }
  (void)NST;
}

// Complete coarse block (I, I + T): the Galerkin flux part plus, on the diagonal,
// the lumped storage and the unit entry of an empty prolongation column.
template <int DIM, bool MASK>
__host__ __device__ __forceinline__ void rap_block(long long I, int T, const Geo &F, const Geo &C,
                                                  const double *__restrict__ B,
                                                  const uint8_t *__restrict__ fmask,
                                                  const double *__restrict__ mf, double vr, double *__restrict__ Ac,
                                                  float *__restrict__ Ac32, double *__restrict__ mc) {
  constexpr int CEN = DIM == 3 ? 13 : 4;
  double a[4];
  rap_ptb_entry<DIM, MASK>(I, T, F, C, B, fmask, a);
  if (T == CEN) {
    double ms0, ms1;
    bool live0, live1;
    rap_storage<DIM, MASK>(I, F, C, fmask, mf, vr, ms0, ms1, live0, live1);
    a[1] += ms0;
    a[3] += ms1;
    if (!live0) a[0] += 1.0;
    if (!live1) a[3] += 1.0;
    *reinterpret_cast<double2 *>(mc + 2 * I) = make_double2(ms0, ms1);
  }
  double *dst = Ac + ((long long)T * C.N + I) * 4;
  reinterpret_cast<double2 *>(dst)[0] = make_double2(a[0], a[1]);
  reinterpret_cast<double2 *>(dst)[1] = make_double2(a[2], a[3]);
  if (Ac32)
    *reinterpret_cast<float4 *>(Ac32 + ((long long)T * C.N + I) * 4) =
        make_float4((float)a[0], (float)a[1], (float)a[2], (float)a[3]);
}

// Thread mapping of both passes: each wavefront computes one slot / coarse offset T
// for 64 consecutive vertices (uniform loops within the wavefront); the NST
// wavefronts of a vertex tile are adjacent, and the XCD-aware block order keeps
// neighbouring tiles on one XCD, so the rows they share are read from that XCD's L2.
template <int DIM>
__host__ __device__ __forceinline__ bool rap_thread(long long wave, int lane, long long N, long long &I, int &T) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  const long long tile = wave / NST;
  T = (int)(wave % NST);
  I = tile * 64 + lane;
  return I < N;
}

template <int DIM, bool MASK>
__global__ void __launch_bounds__(BS) k_rap_ap(const Geo F, const Geo C, const double *__restrict__ Af,
                                               const uint8_t *__restrict__ fmask, const double *__restrict__ mf,
                                               const double vr, double *__restrict__ B) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long wave = (long long)blk * (BS / 64) + (threadIdx.x >> 6);
  long long i;
  int slot;
  if (!rap_thread<DIM>(wave, threadIdx.x & 63, F.N, i, slot)) return;
  double b[4];
  rap_ap_entry<DIM, MASK>(i, slot, F, C, Af, fmask, mf, vr, b);
  double *dst = B + ((long long)slot * F.N + i) * 4;
  reinterpret_cast<double2 *>(dst)[0] = make_double2(b[0], b[1]);
  reinterpret_cast<double2 *>(dst)[1] = make_double2(b[2], b[3]);
}

template <int DIM, bool MASK>
__global__ void __launch_bounds__(BS) k_rap(const Geo F, const Geo C, const double *__restrict__ B,
                                            const uint8_t *__restrict__ fmask, const double *__restrict__ mf,
                                            const double vr, double *__restrict__ Ac, float *__restrict__ Ac32,
                                            double *__restrict__ mc) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long wave = (long long)blk * (BS / 64) + (threadIdx.x >> 6);
  long long I;
  int T;
  if (!rap_thread<DIM>(wave, threadIdx.x & 63, C.N, I, T)) return;
  rap_block<DIM, MASK>(I, T, F, C, B, fmask, mf, vr, Ac, Ac32, mc);
}

}  // namespace

tpf_status launch_rap(int dim, bool mask, const int nf[3], long long Nf, const int nc[3], long long Nc,
                      const double *Af, const uint8_t *fmask, const double *mf, double vr, double *B, double *Ac,
                      float *Ac32, double *mc, hipStream_t s) {
  const Geo F = geo_of(nf, Nf), C = geo_of(nc, Nc);
  const int nst = dim == 3 ? 27 : 9;
  const long long wf = ((Nf + 63) / 64) * nst, wc = ((Nc + 63) / 64) * nst;
  const unsigned nbf = (unsigned)((wf + BS / 64 - 1) / (BS / 64)), nbc = (unsigned)((wc + BS / 64 - 1) / (BS / 64));
  if (dim == 3) {
    if (mask) {
      k_rap_ap<3, true><<<nbf, BS, 0, s>>>(F, C, Af, fmask, mf, vr, B);
      k_rap<3, true><<<nbc, BS, 0, s>>>(F, C, B, fmask, mf, vr, Ac, Ac32, mc);
    } else {
      k_rap_ap<3, false><<<nbf, BS, 0, s>>>(F, C, Af, fmask, mf, vr, B);
      k_rap<3, false><<<nbc, BS, 0, s>>>(F, C, B, fmask, mf, vr, Ac, Ac32, mc);
    }
  } else {
    if (mask) {
      k_rap_ap<2, true><<<nbf, BS, 0, s>>>(F, C, Af, fmask, mf, vr, B);
      k_rap<2, true><<<nbc, BS, 0, s>>>(F, C, B, fmask, mf, vr, Ac, Ac32, mc);
    } else {
      k_rap_ap<2, false><<<nbf, BS, 0, s>>>(F, C, Af, fmask, mf, vr, B);
      k_rap<2, false><<<nbc, BS, 0, s>>>(F, C, B, fmask, mf, vr, Ac, Ac32, mc);
    }
  }
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

}  // namespace tpf
