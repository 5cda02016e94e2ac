// Coarse-level operators of the geometric multigrid hierarchy (gfx950).
//
//   A_c = P^T (A_f - S_f) P + S_c,   S_c = lumped P^T S_f P on the S_n column,
//
// S_f the storage part of the fine centre blocks.  P interpolates each component
// separately: (bi/tri)linearly for the pressure, by piecewise-constant aggregation
// (coarse I <- fine 2I-1, 2I per axis) for the saturation; on the finest level the
// rows of P at Dirichlet components are zero.  One thread per coarse block (I, O)
// sums, per axis, the (d, o) pairs with fine row i = 2I + d, fine column j = i + o
// that carry a non-zero weight (tables below), so only 4 accumulators are live.  A
// coarse unknown whose prolongation column is empty (an aggregate made only of
// Dirichlet components) is decoupled and gets a unit diagonal.
#include "stencil.h"

namespace tpf {
namespace {

// Per axis and coarse offset O in {-1, 0, 1}: every (fine-row offset d, fine-column
// offset o) with j = 2I + d + o interpolating linearly from J = I + O.  The pairs are
// packed 4 bits each ((d+1) | (o+1) << 2) into one integer per O, so that no table
// is indexed at run time (which would put it in scratch memory); the linear weight
// P(j, J) is 1 for s = d + o = 2 O and 1/2 otherwise.  The aggregation weights are
// non-zero on a subset of these pairs.
struct AxisTerms {
  int n;      // number of pairs
  unsigned packed;
  bool flat;  // the absent z axis of 2D grids: the single pair (0, 0)
  __host__ __device__ __forceinline__ int d(int k) const { return flat ? 0 : (int)((packed >> (4 * k)) & 3u) - 1; }
  __host__ __device__ __forceinline__ int o(int k) const { return flat ? 0 : (int)((packed >> (4 * k + 2)) & 3u) - 1; }
};
__host__ __device__ __forceinline__ AxisTerms axis_terms(int O) {
  // O = -1: (-1,-1) (-1,0) (0,-1);  O = +1: (0,1) (1,0) (1,1);
  // O = 0: (-1,0) (0,-1) (-1,1) (0,0) (1,-1) (0,1) (1,0)
  if (O < 0) return AxisTerms{3, 0x140u, false};
  if (O > 0) return AxisTerms{3, 0xA69u, false};
  return AxisTerms{7, 0x6925814u, false};
}
__host__ __device__ __forceinline__ AxisTerms axis_flat() { return AxisTerms{1, 0u, true}; }
__host__ __device__ __forceinline__ double lin_col(int s, int O) { return s == 2 * O ? 1.0 : 0.5; }

// 1-D weights: linear row weight P(2I + d, I), aggregation row weight, aggregation
// column weight P_agg(j, J) for s = j - 2I and O = J - I.
__host__ __device__ __forceinline__ double lin_row(int d) { return d ? 0.5 : 1.0; }
__host__ __device__ __forceinline__ double agg_row(int d) { return d <= 0 ? 1.0 : 0.0; }
__host__ __device__ __forceinline__ double agg_col(int s, int O) { return (s == 2 * O - 1 || s == 2 * O) ? 1.0 : 0.0; }

// Lumped coarse storage of coarse vertex I, sum_i P_r(i, I) keep_S(i) S_f(i, r), and
// whether the prolongation columns of (I, p) and (I, S) carry any weight.
template <int DIM, bool MASK>
__host__ __device__ __forceinline__ void rap_storage(long long I, const Geo &F, const Geo &C,
                                                    const uint8_t *__restrict__ fmask,
                                                    const double *__restrict__ mf, double &ms0, double &ms1,
                                                    bool &live0, bool &live1) {
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
        double k0 = 1.0, k1 = 1.0;
        if (MASK) {
          const uint8_t m = fmask[i];
          if (m & 2) { k0 = 0.0; k1 = 0.0; }  // keep_S(i) = 0: no lumped storage at i
          if (m & 1) k0 = 0.0;                 // keep_p(i) = 0
          if (!(m & 1)) live0 = true;
          if (!(m & 2) && wa != 0.0) live1 = true;
        } else {
          live0 = true;
          if (wa != 0.0) live1 = true;
        }
        ms0 += wl * k0 * mf[2 * i];
        ms1 += wa * k1 * mf[2 * i + 1];
      }
}

// Block (I, I + T) of P^T (A_f - S_f) P: the sum over the per-axis (d, o) pairs of
// fine rows i = 2I + d and columns j = i + o (entries a0..a3 = (p,p), (p,S), (S,p),
// (S,S)).
template <int DIM, bool MASK>
__host__ __device__ __forceinline__ void rap_entry(long long I, int T, const Geo &F, const Geo &C,
                                                  const double *__restrict__ Af,
                                                  const uint8_t *__restrict__ fmask,
                                                  const double *__restrict__ mf, double (&a)[4]) {
  constexpr int CEN = DIM == 3 ? 13 : 4;
  int cx, cy, cz;
  vcoords(I, C, cx, cy, cz);
  const long long sy = F.nx, sz = (long long)F.nx * F.ny;
  const int Ox = T % 3 - 1, Oy = (T / 3) % 3 - 1, Oz = DIM == 3 ? T / 9 - 1 : 0;
  const AxisTerms tx = axis_terms(Ox), ty = axis_terms(Oy);
  const AxisTerms tz = DIM == 3 ? axis_terms(Oz) : axis_flat();
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int kz = 0; kz < tz.n; ++kz) {
    const int dz = tz.d(kz), oz = tz.o(kz);
    const int fz = (DIM == 3 ? 2 * cz : 0) + dz, jz = fz + oz;
    if (fz < 0 || fz >= F.nz || jz < 0 || jz >= F.nz) continue;
    const double rz_l = DIM == 3 ? lin_row(dz) : 1.0, rz_a = DIM == 3 ? agg_row(dz) : 1.0;
    const double cz_l = DIM == 3 ? lin_col(dz + oz, Oz) : 1.0, cz_a = DIM == 3 ? agg_col(dz + oz, Oz) : 1.0;
    for (int ky = 0; ky < ty.n; ++ky) {
      const int dy = ty.d(ky), oy = ty.o(ky);
      const int fy = 2 * cy + dy, jy = fy + oy;
      if (fy < 0 || fy >= F.ny || jy < 0 || jy >= F.ny) continue;
      const double ry_l = lin_row(dy), ry_a = agg_row(dy);
      const double cy_l = lin_col(dy + oy, Oy), cy_a = agg_col(dy + oy, Oy);
      for (int kx = 0; kx < tx.n; ++kx) {
        const int dx = tx.d(kx), ox = tx.o(kx);
        const int fx = 2 * cx + dx, jx = fx + ox;
        if (fx < 0 || fx >= F.nx || jx < 0 || jx >= F.nx) continue;
        const double rl = lin_row(dx) * ry_l * rz_l;          // P_p(i, I)
        const double ra = agg_row(dx) * ry_a * rz_a;          // P_S(i, I)
        const double cl = lin_col(dx + ox, Ox) * cy_l * cz_l;  // P_p(j, J)
        const double ca = agg_col(dx + ox, Ox) * cy_a * cz_a;  // P_S(j, J)
        const long long i = fx + sy * fy + sz * fz;
        const long long j = jx + sy * jy + sz * jz;
        const int oo = DIM == 3 ? (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1) : (ox + 1) + 3 * (oy + 1);
        const double2 *bp = reinterpret_cast<const double2 *>(Af + ((long long)oo * F.N + i) * 4);
        const double2 b01 = bp[0], b23 = bp[1];
        double e1 = b01.y, e3 = b23.y;
        if (oo == CEN) {  // flux part only: remove the fine storage
          e1 -= mf[2 * i];
          e3 -= mf[2 * i + 1];
        }
        double r0 = rl, r1 = ra, c0 = cl, c1 = ca;
        if (MASK) {
          const uint8_t mi = fmask[i], mj = fmask[j];
          if (mi & 1) r0 = 0.0;
          if (mi & 2) r1 = 0.0;
          if (mj & 1) c0 = 0.0;
          if (mj & 2) c1 = 0.0;
        }
        a0 += r0 * b01.x * c0;
        a1 += r0 * e1 * c1;
        a2 += r1 * b23.x * c0;
        a3 += r1 * e3 * c1;
      }
    }
  }
  a[0] = a0;
  a[1] = a1;
  a[2] = a2;
  a[3] = a3;
}

// Complete coarse block (I, I + T): the Galerkin flux part plus, on the diagonal,
// the lumped storage and the unit entry of an empty prolongation column.
template <int DIM, bool MASK>
__host__ __device__ __forceinline__ void rap_block(long long I, int T, const Geo &F, const Geo &C,
                                                  const double *__restrict__ Af,
                                                  const uint8_t *__restrict__ fmask,
                                                  const double *__restrict__ mf, double *__restrict__ Ac,
                                                  float *__restrict__ Ac32, double *__restrict__ mc) {
  constexpr int CEN = DIM == 3 ? 13 : 4;
  double a[4];
  rap_entry<DIM, MASK>(I, T, F, C, Af, fmask, mf, a);
  if (T == CEN) {
    double ms0, ms1;
    bool live0, live1;
    rap_storage<DIM, MASK>(I, F, C, fmask, mf, ms0, ms1, live0, live1);
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

// Thread mapping: each wavefront computes one coarse offset T for 64 consecutive
// coarse vertices (uniform trip counts within the wavefront); the NST wavefronts of a
// vertex tile are adjacent, and the XCD-aware block order keeps neighbouring tiles on
// one XCD, so the fine rows they share are read from that XCD's L2.
template <int DIM>
__host__ __device__ __forceinline__ bool rap_thread(long long wave, int lane, long long Nc, long long &I, int &T) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  const long long tile = wave / NST;
  T = (int)(wave % NST);
  I = tile * 64 + lane;
  return I < Nc;
}

template <int DIM, bool MASK>
__global__ void __launch_bounds__(BS) k_rap(const Geo F, const Geo C, const double *__restrict__ Af,
                                            const uint8_t *__restrict__ fmask, const double *__restrict__ mf,
                                            double *__restrict__ Ac, float *__restrict__ Ac32,
                                            double *__restrict__ mc) {
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const long long wave = (long long)blk * (BS / 64) + (threadIdx.x >> 6);
  long long I;
  int T;
  if (!rap_thread<DIM>(wave, threadIdx.x & 63, C.N, I, T)) return;
  rap_block<DIM, MASK>(I, T, F, C, Af, fmask, mf, Ac, Ac32, mc);
}

}  // namespace

tpf_status launch_rap(int dim, bool mask, const int nf[3], long long Nf, const int nc[3], long long Nc,
                      const double *Af, const uint8_t *fmask, const double *mf, double *Ac, float *Ac32,
                      double *mc, hipStream_t s) {
  const Geo F = geo_of(nf, Nf), C = geo_of(nc, Nc);
  const long long waves = ((Nc + 63) / 64) * (dim == 3 ? 27 : 9);
  const unsigned nb = (unsigned)((waves + BS / 64 - 1) / (BS / 64));
  if (dim == 3) {
    if (mask) k_rap<3, true><<<nb, BS, 0, s>>>(F, C, Af, fmask, mf, Ac, Ac32, mc);
    else k_rap<3, false><<<nb, BS, 0, s>>>(F, C, Af, fmask, mf, Ac, Ac32, mc);
  } else {
    if (mask) k_rap<2, true><<<nb, BS, 0, s>>>(F, C, Af, fmask, mf, Ac, Ac32, mc);
    else k_rap<2, false><<<nb, BS, 0, s>>>(F, C, Af, fmask, mf, Ac, Ac32, mc);
  }
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

}  // namespace tpf
