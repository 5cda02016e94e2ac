// Box-method residual and stage-matrix assembly on structured Q1 grids (gfx950).
//
// Vertex-centric gather (no atomics, deterministic): the thread(s) of a vertex visit
// the 2^d cells around it.  For every cell they evaluate, at the cell's corners, the
// sub-control-volume saturation of the p_dmin interface condition (Eq. hSw) and the
// element-local capillary pressure, then the fluxes through the d sub-control-volume
// faces incident to the vertex (Section 3.1, Eqs. dsW/dpN; upwinding Section 3.2;
// barrier on the non-wetting mobility only, Eqs. krn_ip/krw_ip) with their exact
// derivatives.  The row is accumulated in registers and written once as 2x2 blocks in
// the [offset][vertex][4] layout (coalesced 32-byte stores per lane).  In 3D the
// matrix kernel splits each vertex over two threads by the z half of its cells (18
// stencil slots each) and adds the shared dz = 0 plane through LDS in a fixed order,
// which keeps the accumulators in registers.
//
// Discretisation choices (shared with the independent FP64 oracle, from the paper's
// text): unknowns (p_w, S_n); the convective non-wetting flux is upwinded with the
// velocity -K/mu_n (grad p_w - rho_n g) and the capillary flux -k_rn K/mu_n grad p_c
// is central, k_rn taken at the Q1-interpolated hat saturation of the integration
// point; Brooks-Corey p_c = p_d S_e^(-1/lam) and Burdine k_rw = S_e^((2+3 lam)/lam),
// k_rn = (1-S_e)^2 (1 - S_e^((2+lam)/lam)) (or the polynomial laws a_w S_e^2,
// a_n (1 - S_e) of Section 5's cases 4 and 5), S_e clamped to [1e-6, 1]; storage of each
// sub-control volume uses its hat saturation; SCVF oriented from lower to higher
// vertex index with ties upwinded to the lower one; integration point at the face
// barycentre.
#include <type_traits>
#include <utility>

#include "tpf_internal.h"

namespace tpf {
namespace {

__host__ __device__ __forceinline__ void eff_sat(double sn, const Phys &P, double &se, double &dse) {
  const double raw = ((1.0 - sn) - P.swr) / P.D;
  if (raw < SE_MIN) {
    se = SE_MIN; dse = 0.0;
  } else if (raw > 1.0) {
    se = 1.0; dse = 0.0;
  } else {
    se = raw; dse = -1.0 / P.D;
  }
}

// Natural logarithm of a positive, finite, normal x: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...) with
// s = (m - 1)/(m + 1), |s| <= 0.172, so terms up to s^25 reach double precision
// (a few ulp overall); log 2 is split into a high part exact in 32 bits and the rest.
__host__ __device__ __forceinline__ double log_pos(double x) {
  int e;
  double m = frexp(x, &e);  // m in [0.5, 1)
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double q = 1.0 / 25.0;
  q = fma(q, z, 1.0 / 23.0);
  q = fma(q, z, 1.0 / 21.0);
  q = fma(q, z, 1.0 / 19.0);
  q = fma(q, z, 1.0 / 17.0);
  q = fma(q, z, 1.0 / 15.0);
  q = fma(q, z, 1.0 / 13.0);
  q = fma(q, z, 1.0 / 11.0);
  q = fma(q, z, 1.0 / 9.0);
  q = fma(q, z, 1.0 / 7.0);
  q = fma(q, z, 1.0 / 5.0);
  q = fma(q, z, 1.0 / 3.0);
  const double lm = 2.0 * s + 2.0 * s * z * q;
  constexpr double LN2_HI = 0.693147180369123816490;    // 32 significant bits
  constexpr double LN2_LO = 1.90821492927058770002e-10;  // log 2 - LN2_HI
  return fma((double)e, LN2_HI, fma((double)e, LN2_LO, lm));
}

// exp(x) for finite x: x = k log 2 + r with k = round(x / log 2), |r| <= log(2)/2
// (reduction with the split log 2), exp(r) by its Taylor series to r^14/14!, scaled
// by 2^k (overflow gives inf, underflow 0 or a subnormal).
__host__ __device__ __forceinline__ double exp_fin(double x) {
  constexpr double LN2_HI = 0.693147180369123816490;
  constexpr double LN2_LO = 1.90821492927058770002e-10;
  const double k = rint(x * 1.44269504088896340736);
  const double r = fma(-k, LN2_LO, fma(-k, LN2_HI, x));
  double q = 1.0 / 87178291200.0;           // 1/14!
  q = fma(q, r, 1.0 / 6227020800.0);        // 1/13!
  q = fma(q, r, 1.0 / 479001600.0);
  q = fma(q, r, 1.0 / 39916800.0);
  q = fma(q, r, 1.0 / 3628800.0);
  q = fma(q, r, 1.0 / 362880.0);
  q = fma(q, r, 1.0 / 40320.0);
  q = fma(q, r, 1.0 / 5040.0);
  q = fma(q, r, 1.0 / 720.0);
  q = fma(q, r, 1.0 / 120.0);
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  q = fma(q, r, 1.0);
  return ldexp(q, (int)k);
}

// Every Brooks-Corey / Burdine power of one effective saturation follows from
// t = S_e^(1/lam), one log and one exp: p_c = p_d / t, S_e^((2+lam)/lam) = S_e t^2,
// S_e^((2+3 lam)/lam) = S_e^3 t^2 (S_e >= 1e-6, so the log is finite).
__host__ __device__ __forceinline__ double root_lam(double se, double inv_lam) {
  return exp_fin(log_pos(se) * inv_lam);
}

// Wetting relative permeability and its derivative w.r.t. S_n: Burdine, or the
// polynomial law a_w S_e^2 of Tables case4/case5 (the law is uniform over a launch).
__host__ __device__ __forceinline__ void krw(double sn, double inv_lam, const Phys &P, double &k, double &dk) {
  double se, dse;
  eff_sat(sn, P, se, dse);
  if (P.kr_model == TPF_KR_POLY) {
    k = P.kr_aw * se * se;
    dk = 2.0 * P.kr_aw * se * dse;
    return;
  }
  const double t = root_lam(se, inv_lam);
  k = se * se * se * t * t;
  dk = (3.0 + 2.0 * inv_lam) * (k / se) * dse;
}

// Non-wetting relative permeability from S_e (and, for Burdine, t = S_e^(1/lam)),
// and its derivative w.r.t. S_e: Burdine, or the polynomial law a_n (1 - S_e).
__host__ __device__ __forceinline__ void krn_se(double se, double t, double inv_lam, const Phys &P, double &k,
                                               double &dk_dse) {
  if (P.kr_model == TPF_KR_POLY) {
    k = P.kr_an * (1.0 - se);
    dk_dse = -P.kr_an;
    return;
  }
  const double sa = se * t * t;
  const double om = 1.0 - se;
  k = om * om * (1.0 - sa);
  dk_dse = -2.0 * om * (1.0 - sa) - om * om * (1.0 + 2.0 * inv_lam) * t * t;
}

// Non-wetting relative permeability and its derivative w.r.t. S_n.
__host__ __device__ __forceinline__ void krn(double sn, double inv_lam, const Phys &P, double &k, double &dk) {
  double se, dse;
  eff_sat(sn, P, se, dse);
  double dk_dse;
  krn_se(se, P.kr_model == TPF_KR_POLY ? 1.0 : root_lam(se, inv_lam), inv_lam, P, k, dk_dse);
  dk = dk_dse * dse;
}

// ---------------------------------------------------------------------------------
// Per-vertex pre-processing: p_dmin,i = min of the adjacent cells' entry pressures,
// lambda of the reference medium (lowest cell index attaining the minimum) and the
// Neumann sources integrated exactly over the dual-box face.
// ---------------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(BS) k_setup(const Phys P, const double *__restrict__ pd,
                                              const double *__restrict__ lam, const Patches pt,
                                              double *__restrict__ pdmin, double *__restrict__ lamref,
                                              double *__restrict__ Q) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= P.N) return;
  int ix, iy, iz;
  grid_coords(v, P.nx, P.ny, ix, iy, iz);
  double best = 1.0e308;
  long long bestc = -1;
  // visit adjacent cells in increasing cell index so ties keep the lowest index
  for (int cz = (DIM == 3 ? -1 : 0); cz <= 0; ++cz)
    for (int cy = -1; cy <= 0; ++cy)
      for (int cx = -1; cx <= 0; ++cx) {
        const int ox = ix + cx, oy = iy + cy, oz = iz + cz;
        if (ox < 0 || oy < 0 || oz < 0 || ox >= P.ncx || oy >= P.ncy || oz >= P.ncz) continue;
        const long long c = ox + (long long)P.ncx * (oy + (long long)P.ncy * oz);
        const double p = pd[c];
        if (p < best) { best = p; bestc = c; }
      }
  pdmin[v] = best;
  lamref[v] = lam[bestc];
  const double x[3] = {ix * P.h[0], iy * P.h[1], (DIM == 3 ? iz * P.h[2] : 0.0)};
  const double ext[3] = {(P.nx - 1) * P.h[0], (P.ny - 1) * P.h[1], (P.nz - 1) * P.h[2]};
  double q[2] = {0.0, 0.0};
  for (int k = 0; k < pt.n; ++k) {
    const PatchDev &pa = pt.p[k];
    const int a = pa.axis;
    const double face = pa.side == 0 ? 0.0 : ext[a];
    if (fabs(x[a] - face) > 1e-9 * (ext[a] + 1.0)) continue;
    double meas = 1.0;
    int kk = 0;
    for (int b = 0; b < DIM; ++b) {
      if (b == a) continue;
      const double lo = fmax(fmax(x[b] - 0.5 * P.h[b], 0.0), pa.lo[kk]);
      const double hi = fmin(fmin(x[b] + 0.5 * P.h[b], ext[b]), pa.hi[kk]);
      meas *= fmax(hi - lo, 0.0);
      ++kk;
    }
    q[pa.phase] += pa.rate * meas;
  }
  Q[2 * v] += q[0];  // on top of the vertex sources uploaded at creation
  Q[2 * v + 1] += q[1];
}

// Vertex capillary pressure in the reference medium, P_i = p_dmin,i J(S_i), and its
// derivative w.r.t. S_n,i (an input to every hat evaluation around the vertex).
__host__ __device__ __forceinline__ void vertex_pc(const long long v, const Phys &P, const double *__restrict__ u,
                                                  const double *__restrict__ pdmin,
                                                  const double *__restrict__ lamref,
                                                  double *__restrict__ pv) {
  double se, dse;
  eff_sat(u[2 * v + 1], P, se, dse);
  const double lr = lamref[v];
  const double pc = pdmin[v] / root_lam(se, 1.0 / lr);
  pv[2 * v] = pc;
  pv[2 * v + 1] = pc * (-1.0 / lr) / se * dse;
}

__global__ void __launch_bounds__(BS) k_vertex_pc(const Phys P, const double *__restrict__ u,
                                                  const double *__restrict__ pdmin,
                                                  const double *__restrict__ lamref,
                                                  double *__restrict__ pv) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= P.N) return;
  vertex_pc(v, P, u, pdmin, lamref, pv);
}

template <int DIM>
__host__ __device__ __forceinline__ constexpr int stencil_index(int dx, int dy, int dz) {
  return DIM == 3 ? (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1) : (dx + 1) + 3 * (dy + 1);
}

__host__ __device__ __forceinline__ constexpr int bit(int l, int a) { return (l >> a) & 1; }

struct CellIn {
  const double *u, *Kc, *phic, *pdc, *lamc, *pdmin, *pv;
  const double *cp;  // per (cell, corner) laws from corner_pass (CP doubles each), or null
};

// The quantities of one (cell, corner) pair that depend only on the corner vertex
// and the cell, in this order: the hat saturation of the corner in the cell and its
// S_n-derivative, the element-local capillary pressure and its derivative, the
// non-wetting mobility at the hat saturation and its derivative, the wetting mobility
// at the plain saturation and its derivative (both derivatives w.r.t. S_n).
constexpr int CP = 8;

// Interface condition (Eq. hSw) and the laws at corner saturation sn of a cell with
// entry pressure pde and 1/lambda il; pdm = p_dmin of the corner, pvl = (P, dP/dS_n)
// of the corner.
// The saturation of the sub-control volume (vertex, cell) under the interface
// condition (Eq. hSw): equal entry pressure / barrier / continuity, as a non-wetting
// saturation, and its derivative w.r.t. the vertex S_n.
__host__ __device__ __forceinline__ void hat_sat(const double sn, const double pdm, const double2 pvl,
                                                const double pde, const double lame, const Phys &P, double &sh,
                                                double &dsh) {
  if (pde == pdm) {
    sh = sn; dsh = 1.0;
  } else if (pde >= pvl.x) {
    sh = P.snr; dsh = 0.0;
  } else {
    const double ses = exp_fin(-lame * log_pos(pvl.x / pde));
    sh = 1.0 - (P.swr + ses * P.D);
    dsh = -P.D * (-lame * ses / pvl.x * pvl.y);
  }
}

__host__ __device__ __forceinline__ void corner_laws(const double sn, const double pdm, const double2 pvl,
                                                    const double pde, const double lame, const double il,
                                                    const Phys &P, double &sh, double &dsh, double &pc,
                                                    double &dpc, double &khn, double &dkhn) {
  hat_sat(sn, pdm, pvl, pde, lame, P, sh, dsh);
  double se, dse;
  eff_sat(sh, P, se, dse);
  const double t = root_lam(se, il);
  pc = pde / t;
  dpc = pc * (-il) / se * dse * dsh;
  // non-wetting mobility of the corner at its hat saturation (for upwinding)
  double dk_dse;
  krn_se(se, t, il, P, khn, dk_dse);
  dkhn = dk_dse * dse;
}

// All corners of cell c: the CP quantities of corner l at cp[(c * 2^d + l) * CP].
template <int DIM>
__host__ __device__ __forceinline__ void corner_pass(const long long c, const Phys &P, const CellIn &in,
                                                    double *__restrict__ cp) {
  constexpr int NC = 1 << DIM;
  int ox, oy, oz;
  grid_coords(c, P.ncx, P.ncy, ox, oy, oz);
  const long long sy = P.nx, sz = (long long)P.nx * P.ny;
  const long long v0 = ox + sy * oy + sz * oz;
  const double pde = in.pdc[c], lame = in.lamc[c];
  const double il = 1.0 / lame;
#pragma unroll
  for (int l = 0; l < NC; ++l) {
    const long long vl = v0 + bit(l, 0) + sy * bit(l, 1) + sz * ((DIM == 3) ? bit(l, 2) : 0);
    const double sn = in.u[2 * vl + 1];
    const double2 pvl = *reinterpret_cast<const double2 *>(in.pv + 2 * vl);
    double q[CP];
    corner_laws(sn, in.pdmin[vl], pvl, pde, lame, il, P, q[0], q[1], q[2], q[3], q[4], q[5]);
    krw(sn, il, P, q[6], q[7]);
    double2 *dst = reinterpret_cast<double2 *>(cp + (c * NC + l) * CP);
#pragma unroll
    for (int k = 0; k < CP / 2; ++k) dst[k] = make_double2(q[2 * k], q[2 * k + 1]);
  }
}

// ---------------------------------------------------------------------------------
// Cell contributions to the residual row of vertex v and (WANT_A) to its row of
// -dF/du: cells with corner index cc, restricted to bit 2 of cc == HALF when
// HALF >= 0; stencil slot o goes to acc[o - BASE].  Storage derivatives are returned
// in mwS, mnS (dm_w/dS_n and dm_n/dS_n of the vertex).
// ---------------------------------------------------------------------------------
template <int DIM, bool WANT_A, int HALF, int BASE, int NSLOT, bool PAIRS = false>
__host__ __device__ __forceinline__ void accumulate_cells(const long long v, const Phys &P, const CellIn &in,
                                                         double (&acc)[NSLOT][4], double &Fw, double &Fn,
                                                         double &mwS, double &mnS) {
  constexpr int NC = 1 << DIM;
  int ix, iy, iz;
  grid_coords(v, P.nx, P.ny, ix, iy, iz);
  const long long sy = P.nx, sz = (long long)P.nx * P.ny;
  const double rw = P.rho_w, rn = P.rho_n;

  // The body runs once per adjacent cell with the corner index `cc` a template
  // constant, so every stencil slot of the row accumulator is a compile-time index.
  auto cell = [&]<int cc>(std::integral_constant<int, cc>) {
    if constexpr (HALF >= 0 && bit(cc, 2) != HALF) {
      return;
    } else {
      // cell whose corner `cc` is this vertex: origin = vertex - bits(cc)
      const int ox = ix - bit(cc, 0), oy = iy - bit(cc, 1), oz = (DIM == 3) ? iz - bit(cc, 2) : 0;
      if (ox < 0 || oy < 0 || oz < 0 || ox >= P.ncx || oy >= P.ncy || oz >= P.ncz) return;
      const long long c = ox + (long long)P.ncx * (oy + (long long)P.ncy * oz);
      const double Ke = in.Kc[c], phie = in.phic[c], pde = in.pdc[c], lame = in.lamc[c];
      const double il = 1.0 / lame;
      double p[NC], sn[NC], sh[NC], dsh[NC], pc[NC], dpc[NC], khn[NC], dkhn[NC], kwl[NC], dkwl[NC];
#pragma unroll
      for (int l = 0; l < NC; ++l) {
        const int dx = bit(l, 0) - bit(cc, 0), dy = bit(l, 1) - bit(cc, 1);
        const int dz = (DIM == 3) ? bit(l, 2) - bit(cc, 2) : 0;
        const long long vl = v + dx + sy * dy + sz * dz;
        const double2 ul = *reinterpret_cast<const double2 *>(in.u + 2 * vl);
        p[l] = ul.x;
        sn[l] = ul.y;
        if constexpr (PAIRS) {  // the pair's laws from the corner pass
          const double2 *q = reinterpret_cast<const double2 *>(in.cp + (c * NC + l) * CP);
          const double2 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
          sh[l] = q0.x; dsh[l] = q0.y; pc[l] = q1.x; dpc[l] = q1.y;
          khn[l] = q2.x; dkhn[l] = q2.y; kwl[l] = q3.x; dkwl[l] = q3.y;
        } else {
          const double2 pvl = *reinterpret_cast<const double2 *>(in.pv + 2 * vl);
          corner_laws(sn[l], in.pdmin[vl], pvl, pde, lame, il, P, sh[l], dsh[l], pc[l], dpc[l], khn[l], dkhn[l]);
          kwl[l] = dkwl[l] = 0.0;  // unused: the wetting mobility is evaluated per face
        }
      }
      // storage of the sub-control volume (vertex, cell): only dM/dS_n is non-zero
      mwS -= phie * rw * P.scv * dsh[cc];
      mnS += phie * rn * P.scv * dsh[cc];
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const int cj = cc ^ (1 << a);
        const int l0 = bit(cc, a) ? cj : cc;
        const int l1 = bit(cc, a) ? cc : cj;
        const double sgn = bit(cc, a) ? 1.0 : -1.0;  // F_l0 -= flux, F_l1 += flux
        // shape functions and x_a-derivatives at the SCVF barycentre
        double Nl[NC], Gl[NC];
#pragma unroll
        for (int l = 0; l < NC; ++l) {
          double n = 1.0, gg = (bit(l, a) ? 1.0 : -1.0) / P.h[a];
#pragma unroll
          for (int b = 0; b < DIM; ++b) {
            const double xi = (b == a) ? 0.5 : (bit(cc, b) ? 0.75 : 0.25);
            const double f = bit(l, b) ? xi : 1.0 - xi;
            n *= f;
            if (b != a) gg *= f;
          }
          Nl[l] = n;
          Gl[l] = gg;
        }
        double dp = 0.0, sip = 0.0, gpc = 0.0;
#pragma unroll
        for (int l = 0; l < NC; ++l) {
          dp += p[l] * Gl[l];
          sip += Nl[l] * sh[l];
          gpc += pc[l] * Gl[l];
        }
        const double area = P.area[a];
        const double ga = P.g[a];
        // wetting phase, upwinded plain saturation
        const double cw = -(Ke / P.mu_w) * area;
        const double phw = cw * (dp - rw * ga);
        const bool upw0 = phw >= 0.0;
        double kw, dkw;
        if constexpr (PAIRS) {
          kw = upw0 ? kwl[l0] : kwl[l1];
          dkw = upw0 ? dkwl[l0] : dkwl[l1];
        } else {
          krw(upw0 ? sn[l0] : sn[l1], il, P, kw, dkw);
        }
        const double fw = rw * kw * phw;
        // non-wetting phase, upwinded hat saturation
        const double cn = -(Ke / P.mu_n) * area;
        const double phn = cn * (dp - rn * ga);
        const bool upn0 = phn >= 0.0;
        const double kn = upn0 ? khn[l0] : khn[l1], dkn = upn0 ? dkhn[l0] : dkhn[l1];
        const double fn = rn * kn * phn;
        // capillary diffusion, central
        double kip, dkip;
        krn(sip, il, P, kip, dkip);
        const double cc_ = -rn * (Ke / P.mu_n) * area;
        const double fc = cc_ * kip * gpc;
        Fw += sgn * fw;
        Fn += sgn * (fn + fc);
        if (WANT_A) {
          // A_{i,l} -= sgn * d(flux)/du_l
#pragma unroll
          for (int l = 0; l < NC; ++l) {
            const int dx = bit(l, 0) - bit(cc, 0), dy = bit(l, 1) - bit(cc, 1);
            const int dz = (DIM == 3) ? bit(l, 2) - bit(cc, 2) : 0;
            const int o = stencil_index<DIM>(dx, dy, dz) - BASE;
            acc[o][0] -= sgn * (rw * kw * cw * Gl[l]);
            acc[o][2] -= sgn * (rn * kn * cn * Gl[l]);
            acc[o][3] -= sgn * (cc_ * (dkip * Nl[l] * dsh[l] * gpc + kip * Gl[l] * dpc[l]));
          }
          const double dfw = rw * phw * dkw;
          const double dfn = rn * phn * dkn;
          const int dx0 = bit(l0, 0) - bit(cc, 0), dy0 = bit(l0, 1) - bit(cc, 1);
          const int dz0 = (DIM == 3) ? bit(l0, 2) - bit(cc, 2) : 0;
          const int dx1 = bit(l1, 0) - bit(cc, 0), dy1 = bit(l1, 1) - bit(cc, 1);
          const int dz1 = (DIM == 3) ? bit(l1, 2) - bit(cc, 2) : 0;
          const int o0 = stencil_index<DIM>(dx0, dy0, dz0) - BASE;
          const int o1 = stencil_index<DIM>(dx1, dy1, dz1) - BASE;
          if (upw0) acc[o0][1] -= sgn * dfw; else acc[o1][1] -= sgn * dfw;
          if (upn0) acc[o0][3] -= sgn * dfn * dsh[l0]; else acc[o1][3] -= sgn * dfn * dsh[l1];
        }
      }
    }
  };
  [&]<int... CCs>(std::integer_sequence<int, CCs...>) {
    (cell(std::integral_constant<int, CCs>{}), ...);
  }(std::make_integer_sequence<int, NC>{});
}

// Completes and stores the row of vertex v for the stencil slots BASE..BASE+NSLOT-1
// (acc[k] = slot BASE + k): Dirichlet rows become unit rows (the unit entry on the
// centre slot), and the thread holding the centre (OWNER) adds the storage M/h,
// the Neumann source, and writes F and the storage part.
template <int DIM, bool WANT_A, bool W32, bool OWNER, int BASE, int NSLOT>
__host__ __device__ __forceinline__ void finish_vertex(const long long v, const Phys &P,
                                                      const uint8_t *__restrict__ dmask,
                                                      const double *__restrict__ Q, const double inv_h,
                                                      double (&acc)[NSLOT][4], double Fw, double Fn, double mwS,
                                                      double mnS, double *__restrict__ A64, float *__restrict__ A32,
                                                      double *__restrict__ F, double *__restrict__ mst) {
  constexpr int CEN = DIM == 3 ? 13 : 4;
  constexpr bool HAS_CEN = CEN >= BASE && CEN < BASE + NSLOT;
  const uint8_t m = dmask[v];
  if (OWNER) {
    const double2 q = *reinterpret_cast<const double2 *>(Q + 2 * v);
    Fw += q.x;
    Fn += q.y;
    if (m & 1) Fw = 0.0;
    if (m & 2) Fn = 0.0;
    if (F != nullptr) *reinterpret_cast<double2 *>(F + 2 * v) = make_double2(Fw, Fn);
  }
  if (!WANT_A) return;
  if constexpr (OWNER && HAS_CEN) {
    acc[CEN - BASE][1] += mwS * inv_h;
    acc[CEN - BASE][3] += mnS * inv_h;
    // storage part of the centre block (kept apart for the coarse-level lumping)
    *reinterpret_cast<double2 *>(mst + 2 * v) =
        make_double2((m & 1) ? 0.0 : mwS * inv_h, (m & 2) ? 0.0 : mnS * inv_h);
  }
  if (m & 1) {
#pragma unroll
    for (int o = 0; o < NSLOT; ++o) { acc[o][0] = 0.0; acc[o][1] = 0.0; }
    if constexpr (HAS_CEN) acc[CEN - BASE][0] = 1.0;
  }
  if (m & 2) {
#pragma unroll
    for (int o = 0; o < NSLOT; ++o) { acc[o][2] = 0.0; acc[o][3] = 0.0; }
    if constexpr (HAS_CEN) acc[CEN - BASE][3] = 1.0;
  }
#pragma unroll
  for (int k = 0; k < NSLOT; ++k) {
    const int o = BASE + k;
    double *dst = A64 + ((long long)o * P.N + v) * 4;
    reinterpret_cast<double2 *>(dst)[0] = make_double2(acc[k][0], acc[k][1]);
    reinterpret_cast<double2 *>(dst)[1] = make_double2(acc[k][2], acc[k][3]);
    if (W32) {
      float4 f4 = make_float4((float)acc[k][0], (float)acc[k][1], (float)acc[k][2], (float)acc[k][3]);
      *reinterpret_cast<float4 *>(A32 + tiled_block(o, v, DIM == 3 ? 27 : 9) * 4) = f4;
    }
  }
}

// Residual F(u) and (WANT_A) the stage matrix A = M(u)/h - dF/du for one vertex,
// all cells in one thread.
template <int DIM, bool WANT_A, bool W32, bool PAIRS = false>
__host__ __device__ __forceinline__ void assemble_vertex(const long long v, const Phys &P, const CellIn &in,
                                                        const uint8_t *__restrict__ dmask,
                                                        const double *__restrict__ Q, const double inv_h,
                                                        double *__restrict__ A64, float *__restrict__ A32,
                                                        double *__restrict__ F, double *__restrict__ mst) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  constexpr int NS = WANT_A ? NST : 1;
  double acc[NS][4];
#pragma unroll
  for (int o = 0; o < NS; ++o)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[o][e] = 0.0;
  double Fw = 0.0, Fn = 0.0, mwS = 0.0, mnS = 0.0;
  accumulate_cells<DIM, WANT_A, -1, 0, NS, PAIRS>(v, P, in, acc, Fw, Fn, mwS, mnS);
  finish_vertex<DIM, WANT_A, W32, true, 0, NS>(v, P, dmask, Q, inv_h, acc, Fw, Fn, mwS, mnS, A64, A32, F, mst);
}

template <int DIM, bool WANT_A, bool W32, bool PAIRS = false>
__global__ void __launch_bounds__(BS)
k_assemble(const Phys P, const CellIn in, const uint8_t *__restrict__ dmask, const double *__restrict__ Q,
           const double inv_h, double *__restrict__ A64, float *__restrict__ A32, double *__restrict__ F,
           double *__restrict__ mst) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= P.N) return;
  assemble_vertex<DIM, WANT_A, W32, PAIRS>(v, P, in, dmask, Q, inv_h, A64, A32, F, mst);
}

// The per-(cell, corner) laws of every cell, one thread per cell.  A vertex's row
// needs them at all corners of its 2^d cells, so evaluating them once per pair
// instead of once per (row, pair) removes most of the assembly's logarithms and
// exponentials (64 + 24 -> 8 + 8 per 3D vertex besides the 24 face mobilities).
template <int DIM>
__global__ void __launch_bounds__(BS) k_corners(const Phys P, const CellIn in, double *__restrict__ cp) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long long)P.ncx * P.ncy * P.ncz) return;
  corner_pass<DIM>(c, P, in, cp);
}

// 3D matrix assembly with two threads per vertex.  Thread half 1 takes the four
// cells below the vertex (stencil planes dz = -1, 0: slots 0..17), half 0 the four
// above (dz = 0, +1: slots 9..26).  Half 1 hands its dz = 0 plane and its partial
// sums to half 0 through LDS; half 0 owns the centre, the residual and the storage.
constexpr int SPLIT_V = BS / 2;  // vertices per block
template <bool W32, bool PAIRS>
__global__ void __launch_bounds__(BS)
k_assemble3_split(const Phys P, const CellIn in, const uint8_t *__restrict__ dmask, const double *__restrict__ Q,
                  const double inv_h, double *__restrict__ A64, float *__restrict__ A32, double *__restrict__ F,
                  double *__restrict__ mst) {
  __shared__ double xch[SPLIT_V][9 * 4 + 4];
  const int half = threadIdx.x / SPLIT_V;  // waves 0-1: half 0, waves 2-3: half 1
  const int lv = threadIdx.x % SPLIT_V;
  // XCD-aware order: consecutive vertex rows run on one XCD, whose L2 then holds the
  // per-(cell, corner) laws that neighbouring rows share
  const long long v = (long long)xcd_block(blockIdx.x, gridDim.x) * SPLIT_V + lv;
  const bool valid = v < P.N;
  double acc[18][4];
#pragma unroll
  for (int o = 0; o < 18; ++o)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[o][e] = 0.0;
  double Fw = 0.0, Fn = 0.0, mwS = 0.0, mnS = 0.0;
  if (valid) {
    if (half == 1)
      accumulate_cells<3, true, 1, 0, 18, PAIRS>(v, P, in, acc, Fw, Fn, mwS, mnS);
    else
      accumulate_cells<3, true, 0, 9, 18, PAIRS>(v, P, in, acc, Fw, Fn, mwS, mnS);
  }
  if (half == 1) {
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) xch[lv][4 * k + e] = acc[9 + k][e];
    xch[lv][36] = Fw;
    xch[lv][37] = Fn;
    xch[lv][38] = mwS;
    xch[lv][39] = mnS;
  }
  __syncthreads();
  if (!valid) return;
  if (half == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[k][e] += xch[lv][4 * k + e];
    Fw += xch[lv][36];
    Fn += xch[lv][37];
    mwS += xch[lv][38];
    mnS += xch[lv][39];
    finish_vertex<3, true, W32, true, 9, 18>(v, P, dmask, Q, inv_h, acc, Fw, Fn, mwS, mnS, A64, A32, F, mst);
  } else {
    double low[9][4];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) low[k][e] = acc[k][e];
    finish_vertex<3, true, W32, false, 0, 9>(v, P, dmask, Q, inv_h, low, 0.0, 0.0, 0.0, 0.0, A64, A32, nullptr,
                                             nullptr);
  }
}

// Storage of vertex v, m_i = sum over its sub-control volumes of Phi_e rho_a S^_a |SCV|
// with the saturation of the interface condition (Section 3.1, Eqs. dsW/dpN; the
// quantity whose derivative is M(u) in M(u) u' = F(u)).  in.pv must hold the vertex
// capillary pressures of in.u.
template <int DIM>
__host__ __device__ __forceinline__ void storage_vertex(const long long v, const Phys &P, const CellIn &in,
                                                       double &mw, double &mn) {
  constexpr int NC = 1 << DIM;
  int ix, iy, iz;
  grid_coords(v, P.nx, P.ny, ix, iy, iz);
  const double sn = in.u[2 * v + 1], pdm = in.pdmin[v];
  const double2 pvl = *reinterpret_cast<const double2 *>(in.pv + 2 * v);
  mw = 0.0;
  mn = 0.0;
#pragma unroll
  for (int cc = 0; cc < NC; ++cc) {
    const int ox = ix - bit(cc, 0), oy = iy - bit(cc, 1), oz = (DIM == 3) ? iz - bit(cc, 2) : 0;
    if (ox < 0 || oy < 0 || oz < 0 || ox >= P.ncx || oy >= P.ncy || oz >= P.ncz) continue;
    const long long c = ox + (long long)P.ncx * (oy + (long long)P.ncy * oz);
    double sh, dsh;
    hat_sat(sn, pdm, pvl, in.pdc[c], in.lamc[c], P, sh, dsh);
    const double w = in.phic[c] * P.scv;
    mw += w * P.rho_w * (1.0 - sh);
    mn += w * P.rho_n * sh;
  }
}

template <int DIM>
__global__ void __launch_bounds__(BS) k_storage(const Phys P, const CellIn in, double *__restrict__ m) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= P.N) return;
  double mw, mn;
  storage_vertex<DIM>(v, P, in, mw, mn);
  *reinterpret_cast<double2 *>(m + 2 * v) = make_double2(mw, mn);
}

// Newton right-hand side of the implicit Euler step m(u) - m(u_old) - tau F(u) = 0:
// r = F(u) - (m(u) - m_old) / tau in place of F (Dirichlet components 0), and the
// block partial sums of r.r (grid-stride over the vertices, fixed order).
template <int DIM>
__global__ void __launch_bounds__(BS) k_ie_rhs(const Phys P, const CellIn in, const uint8_t *__restrict__ dmask,
                                               const double *__restrict__ mold, const double inv_tau,
                                               double *__restrict__ r, double *__restrict__ part) {
  __shared__ double sm[BS / 64];
  double acc = 0.0;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < P.N; v += (long long)gridDim.x * blockDim.x) {
    double mw, mn;
    storage_vertex<DIM>(v, P, in, mw, mn);
    const double2 f = *reinterpret_cast<const double2 *>(r + 2 * v);
    const double2 mo = *reinterpret_cast<const double2 *>(mold + 2 * v);
    const uint8_t m = dmask[v];
    const double rw = (m & 1) ? 0.0 : f.x - (mw - mo.x) * inv_tau;
    const double rn = (m & 2) ? 0.0 : f.y - (mn - mo.y) * inv_tau;
    *reinterpret_cast<double2 *>(r + 2 * v) = make_double2(rw, rn);
    acc += rw * rw + rn * rn;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) t += sm[w];
    part[blockIdx.x] = t;
  }
}

__global__ void k_apply_dirichlet(long long N, const uint8_t *__restrict__ m,
                                  const double *__restrict__ val, double *__restrict__ u) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const uint8_t b = m[v];
  if (b & 1) u[2 * v] = val[2 * v];
  if (b & 2) u[2 * v + 1] = val[2 * v + 1];
}

inline CellIn cell_in(const tpf_grid *g, const double *u) {
  return CellIn{u, g->K, g->phi, g->pd, g->lam, g->pdmin, g->pv, nullptr};
}

}  // namespace

tpf_status setup_vertices(tpf_grid *g, const Patches &pt, hipStream_t s) {
  const unsigned nb = blocks_for(g->P.N);
  if (g->dim == 3)
    k_setup<3><<<nb, BS, 0, s>>>(g->P, g->pd, g->lam, pt, g->pdmin, g->lamref, g->Q);
  else
    k_setup<2><<<nb, BS, 0, s>>>(g->P, g->pd, g->lam, pt, g->pdmin, g->lamref, g->Q);
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

tpf_status launch_residual(tpf_grid *g, const double *u, double *f, hipStream_t s) {
  const unsigned nb = blocks_for(g->P.N);
  k_vertex_pc<<<nb, BS, 0, s>>>(g->P, u, g->pdmin, g->lamref, g->pv);
  TPF_LAUNCH_CHECK();
  CellIn in = cell_in(g, u);
  if (g->L > 1) {  // the per-(cell, corner) laws first, as in the assembly
    in.cp = g->rapb;
    const long long ncell = (long long)g->P.ncx * g->P.ncy * g->P.ncz;
    if (g->dim == 3)
      k_corners<3><<<blocks_for(ncell), BS, 0, s>>>(g->P, in, g->rapb);
    else
      k_corners<2><<<blocks_for(ncell), BS, 0, s>>>(g->P, in, g->rapb);
    TPF_LAUNCH_CHECK();
    if (g->dim == 3)
      k_assemble<3, false, false, true><<<nb, BS, 0, s>>>(g->P, in, g->dmask, g->Q, 0.0, nullptr, nullptr, f, nullptr);
    else
      k_assemble<2, false, false, true><<<nb, BS, 0, s>>>(g->P, in, g->dmask, g->Q, 0.0, nullptr, nullptr, f, nullptr);
  } else {
    if (g->dim == 3)
      k_assemble<3, false, false><<<nb, BS, 0, s>>>(g->P, in, g->dmask, g->Q, 0.0, nullptr, nullptr, f, nullptr);
    else
      k_assemble<2, false, false><<<nb, BS, 0, s>>>(g->P, in, g->dmask, g->Q, 0.0, nullptr, nullptr, f, nullptr);
  }
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

tpf_status launch_assemble(tpf_grid *g, const double *u0, double h, double *f0, hipStream_t s) {
  {  // (one level: the finest matrix is the one a pending coarsest factorisation reads)
    const tpf_status st = lu_join(g, s);
    if (st != TPF_OK) return st;
  }
  const unsigned nb = blocks_for(g->P.N);
  g->h_stage = h;
  k_vertex_pc<<<nb, BS, 0, s>>>(g->P, u0, g->pdmin, g->lamref, g->pv);
  TPF_LAUNCH_CHECK();
  double *A64 = g->lv[0].A64;
  float *A32 = g->prec != TPF_FP64 ? g->lv[0].A32 : nullptr;
  double *mst = g->lv[0].mst;
  const double ih = 1.0 / h;
  CellIn in = cell_in(g, u0);
  // The per-(cell, corner) laws go to the Galerkin-product scratch, which is idle
  // until the hierarchy is built and holds NST * 4 doubles per vertex, more than the
  // 2^d * CP per cell needed (grids of one level have none: the rows then evaluate
  // the laws themselves).
  const bool pairs = g->L > 1;
  const int ps = prof_begin(g, TPF_K_ASSEMBLE, s);
  if (pairs) {
    in.cp = g->rapb;
    const long long ncell = (long long)g->P.ncx * g->P.ncy * g->P.ncz;
    if (g->dim == 3)
      k_corners<3><<<blocks_for(ncell), BS, 0, s>>>(g->P, in, g->rapb);
    else
      k_corners<2><<<blocks_for(ncell), BS, 0, s>>>(g->P, in, g->rapb);
    TPF_LAUNCH_CHECK();
  }
  if (g->dim == 3) {
    const unsigned nb2 = blocks_for(g->P.N, SPLIT_V);
    if (A32 && pairs)
      k_assemble3_split<true, true><<<nb2, BS, 0, s>>>(g->P, in, g->dmask, g->Q, ih, A64, A32, f0, mst);
    else if (A32)
      k_assemble3_split<true, false><<<nb2, BS, 0, s>>>(g->P, in, g->dmask, g->Q, ih, A64, A32, f0, mst);
    else if (pairs)
      k_assemble3_split<false, true><<<nb2, BS, 0, s>>>(g->P, in, g->dmask, g->Q, ih, A64, nullptr, f0, mst);
    else
      k_assemble3_split<false, false><<<nb2, BS, 0, s>>>(g->P, in, g->dmask, g->Q, ih, A64, nullptr, f0, mst);
  } else {
    if (A32 && pairs)
      k_assemble<2, true, true, true><<<nb, BS, 0, s>>>(g->P, in, g->dmask, g->Q, ih, A64, A32, f0, mst);
    else if (A32)
      k_assemble<2, true, true, false><<<nb, BS, 0, s>>>(g->P, in, g->dmask, g->Q, ih, A64, A32, f0, mst);
    else if (pairs)
      k_assemble<2, true, false, true><<<nb, BS, 0, s>>>(g->P, in, g->dmask, g->Q, ih, A64, nullptr, f0, mst);
    else
      k_assemble<2, true, false, false><<<nb, BS, 0, s>>>(g->P, in, g->dmask, g->Q, ih, A64, nullptr, f0, mst);
  }
  TPF_LAUNCH_CHECK();
  prof_end(g, ps, s);
  return TPF_OK;
}

tpf_status launch_storage(tpf_grid *g, const double *u, double *m, hipStream_t s) {
  const unsigned nb = blocks_for(g->P.N);
  k_vertex_pc<<<nb, BS, 0, s>>>(g->P, u, g->pdmin, g->lamref, g->pv);
  TPF_LAUNCH_CHECK();
  const CellIn in = cell_in(g, u);
  if (g->dim == 3)
    k_storage<3><<<nb, BS, 0, s>>>(g->P, in, m);
  else
    k_storage<2><<<nb, BS, 0, s>>>(g->P, in, m);
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

tpf_status launch_ie_rhs(tpf_grid *g, const double *u, double *r, const double *mold, double inv_tau, double *part,
                         unsigned nblk, hipStream_t s) {
  k_vertex_pc<<<blocks_for(g->P.N), BS, 0, s>>>(g->P, u, g->pdmin, g->lamref, g->pv);
  TPF_LAUNCH_CHECK();
  const CellIn in = cell_in(g, u);
  if (g->dim == 3)
    k_ie_rhs<3><<<nblk, BS, 0, s>>>(g->P, in, g->dmask, mold, inv_tau, r, part);
  else
    k_ie_rhs<2><<<nblk, BS, 0, s>>>(g->P, in, g->dmask, mold, inv_tau, r, part);
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

tpf_status launch_apply_dirichlet(tpf_grid *g, double *u, hipStream_t s) {
  k_apply_dirichlet<<<blocks_for(g->P.N), BS, 0, s>>>(g->P.N, g->dmask, g->dval, u);
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

}  // namespace tpf
