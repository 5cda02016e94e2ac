// Device helpers shared by the stencil kernels (structured vertex grids, 2x2
// blocks stored [offset][vertex][4]).
#pragma once
#include "tpf_internal.h"

namespace tpf {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename T> struct Blk;
template <> struct Blk<double> {
  __device__ static __forceinline__ void load(const double *p, double (&b)[4]) {
    const double2 a = reinterpret_cast<const double2 *>(p)[0];
    const double2 c = reinterpret_cast<const double2 *>(p)[1];
    b[0] = a.x; b[1] = a.y; b[2] = c.x; b[3] = c.y;
  }
};
template <> struct Blk<float> {
  __device__ static __forceinline__ void load(const float *p, float (&b)[4]) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    b[0] = a.x; b[1] = a.y; b[2] = a.z; b[3] = a.w;
  }
};

struct Geo {
  int nx, ny, nz;
  long long N;
};

__host__ __device__ __forceinline__ void vcoords(long long v, const Geo &G, int &ix, int &iy, int &iz) {
  grid_coords(v, G.nx, G.ny, ix, iy, iz);
}

__host__ __device__ inline Geo geo_of(const int n[3], long long N) { return Geo{n[0], n[1], n[2], N}; }


// B: scratch of NST * 4 * Nf doubles.  mask: the fine level is the finest (Dirichlet
// mask fmask applies, rows in volume-balance form with vr = rho_w / rho_n).
tpf_status launch_rap(int dim, bool mask, const int nf[3], long long Nf, const int nc[3], long long Nc,
                      const double *Af, const uint8_t *fmask, const double *mf, double vr, double *B, double *Ac,
                      float *Ac32, double *mc, hipStream_t s);

}  // namespace tpf
