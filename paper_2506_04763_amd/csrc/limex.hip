// Adaptive LIMEX step (Section 4): linearly implicit Euler substeps with the matrix
// frozen at the step's initial state, Aitken-Neville extrapolation over the
// harmonic stage sequence n_j = j, relative error in the scaled norm of Eq. norm_u
// and the step-size rule with order q = 2.
//
// Error norm: |||u|||^2 = alpha ||grad p_w||^2 + beta ||S_w||^2 with
// alpha = 1/(2 ||grad p_w(T_kk)||^2) and beta = 1/(2 ||S_w(T_kk)||^2), so that
// eps^2 = (e_p^2 + e_S^2)/2 balances pressure and saturation errors.  The pressure is
// the one whose gradient drives the convective parts of both balances (the argument of
// Eqs. norm_uw/norm_un): p_n in the paper's (p_n, S_w) unknowns, p_w in the (p_w, S_n)
// unknowns here.  ||grad p||^2 is the exact integral of the Q1 interpolant
// (closed-form element stiffness of a box), ||S_w||^2 the lumped (dual-box) L2 norm.
#include <cmath>

#include "tpf_internal.h"

namespace tpf {

tpf_status bicgstab(tpf_grid *g, const double *f, double *x, double rtol, int maxit, tpf_solve_stats *st,
                    hipStream_t s);

namespace {

__global__ void __launch_bounds__(BS) k_axpy(long long n, double *__restrict__ y, const double *__restrict__ x) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] += x[i];
}

// T_j <- T_j + (T_j - T_jm) * c
__global__ void __launch_bounds__(BS) k_extrap(long long n, double *__restrict__ Tj, const double *__restrict__ Tjm,
                                               double c) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double a = Tj[i];
    Tj[i] = a + (a - Tjm[i]) * c;
  }
}

// Partial sums of ||grad (a_p - b_p)||^2, ||grad a_p||^2, ||b_Sw - a_Sw||^2, ||a_Sw||^2
// (a = T_kk, b = T_{k,k-1}); each vertex owns the cell whose origin it is.
template <int DIM>
__global__ void __launch_bounds__(BS) k_norms(const Phys P, const double *__restrict__ a,
                                              const double *__restrict__ b, double *__restrict__ part) {
  constexpr int NC = 1 << DIM;
  __shared__ double sm[4][BS / 64];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const long long sy = P.nx, sz = (long long)P.nx * P.ny;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < P.N; v += (long long)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    grid_coords(v, P.nx, P.ny, ix, iy, iz);
    // lumped saturation norm: dual-box volume times S_w^2
    double dual = P.h[0] * P.h[1] * (DIM == 3 ? P.h[2] : 1.0);
    if (ix == 0 || ix == P.nx - 1) dual *= 0.5;
    if (iy == 0 || iy == P.ny - 1) dual *= 0.5;
    if (DIM == 3 && (iz == 0 || iz == P.nz - 1)) dual *= 0.5;
    const double swa = 1.0 - a[2 * v + 1];
    const double dsw = -(a[2 * v + 1] - b[2 * v + 1]);
    acc[2] += dual * dsw * dsw;
    acc[3] += dual * swa * swa;
    if (ix < P.nx - 1 && iy < P.ny - 1 && (DIM == 2 || iz < P.nz - 1)) {
      double pa[NC], pd[NC];
#pragma unroll
      for (int l = 0; l < NC; ++l) {
        const long long vl = v + (l & 1) + sy * ((l >> 1) & 1) + (DIM == 3 ? sz * ((l >> 2) & 1) : 0);
        pa[l] = a[2 * vl];
        pd[l] = a[2 * vl] - b[2 * vl];
      }
#pragma unroll
      for (int ax = 0; ax < DIM; ++ax) {
        // edge differences along ax at the 2^(d-1) transverse corners
        constexpr int NE = NC / 2;
        double ea[NE], ed[NE];
        int k = 0;
#pragma unroll
        for (int l = 0; l < NC; ++l) {
          if ((l >> ax) & 1) continue;
          const int l1 = l | (1 << ax);
          ea[k] = pa[l1] - pa[l];
          ed[k] = pd[l1] - pd[l];
          ++k;
        }
        const double w = P.vol / (P.h[ax] * P.h[ax]);
        // transverse Q1 mass matrix on the unit (d-1)-cube: product of 1/3 (same
        // coordinate bit) and 1/6 (different bit) per transverse axis
        double qa = 0.0, qd = 0.0;
#pragma unroll
        for (int i = 0; i < NE; ++i)
#pragma unroll
          for (int j = 0; j < NE; ++j) {
            double m = 1.0;
#pragma unroll
            for (int tb = 0; tb < DIM - 1; ++tb) m *= (((i ^ j) >> tb) & 1) ? (1.0 / 6.0) : (1.0 / 3.0);
            qa += ea[i] * m * ea[j];
            qd += ed[i] * m * ed[j];
          }
        acc[0] += w * qd;
        acc[1] += w * qa;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double s = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) s += sm[threadIdx.x][w];
    part[(long long)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(1024) k_sum4(const double *__restrict__ part, unsigned nblk, double *__restrict__ out) {
  __shared__ double sm[4][16];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double s = 0.0;
    for (unsigned b = threadIdx.x; b < nblk; b += 1024) s += part[(long long)k * nblk + b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += sm[threadIdx.x][w];
    out[threadIdx.x] = s;
  }
}

}  // namespace

tpf_status launch_assemble(tpf_grid *g, const double *u0, double h, double *f0, hipStream_t s);
tpf_status launch_residual(tpf_grid *g, const double *u, double *f, hipStream_t s);
tpf_status build_hierarchy(tpf_grid *g, hipStream_t s);
tpf_status copy_vec(double *dst, const double *src, long long n, hipStream_t s);
tpf_status rescale_stage(tpf_grid *g, double ratio, hipStream_t s);

#define TPF_TRY(x)                   \
  do {                               \
    tpf_status st_ = (x);            \
    if (st_ < 0) return st_;         \
  } while (0)

tpf_status limex_step(tpf_grid *g, double *u, double *t, double *dt, const tpf_limex_opts *o,
                      tpf_limex_stats *stats, hipStream_t s) {
  const long long n = 2 * g->P.N;
  const int k = o->stages;
  const double H = *dt;
  tpf_limex_stats ls{};
  ls.dt_used = H;
  TPF_TRY(copy_vec(g->u0, u, n, s));
  bool failed = false;  // a stage solve missed rtol within maxit or broke down
  for (int j = 1; j <= k && !failed; ++j) {
    if (j == 1) {  // A(H) = M(u0)/H - J(u0), F(u0) and the hierarchy
      TPF_TRY(launch_assemble(g, g->u0, H, g->f0, s));
      TPF_TRY(build_hierarchy(g, s));
    } else {  // M and J stay frozen at u0: only the storage parts follow the step H/j
      const double h = H / j;
      TPF_TRY(rescale_stage(g, g->h_stage / h, s));
      g->h_stage = h;
    }
    g->assembled = true;
    g->has_f0 = true;
    double *Tj = g->T[j - 1];
    TPF_TRY(copy_vec(Tj, g->u0, n, s));
    for (int m = 0; m < j && !failed; ++m) {
      const double *rhs = g->f0;
      if (m > 0) {
        TPF_TRY(launch_residual(g, Tj, g->fv, s));
        rhs = g->fv;
      }
      tpf_solve_stats st{};
      const tpf_status rs = bicgstab(g, rhs, g->xb, o->rtol, o->maxit, &st, s);
      ls.solves++;
      ls.iters_total += st.iters;
      // a non-finite right-hand side is bad input, and device errors are hard errors;
      // a solve that fails on finite data asks for a shorter step
      if (rs < 0 && (rs != TPF_EBREAKDOWN || !std::isfinite(st.fnorm))) return rs;
      if (rs != TPF_OK) {
        ls.unconverged++;
        failed = true;
        break;
      }
      k_axpy<<<RED_BLOCKS, BS, 0, s>>>(n, Tj, g->xb);
      TPF_LAUNCH_CHECK();
    }
  }
  if (failed) {  // reject: u and t unchanged, a quarter of the step next
    ls.eps = INFINITY;
    ls.accepted = 0;
    ls.dt_next = fmin(o->dt_max, 0.25 * H);
    *dt = ls.dt_next;
    if (stats) *stats = ls;
    TPF_HIP(hipStreamSynchronize(s));
    return TPF_STEP_REJECTED;
  }
  // Aitken-Neville tableau in place: pass l builds column l+1 for rows k..l+1
  for (int l = 1; l <= k - 1; ++l) {
    if (l == k - 1) TPF_TRY(copy_vec(g->Tp, g->T[k - 1], n, s));
    for (int j = k; j >= l + 1; --j) {
      const double ratio = (double)j / (double)(j - l);
      k_extrap<<<RED_BLOCKS, BS, 0, s>>>(n, g->T[j - 1], g->T[j - 2], 1.0 / (ratio - 1.0));
      TPF_LAUNCH_CHECK();
    }
  }
  double eps = 0.0;
  if (k > 1) {
    if (g->dim == 3)
      k_norms<3><<<RED_BLOCKS, BS, 0, s>>>(g->P, g->T[k - 1], g->Tp, g->part);
    else
      k_norms<2><<<RED_BLOCKS, BS, 0, s>>>(g->P, g->T[k - 1], g->Tp, g->part);
    TPF_LAUNCH_CHECK();
    k_sum4<<<1, 1024, 0, s>>>(g->part, RED_BLOCKS, g->scal + S_NORM_A);
    TPF_LAUNCH_CHECK();
    TPF_HIP(hipMemcpyAsync(g->hscal, g->scal, NSCAL * sizeof(double), hipMemcpyDeviceToHost, s));
    TPF_HIP(hipStreamSynchronize(s));
    const double gd = g->hscal[S_NORM_A], ga = fmax(g->hscal[S_NORM_B], 1e-300);
    const double sd = g->hscal[S_NORM_C], sa = fmax(g->hscal[S_NORM_D], 1e-300);
    eps = sqrt(0.5 * (gd / ga + sd / sa));
  }
  ls.eps = eps;
  const bool acc = eps <= o->tol;
  ls.accepted = acc ? 1 : 0;
  double nxt = H * cbrt(o->safety * o->tol / fmax(eps, 1e-300));
  if (k == 1) nxt = H;
  ls.dt_next = fmin(o->dt_max, nxt);
  if (acc) {
    TPF_TRY(copy_vec(u, g->T[k - 1], n, s));
    *t += H;
  }
  *dt = ls.dt_next;
  if (stats) *stats = ls;
  TPF_HIP(hipStreamSynchronize(s));
  return acc ? TPF_OK : TPF_STEP_REJECTED;
}

}  // namespace tpf
