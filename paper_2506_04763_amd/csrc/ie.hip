// Fixed-step implicit Euler with Newton's method: the time-stepping scheme the paper
// compares LIMEX with (Section 5: the nonlinear iteration stops at an absolute defect
// of 1e-8 or a relative one of 1e-6).
//
// One step solves G(u) = m(u) - m(u_old) - tau F(u) = 0, the conservative backward Euler
// step of M(u) u' = F(u) (m the box-method storage, M = dm/du).  Its Jacobian
// M(u) - tau J(u) is tau times the LIMEX stage matrix A(u; h = tau), so each Newton
// iteration reuses the stage path: assemble A(u_k; tau) and F(u_k) in one kernel, build
// the multigrid hierarchy, form r = F(u_k) - (m(u_k) - m(u_old))/tau (Dirichlet rows 0)
// with its norm, and solve A delta = r with BiCGSTAB + GMG.  The defect is
// ||G(u_k)|| = tau ||r||; u_0 = u_old.  Globalisation: a trial u_k + lam delta whose
// defect is not below its base's is halved (at most max_halvings times in a row).
// Convergence: the defect meets atol or rtol times its first value, or the accepted
// update is negligible (xtol): near equilibrium the defect can sit on its FP64
// rounding floor above both.
#include <cmath>

#include "tpf_internal.h"

namespace tpf {
namespace {

// u = ua + lam * d
__global__ void __launch_bounds__(BS) k_lincomb(long long n, double *__restrict__ u, const double *__restrict__ ua,
                                                const double *__restrict__ d, double lam) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    u[i] = ua[i] + lam * d[i];
}

// out = sum of nblk partials, fixed order (one block)
__global__ void __launch_bounds__(1024) k_sum1(const double *__restrict__ part, unsigned nblk,
                                               double *__restrict__ out) {
  __shared__ double sm[16];
  double s = 0.0;
  for (unsigned b = threadIdx.x; b < nblk; b += 1024) s += part[b];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sm[w];
    *out = t;
  }
}

// p += dp on the pressure components only (S untouched); block maxima of |dp| and of
// the updated |p| (grid-stride)
__global__ void __launch_bounds__(BS) k_add_p(long long N, double *__restrict__ u, const double *__restrict__ d,
                                              double *__restrict__ part) {
  __shared__ double sm[2][BS / 64];
  double md = 0.0, mp = 0.0;
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    const double dp = d[2 * v];
    const double p = u[2 * v] + dp;
    u[2 * v] = p;
    md = fmax(md, fabs(dp));
    mp = fmax(mp, fabs(p));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    md = fmax(md, __shfl_down(md, off, 64));
    mp = fmax(mp, __shfl_down(mp, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    sm[0][threadIdx.x >> 6] = md;
    sm[1][threadIdx.x >> 6] = mp;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double m = 0.0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) m = fmax(m, sm[threadIdx.x][w]);
    part[(long long)threadIdx.x * gridDim.x + blockIdx.x] = m;
  }
}

// block maxima of |u - ua| on the pressure and the saturation components and of the
// updated |p| (grid-stride): the size of the accepted Newton update
__global__ void __launch_bounds__(BS) k_upd_max(long long N, const double *__restrict__ u,
                                                const double *__restrict__ ua, double *__restrict__ part) {
  __shared__ double sm[3][BS / 64];
  double m[3] = {0.0, 0.0, 0.0};
  for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += (long long)gridDim.x * blockDim.x) {
    m[0] = fmax(m[0], fabs(u[2 * v] - ua[2 * v]));
    m[1] = fmax(m[1], fabs(u[2 * v + 1] - ua[2 * v + 1]));
    m[2] = fmax(m[2], fabs(u[2 * v]));
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m[k] = fmax(m[k], __shfl_down(m[k], off, 64));
    if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = m[k];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) r = fmax(r, sm[threadIdx.x][w]);
    part[(long long)threadIdx.x * gridDim.x + blockIdx.x] = r;
  }
}

// out[0 .. K-1] = maxima of the K rows of nblk partials (one block)
template <int K>
__global__ void __launch_bounds__(1024) k_maxk(const double *__restrict__ part, unsigned nblk,
                                               double *__restrict__ out) {
  __shared__ double sm[K][16];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double m = 0.0;
    for (unsigned b = threadIdx.x; b < nblk; b += 1024) m = fmax(m, part[(long long)k * nblk + b]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = m;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double m = 0.0;
    for (int w = 0; w < 16; ++w) m = fmax(m, sm[threadIdx.x][w]);
    out[threadIdx.x] = m;
  }
}

#define TPF_TRY(x)                   \
  do {                               \
    tpf_status st_ = (x);            \
    if (st_ < 0) return st_;         \
  } while (0)

// r = F(u) - (m(u) - m_old)/tau in g->f0 (which holds F(u)); returns ||r||^2 on the host
tpf_status rhs_norm2(tpf_grid *g, const double *u, double inv_tau, double &rr, hipStream_t s) {
  TPF_TRY(launch_ie_rhs(g, u, g->f0, g->fv, inv_tau, g->part, RED_BLOCKS, s));
  k_sum1<<<1, 1024, 0, s>>>(g->part, RED_BLOCKS, g->scal + S_IE_RR);
  TPF_LAUNCH_CHECK();
  TPF_HIP(hipMemcpyAsync(g->hscal, g->scal, NSCAL * sizeof(double), hipMemcpyDeviceToHost, s));
  TPF_HIP(hipStreamSynchronize(s));
  rr = g->hscal[S_IE_RR];
  return TPF_OK;
}

}  // namespace

tpf_status ie_step(tpf_grid *g, double *u, double tau, const tpf_newton_opts *o, tpf_newton_stats *st,
                   hipStream_t s) {
  const long long n = 2 * g->P.N;
  const double inv_tau = 1.0 / tau;
  tpf_newton_stats ns{};
  TPF_TRY(copy_vec(g->u0, u, n, s));        // u_old: restored if the step fails
  TPF_TRY(launch_storage(g, u, g->fv, s));  // m(u_old)
  double d0 = 0.0, dprev = 0.0, lam = 1.0;
  int halv_row = 0;
  bool have_dir = false;  // a Newton direction in xb from the base point in ua
  bool ok = false;
  tpf_status hard = TPF_OK;
  for (;;) {
    // A(u; tau) and F(u) -> f0, the hierarchy, then r and its norm at u
    TPF_TRY(launch_assemble(g, u, tau, g->f0, s));
    TPF_TRY(build_hierarchy(g, s));
    g->assembled = true;
    g->has_f0 = false;
    if (have_dir) {  // size of the update from the base point (read back with the defect;
                     // three rows of partials, consumed before the defect reuses them)
      k_upd_max<<<RED_BLOCKS, BS, 0, s>>>(g->P.N, u, g->ua, g->part);
      TPF_LAUNCH_CHECK();
      k_maxk<3><<<1, 1024, 0, s>>>(g->part, RED_BLOCKS, g->scal + S_IE_DP);
      TPF_LAUNCH_CHECK();
    }
    double rr = 0.0;
    TPF_TRY(rhs_norm2(g, u, inv_tau, rr, s));
    const double d = tau * sqrt(rr);
    if (!std::isfinite(d)) {
      set_error("implicit Euler: non-finite defect at Newton iteration %d", ns.newton);
      hard = TPF_EBREAKDOWN;
      break;
    }
    if (!have_dir) {  // the initial defect G(u_old) = -tau F(u_old)
      d0 = d;
      ns.defect0 = d;
      ns.defect = d;
      if (d <= o->atol) {
        ok = true;
        ns.criterion = 1;
        break;
      }
    } else {
      if (!(d < dprev) && halv_row < o->max_halvings) {  // backtrack along the direction
        lam *= 0.5;
        ++halv_row;
        ++ns.halvings;
        k_lincomb<<<RED_BLOCKS, BS, 0, s>>>(n, u, g->ua, g->xb, lam);
        TPF_LAUNCH_CHECK();
        continue;
      }
      ++ns.newton;
      ns.defect = d;
      if (d <= o->atol || d <= o->rtol * d0) {
        ok = true;
        ns.criterion = 1;
        break;
      }
      const double up = g->hscal[S_IE_DP], us = g->hscal[S_IE_DS], pmax = g->hscal[S_IE_PMAX];
      if (o->xtol > 0.0 && up <= o->xtol * pmax && us <= o->xtol) {  // the update is at rounding level
        ok = true;
        ns.criterion = 2;
        break;
      }
      if (ns.newton >= o->max_newton) break;
    }
    // the Newton direction at u: A(u; tau) delta = r
    tpf_solve_stats ls{};
    const tpf_status rs = bicgstab(g, g->f0, g->xb, o->lin_rtol, o->maxit, &ls, s);
    ns.linear_iters += ls.iters;
    ++ns.linear_solves;
    if (rs < 0) {
      // breakdown on finite data fails the step; anything else is a hard error
      if (rs != TPF_EBREAKDOWN || !std::isfinite(ls.fnorm)) hard = rs;
      break;
    }
    TPF_TRY(copy_vec(g->ua, u, n, s));
    lam = 1.0;
    halv_row = 0;
    dprev = d;
    have_dir = true;
    k_lincomb<<<RED_BLOCKS, BS, 0, s>>>(n, u, g->ua, g->xb, 1.0);
    TPF_LAUNCH_CHECK();
  }
  ns.converged = ok ? 1 : 0;
  if (!ok) TPF_TRY(copy_vec(u, g->u0, n, s));  // a failed step leaves u unchanged
  TPF_HIP(hipStreamSynchronize(s));
  if (st) *st = ns;
  if (hard != TPF_OK) return hard;
  return ok ? TPF_OK : TPF_NOT_CONVERGED;
}

// Consistent pressure for the saturation of u: Newton at fixed S on the stage system
// with a vanishing step h_p (A(u; h_p) delta = F(u), p += delta_p).  With incompressible
// phases the pressure column carries no storage, so p is the algebraic unknown of
// M(u) u' = F(u); as h_p -> 0 the pressure update is the Newton step of the volume
// balance F_w/rho_w + F_n/rho_n = 0, in which the two storages cancel.
tpf_status project_pressure(tpf_grid *g, double *u, double h_p, const tpf_newton_opts *o, tpf_newton_stats *st,
                            hipStream_t s) {
  const long long n = 2 * g->P.N;
  tpf_newton_stats ns{};
  TPF_TRY(copy_vec(g->u0, u, n, s));  // restored if Newton fails
  bool ok = false;
  tpf_status hard = TPF_OK;
  while (ns.newton < o->max_newton) {
    TPF_TRY(launch_assemble(g, u, h_p, g->f0, s));
    TPF_TRY(build_hierarchy(g, s));
    g->assembled = true;
    g->has_f0 = true;
    tpf_solve_stats ls{};
    const tpf_status rs = bicgstab(g, g->f0, g->xb, o->lin_rtol, o->maxit, &ls, s);
    ns.linear_iters += ls.iters;
    ++ns.linear_solves;
    if (rs < 0) {
      if (rs != TPF_EBREAKDOWN || !std::isfinite(ls.fnorm)) hard = rs;
      break;
    }
    k_add_p<<<RED_BLOCKS, BS, 0, s>>>(g->P.N, u, g->xb, g->part);
    TPF_LAUNCH_CHECK();
    k_maxk<2><<<1, 1024, 0, s>>>(g->part, RED_BLOCKS, g->scal + S_PROJ_DP);
    TPF_LAUNCH_CHECK();
    TPF_HIP(hipMemcpyAsync(g->hscal, g->scal, NSCAL * sizeof(double), hipMemcpyDeviceToHost, s));
    TPF_HIP(hipStreamSynchronize(s));
    const double dp = g->hscal[S_PROJ_DP], pmax = g->hscal[S_PROJ_P];
    ++ns.newton;
    if (ns.newton == 1) ns.defect0 = dp;
    ns.defect = dp;
    if (!std::isfinite(dp)) {
      set_error("pressure projection: non-finite update at Newton iteration %d", ns.newton);
      hard = TPF_EBREAKDOWN;
      break;
    }
    if (dp <= fmax(o->atol, o->rtol * pmax)) {
      ok = true;
      break;
    }
  }
  ns.converged = ok ? 1 : 0;
  if (!ok) TPF_TRY(copy_vec(u, g->u0, n, s));
  TPF_HIP(hipStreamSynchronize(s));
  if (st) *st = ns;
  if (hard != TPF_OK) return hard;
  return ok ? TPF_OK : TPF_NOT_CONVERGED;
}

}  // namespace tpf
