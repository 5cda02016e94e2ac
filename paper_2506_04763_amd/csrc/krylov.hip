// Right-preconditioned BiCGSTAB (van der Vorst 1992) for the stage system, FP64.
//
// The scalars of the recurrence (rho, alpha, omega, beta) live in device memory and
// are produced by single-block finalisation kernels from per-block partial sums, so
// a whole iteration runs on the stream without host round trips; the host reads
// the residual norm once per iteration to decide convergence.  Every inner product
// is reduced in a fixed order (per-block tree, then one block over the partials):
// results are bitwise reproducible for a given grid size, independent of what else
// runs on the device.
#include "tpf_internal.h"

namespace tpf {

tpf_status spmv64_mode(tpf_grid *g, int mode, const double *x, double *y, const double *d0, double *part,
                       unsigned *nblk_out, hipStream_t s);

namespace {

template <int NDOT>
__device__ __forceinline__ void block_partials(double (&val)[NDOT], double *__restrict__ part, unsigned blk,
                                               unsigned nblk) {
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

__global__ void __launch_bounds__(BS) k_fill(double *__restrict__ p, long long n, double val) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = val;
}

__global__ void __launch_bounds__(BS) k_copy(double *__restrict__ d, const double *__restrict__ a, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    d[i] = a[i];
}

// r = f, rh = f, x = 0; partial (f, f)
__global__ void __launch_bounds__(BS) k_init(long long n, const double *__restrict__ f, double *__restrict__ r,
                                             double *__restrict__ rh, double *__restrict__ x,
                                             double *__restrict__ part) {
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double fi = f[i];
    r[i] = fi;
    rh[i] = fi;
    x[i] = 0.0;
    acc[0] += fi * fi;
  }
  block_partials<1>(acc, part, blockIdx.x, gridDim.x);
}

// p = r (first) or p = r + beta (p - omega v)
// (b32: the FP32 copy of the result for a mixed-precision V-cycle, or null)
__global__ void __launch_bounds__(BS) k_update_p(long long n, const double *__restrict__ r,
                                                 const double *__restrict__ v, double *__restrict__ p,
                                                 const double *__restrict__ sc, int first, float *__restrict__ b32) {
  const double beta = sc[S_BETA], omega = sc[S_OMEGA];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double pi = first ? r[i] : r[i] + beta * (p[i] - omega * v[i]);
    p[i] = pi;
    if (b32) b32[i] = (float)pi;
  }
}

// s = r - alpha v
__global__ void __launch_bounds__(BS) k_update_s(long long n, const double *__restrict__ r,
                                                 const double *__restrict__ v, double *__restrict__ s,
                                                 const double *__restrict__ sc, float *__restrict__ b32) {
  const double alpha = sc[S_ALPHA];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double si = r[i] - alpha * v[i];
    s[i] = si;
    if (b32) b32[i] = (float)si;
  }
}

// x += alpha ph + omega sh; r = s - omega t; partials (r, r), (rh, r)
__global__ void __launch_bounds__(BS) k_update_xr(long long n, double *__restrict__ x, const double *__restrict__ ph,
                                                  const double *__restrict__ sh, const double *__restrict__ s,
                                                  const double *__restrict__ t, double *__restrict__ r,
                                                  const double *__restrict__ rh, const double *__restrict__ sc,
                                                  double *__restrict__ part) {
  const double alpha = sc[S_ALPHA], omega = sc[S_OMEGA];
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    x[i] = x[i] + alpha * ph[i] + omega * sh[i];
    const double ri = s[i] - omega * t[i];
    r[i] = ri;
    acc[0] += ri * ri;
    acc[1] += rh[i] * ri;
  }
  block_partials<2>(acc, part, blockIdx.x, gridDim.x);
}

// restart: rh = r; partial (r, r)
__global__ void __launch_bounds__(BS) k_restart(long long n, const double *__restrict__ r, double *__restrict__ rh,
                                                double *__restrict__ part) {
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double ri = r[i];
    rh[i] = ri;
    acc[0] += ri * ri;
  }
  block_partials<1>(acc, part, blockIdx.x, gridDim.x);
}

enum Fin { F_INIT = 0, F_ALPHA, F_OMEGA, F_RHO, F_TRUE, F_RESTART };

// Reduces NDOT rows of partials (fixed order) and updates the recurrence scalars.
template <int NDOT>
__global__ void __launch_bounds__(1024) k_finalize(const double *__restrict__ part, unsigned nblk,
                                                   double *__restrict__ sc, int mode) {
  __shared__ double sm[NDOT][1024 / 64];
  double val[NDOT];
#pragma unroll
  for (int k = 0; k < NDOT; ++k) {
    double s = 0.0;
    for (unsigned b = threadIdx.x; b < nblk; b += 1024) s += part[(long long)k * nblk + b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sm[k][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int k = 0; k < NDOT; ++k) {
    double s = 0.0;
    for (int w = 0; w < 1024 / 64; ++w) s += sm[k][w];
    val[k] = s;
  }
  switch (mode) {
    case F_INIT:
      sc[S_FF] = val[0];
      sc[S_RHO] = val[0];
      sc[S_RR] = val[0];
      sc[S_RHO_OLD] = 1.0;
      sc[S_ALPHA] = 1.0;
      sc[S_OMEGA] = 1.0;
      sc[S_BETA] = 0.0;
      break;
    case F_ALPHA:
      sc[S_RV] = val[0];
      sc[S_ALPHA] = sc[S_RHO] / val[0];
      break;
    case F_OMEGA:
      sc[S_TS] = val[0];
      sc[S_TT] = NDOT > 1 ? val[NDOT > 1 ? 1 : 0] : 0.0;
      sc[S_OMEGA] = sc[S_TT] > 0.0 ? sc[S_TS] / sc[S_TT] : 0.0;
      break;
    case F_RHO: {
      const double rho_new = NDOT > 1 ? val[NDOT > 1 ? 1 : 0] : 0.0;
      sc[S_RR] = val[0];
      sc[S_RHO_OLD] = sc[S_RHO];
      sc[S_RHO] = rho_new;
      sc[S_BETA] = (rho_new / sc[S_RHO_OLD]) * (sc[S_ALPHA] / sc[S_OMEGA]);
      break;
    }
    case F_TRUE:
      sc[S_WW] = val[0];
      break;
    case F_RESTART:
      sc[S_RR] = val[0];
      sc[S_RHO] = val[0];
      break;
  }
}

}  // namespace

tpf_status fill_zero(double *p, long long n, hipStream_t s) {
  k_fill<<<RED_BLOCKS, BS, 0, s>>>(p, n, 0.0);
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

tpf_status copy_vec(double *dst, const double *src, long long n, hipStream_t s) {
  k_copy<<<RED_BLOCKS, BS, 0, s>>>(dst, src, n);
  TPF_LAUNCH_CHECK();
  return TPF_OK;
}

#define TPF_TRY(x)                   \
  do {                               \
    tpf_status st_ = (x);            \
    if (st_ != TPF_OK) return st_;   \
  } while (0)

static tpf_status read_scalars(tpf_grid *g, hipStream_t s) {
  TPF_HIP(hipMemcpyAsync(g->hscal, g->scal, NSCAL * sizeof(double), hipMemcpyDeviceToHost, s));
  TPF_HIP(hipStreamSynchronize(s));
  return TPF_OK;
}

tpf_status check_line_factors(tpf_grid *g, hipStream_t s) {
  if (g->smoother != TPF_SMOOTH_LINE) return TPF_OK;
  if (g->line_unchecked) {
    TPF_HIP(hipMemcpyAsync(&g->line_bad_count, g->line_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    TPF_HIP(hipStreamSynchronize(s));
    g->line_unchecked = false;
  }
  if (g->line_bad_count > 0) {
    set_error("line smoother: %d vertex lines met a singular pivot block in their block LU", g->line_bad_count);
    return TPF_EBREAKDOWN;
  }
  return TPF_OK;
}

tpf_status bicgstab(tpf_grid *g, const double *f, double *x, double rtol, int maxit, tpf_solve_stats *st,
                    hipStream_t s) {
  const long long n = 2 * g->P.N;
  double *part = g->part;
  unsigned nb = 0;
  // mixed precision: the p and s updates also write the FP32 right-hand side of the
  // V-cycle that follows them, which then needs no cast pass of its own
  float *b32 = g->prec != TPF_FP64 ? static_cast<float *>(g->lv[0].b) : nullptr;
  k_init<<<RED_BLOCKS, BS, 0, s>>>(n, f, g->r, g->rh, x, part);
  TPF_LAUNCH_CHECK();
  k_finalize<1><<<1, 1024, 0, s>>>(part, RED_BLOCKS, g->scal, F_INIT);
  TPF_LAUNCH_CHECK();
  TPF_TRY(read_scalars(g, s));
  const double ff = g->hscal[S_FF];
  tpf_solve_stats local{};
  local.fnorm = sqrt(ff);
  {
    const tpf_status lc = check_line_factors(g, s);
    if (lc != TPF_OK) {
      local.rel_res = local.rel_res_true = 1.0;
      if (st) *st = local;
      return lc;
    }
  }
  if (!(ff > 0.0)) {
    local.iters = 0;
    local.rel_res = 0.0;
    local.rel_res_true = 0.0;
    if (st) *st = local;
    if (ff != ff) { set_error("non-finite right-hand side"); return TPF_EBREAKDOWN; }
    return TPF_OK;
  }
  const double thr2 = rtol * rtol * ff;
  int first = 1, it = 0, restarts = 0;
  bool breakdown_restart_used = false;
  bool p_ready = false;  // this iteration's p update was enqueued during the last readback
  double rr = ff;
  bool true_fresh = false;  // S_WW holds the true residual of the final x
  tpf_status result = TPF_NOT_CONVERGED;
  while (it < maxit) {
    ++it;
    if (!p_ready) {
      k_update_p<<<RED_BLOCKS, BS, 0, s>>>(n, g->r, g->v, g->p, g->scal, first, b32);
      TPF_LAUNCH_CHECK();
    }
    p_ready = false;
    first = 0;
    TPF_TRY(vcycle(g, g->p, g->ph, s, b32 != nullptr));
    TPF_TRY(spmv64_mode(g, 1, g->ph, g->v, g->rh, part, &nb, s));
    k_finalize<1><<<1, 1024, 0, s>>>(part, nb, g->scal, F_ALPHA);
    TPF_LAUNCH_CHECK();
    k_update_s<<<RED_BLOCKS, BS, 0, s>>>(n, g->r, g->v, g->s, g->scal, b32);
    TPF_LAUNCH_CHECK();
    TPF_TRY(vcycle(g, g->s, g->sh, s, b32 != nullptr));
    TPF_TRY(spmv64_mode(g, 2, g->sh, g->t, g->s, part, &nb, s));
    k_finalize<2><<<1, 1024, 0, s>>>(part, nb, g->scal, F_OMEGA);
    TPF_LAUNCH_CHECK();
    k_update_xr<<<RED_BLOCKS, BS, 0, s>>>(n, x, g->ph, g->sh, g->s, g->t, g->r, g->rh, g->scal, part);
    TPF_LAUNCH_CHECK();
    k_finalize<2><<<1, 1024, 0, s>>>(part, RED_BLOCKS, g->scal, F_RHO);
    TPF_LAUNCH_CHECK();
    // Read the scalars back.  The next iteration's p update needs only the device-side
    // beta and omega, so it is enqueued behind the copy and runs while the host waits
    // for the copy alone; the restart paths below (first = 1) enqueue it again.
    TPF_HIP(hipMemcpyAsync(g->hscal, g->scal, NSCAL * sizeof(double), hipMemcpyDeviceToHost, s));
    TPF_HIP(hipEventRecord(g->scal_ev, s));
    if (it < maxit) {
      k_update_p<<<RED_BLOCKS, BS, 0, s>>>(n, g->r, g->v, g->p, g->scal, 0, b32);
      TPF_LAUNCH_CHECK();
      p_ready = true;
    }
    TPF_HIP(hipEventSynchronize(g->scal_ev));
    rr = g->hscal[S_RR];
    const double rho = g->hscal[S_RHO];
    if (!(rr == rr) || !(rho == rho)) {
      set_error("BiCGSTAB produced a non-finite residual at iteration %d", it);
      result = TPF_EBREAKDOWN;
      break;
    }
    if (rr <= thr2) {
      // confirm with the true residual f - A x (FP64)
      TPF_TRY(spmv64_mode(g, 3, x, g->w, f, part, &nb, s));
      k_finalize<1><<<1, 1024, 0, s>>>(part, nb, g->scal, F_TRUE);
      TPF_LAUNCH_CHECK();
      TPF_TRY(read_scalars(g, s));
      const double ww = g->hscal[S_WW];
      if (ww <= thr2 || restarts >= 2) {
        result = ww <= thr2 ? TPF_OK : TPF_NOT_CONVERGED;
        true_fresh = true;
        break;
      }
      // the recursive residual drifted: restart from the true residual
      TPF_TRY(copy_vec(g->r, g->w, n, s));
      k_restart<<<RED_BLOCKS, BS, 0, s>>>(n, g->r, g->rh, part);
      TPF_LAUNCH_CHECK();
      k_finalize<1><<<1, 1024, 0, s>>>(part, RED_BLOCKS, g->scal, F_RESTART);
      TPF_LAUNCH_CHECK();
      ++restarts;
      first = 1;
      p_ready = false;
      continue;
    }
    if (rho == 0.0) {
      if (breakdown_restart_used) {
        set_error("BiCGSTAB breakdown (rho = 0) after a restart, iteration %d", it);
        result = TPF_EBREAKDOWN;
        break;
      }
      k_restart<<<RED_BLOCKS, BS, 0, s>>>(n, g->r, g->rh, part);
      TPF_LAUNCH_CHECK();
      k_finalize<1><<<1, 1024, 0, s>>>(part, RED_BLOCKS, g->scal, F_RESTART);
      TPF_LAUNCH_CHECK();
      breakdown_restart_used = true;
      ++restarts;
      first = 1;
      p_ready = false;
    }
  }
  // final true residual, unless the convergence check has just computed it for this x
  if (!true_fresh) {
    TPF_TRY(spmv64_mode(g, 3, x, g->w, f, part, &nb, s));
    k_finalize<1><<<1, 1024, 0, s>>>(part, nb, g->scal, F_TRUE);
    TPF_LAUNCH_CHECK();
    TPF_TRY(read_scalars(g, s));
  }
  local.iters = it;
  local.restarts = restarts;
  local.rel_res = sqrt(rr / ff);
  local.rel_res_true = sqrt(g->hscal[S_WW] / ff);
  if (st) *st = local;
  return result;
}

}  // namespace tpf
