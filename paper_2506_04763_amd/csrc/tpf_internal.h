// Internal declarations of the gfx950 stage-solver library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "tpf.h"

namespace tpf {

constexpr int MAXL = 12;          // multigrid levels
constexpr int MAXK = 6;           // LIMEX stages
constexpr double SE_MIN = 1.0e-6; // lower clamp of the effective saturation
constexpr int BS = 256;           // threads per block of the vertex kernels
constexpr int RED_BLOCKS = 1024;  // fixed grid of the grid-stride reduction kernels
constexpr int NSCAL = 32;         // device scalars of the Krylov solver
constexpr long long TPF_LINE_PAIR_MAX_LINES = 32768;  // default of tpf_set_line_pairs

// Scalars of the Krylov recurrence kept on the device (indices into g->scal).
enum Scal {
  S_RHO = 0, S_RHO_OLD, S_ALPHA, S_OMEGA, S_BETA, S_RV, S_TS, S_TT, S_RR, S_FF, S_WW,
  S_NORM_A, S_NORM_B, S_NORM_C, S_NORM_D, S_IE_RR, S_PROJ_DP, S_PROJ_P, S_IE_DP, S_IE_DS, S_IE_PMAX, S_COUNT
};
static_assert(S_COUNT <= NSCAL, "device scalars exceed their array");

// Physical and geometric constants passed by value to every kernel.
struct Phys {
  int nx, ny, nz;
  long long N;        // vertices
  int ncx, ncy, ncz;  // cells per axis (ncz = 1 in 2D)
  double h[3];        // spacing (h[2] = 1 in 2D: unit depth)
  double g[3];        // gravity
  double rho_w, rho_n, mu_w, mu_n;
  double swr, snr, D; // D = (1 - S_wr) - S_nr
  double vol, scv;    // cell volume, sub-control-volume volume
  double area[3];     // SCVF area of an edge along each axis
  int kr_model, pad_; // TPF_KR_BURDINE or TPF_KR_POLY
  double kr_aw, kr_an;  // coefficients of TPF_KR_POLY
};

struct PatchDev {
  int axis, side, phase, pad;
  double lo[2], hi[2], rate;
};
struct Patches {
  int n;
  PatchDev p[TPF_MAX_PATCHES];
};

// Event timer of selected launch classes (host state only).
struct Prof {
  int active = 0, cap = 0, used = 0;
  unsigned mask = ~0u;       // classes timed
  hipEvent_t *ev = nullptr;  // 2 * cap
  int *cls = nullptr;        // cap
};

struct Level {
  int n[3];
  long long N;
  double *A64;  // [nst][N][4]
  float *A32;   // [nst][N][4] (mixed precision only; tiled on the finest level)
  uint16_t *A16;  // [nst][N][4] FP16 bits (coarse levels of TPF_MIXED16)
  float *s16;     // [N][2] row scales of A16
  double *mst;  // [N][2] storage part of the centre block, (w,S) and (n,S) entries
  void *x, *y, *b, *r;  // level vectors, 2N entries of the level type
  void *lf;     // TPF_SMOOTH_LINE: line-LU blocks G, V, W, [3][N][4] of the level type
};

}  // namespace tpf

struct tpf_grid {
  tpf::Phys P;
  int dim, nst, L, prec, nu_pre, nu_post, kmax, smoother;
  double omega;
  long long ncells;
  // scenario
  double *K, *phi, *pd, *lam;
  double *pdmin, *lamref, *pv;
  uint8_t *dmask;
  double *dval, *Q;
  tpf::Level lv[tpf::MAXL];
  // coarsest level, dense
  int nc;
  double *lu, *ainv;
  double *rapb;  // Galerkin-product scratch: NST * 4 * N (finest) doubles
  int *piv;
  // Krylov vectors (double[2N])
  double *r, *rh, *p, *v, *s, *t, *ph, *sh, *w, *xb;
  double *part;
  long long npart;
  double *scal;
  int *line_bad;        // TPF_SMOOTH_LINE: lines whose LU met a singular pivot block
  bool line_unchecked;  // line LU recomputed since line_bad was last read
  int line_bad_count;   // line_bad as last read
  long long line_pair_max;  // levels with fewer lines solve each line with two threads
  // LIMEX
  double *u0, *f0, *fv, *ua, *T[tpf::MAXK], *Tp;
  // host side
  double *hscal;  // pinned, NSCAL doubles
  hipEvent_t scal_ev;  // recorded after each per-iteration copy of the scalars to hscal
  bool assembled;
  bool has_f0;
  double h_stage;  // step of the assembled stage operator
  // V-cycle coarse tail as a captured graph (levels below the finest)
  int coarse_graph;           // use it (tpf_set_coarse_graph)
  hipStream_t cap_stream;     // capture stream (default priority)
  hipGraph_t vgraph;
  hipGraphExec_t vgraph_exec;
  void *vgraph_cur1;          // level-1 correction the tail leaves (fixed per grid)
  // the coarsest factorisation runs on the grid's own stream, forked from the caller's
  // stream after the Galerkin products; lu_pending until a stream has waited for it
  hipStream_t lu_stream = nullptr;  // default priority
  hipEvent_t lu_fork = nullptr, lu_done = nullptr;
  bool lu_pending = false;
  size_t bytes;
  int device;
  tpf::Prof prof;
};

namespace tpf {
// Records the start event of a timed launch of class `c`; returns the slot or -1.
inline int prof_begin(tpf_grid *g, int c, hipStream_t s) {
  Prof &p = g->prof;
  if (!p.active || p.used >= p.cap || !((p.mask >> c) & 1u)) return -1;
  const int i = p.used++;
  p.cls[i] = c;
  if (hipEventRecord(p.ev[2 * i], s) != hipSuccess) return -1;
  return i;
}
inline void prof_end(tpf_grid *g, int slot, hipStream_t s) {
  if (slot >= 0) (void)hipEventRecord(g->prof.ev[2 * slot + 1], s);
}
// Launches kern<<<grid, block, 0, s>>>(args...).  While launches of class c are timed,
// the class's event pair is attached to the dispatch itself (the extended launch), so
// the events hold the kernel's own start and end and the stream gets no marker packets
// between kernels; otherwise this is a plain launch.  Returns the launch status.
template <typename... P, typename... A>
inline hipError_t launch(tpf_grid *g, int c, void (*kern)(P...), unsigned grid, unsigned block, hipStream_t s,
                         A... args) {
  Prof &p = g->prof;
  if (p.active && p.used < p.cap && ((p.mask >> c) & 1u)) {
    const int i = p.used++;
    p.cls[i] = c;
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, p.ev[2 * i], p.ev[2 * i + 1], 0u, args...);
  } else {
    kern<<<grid, block, 0, s>>>(args...);
  }
  return hipGetLastError();
}
}  // namespace tpf

namespace tpf {

void set_error(const char *fmt, ...);

#define TPF_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::tpf::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),      \
                       __FILE__, __LINE__);                                        \
      return TPF_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

#define TPF_LAUNCH_CHECK() TPF_HIP(hipGetLastError())

// Orders stream s after the pending coarsest factorisation, if there is one: called
// before anything on s reads the coarse factors, or writes a matrix the factorisation
// reads.  Once one stream has waited, the work it queues after the wait is ordered
// after the factorisation (a grid is used from one stream at a time).
inline tpf_status lu_join(tpf_grid *g, hipStream_t s) {
  if (g->lu_pending) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TPF_HIP(hipStreamIsCapturing(s, &cs));
    if (cs == hipStreamCaptureStatusNone)
      TPF_HIP(hipStreamWaitEvent(s, g->lu_done, 0));
    else  // a stream being captured cannot wait for an event recorded outside the capture
      TPF_HIP(hipEventSynchronize(g->lu_done));
    g->lu_pending = false;
  }
  return TPF_OK;
}

inline unsigned blocks_for(long long n, int bs = BS) { return (unsigned)((n + bs - 1) / bs); }

// Grid coordinates of vertex v (x fastest).  Grids have fewer than 2^31 vertices
// (validated), so 32-bit unsigned division suffices, far cheaper on the GPU than the
// 64-bit one.
__host__ __device__ __forceinline__ void grid_coords(long long v, int nx, int ny, int &ix, int &iy, int &iz) {
  const unsigned u = (unsigned)v;
  const unsigned t = u / (unsigned)nx;
  ix = (int)(u - t * (unsigned)nx);
  iz = (int)(t / (unsigned)ny);
  iy = (int)(t - (unsigned)iz * (unsigned)ny);
}

// Block (o, v) of the finest level's FP32 matrix copy, which the smoother streams from
// HBM every sweep: vertices in tiles of 64 (one wavefront), the 64 blocks of one
// offset of a tile contiguous and a tile's offsets one after the other, so that the
// whole row set a wavefront needs is one contiguous range (27 KB in 3D).  Every other
// matrix is stored [offset][vertex] (block o * N + v).
__host__ __device__ __forceinline__ long long tiled_block(int o, long long v, int nst) {
  return (((v >> 6) * nst + o) << 6) + (v & 63);
}
__host__ __device__ __forceinline__ long long tiled_blocks(long long N, int nst) { return ((N + 63) >> 6) * 64 * nst; }

// Logical block index of an XCD-aware launch: the hardware dispatches block k to
// XCD k mod 8; this mapping gives every XCD one contiguous eighth of the grid so
// that neighbouring rows (which share x entries) meet in the same L2.
__host__ __device__ __forceinline__ unsigned xcd_block(unsigned bid, unsigned nblk) {
  const unsigned per = nblk >> 3;
  const unsigned full = per << 3;
  if (bid >= full) return bid;
  return (bid & 7u) * per + (bid >> 3);
}

// ---- launchers (assemble.hip) ----
tpf_status setup_vertices(tpf_grid *g, const Patches &pt, hipStream_t s);
tpf_status launch_residual(tpf_grid *g, const double *u, double *f, hipStream_t s);
tpf_status launch_assemble(tpf_grid *g, const double *u0, double h, double *f0, hipStream_t s);
tpf_status launch_apply_dirichlet(tpf_grid *g, double *u, hipStream_t s);
// m(u): the storage of both phases per vertex (double[2N], kg)
tpf_status launch_storage(tpf_grid *g, const double *u, double *m, hipStream_t s);
// r <- r - (m(u) - mold) / tau with Dirichlet components 0 (r holds F(u) on entry),
// and nblk block partial sums of r.r in part (grid-stride launch of nblk blocks)
tpf_status launch_ie_rhs(tpf_grid *g, const double *u, double *r, const double *mold, double inv_tau, double *part,
                         unsigned nblk, hipStream_t s);

// ---- launchers (mg.hip) ----
tpf_status build_hierarchy(tpf_grid *g, hipStream_t s);
// Moves the assembled stage operator and the whole hierarchy from the step h to
// h / ratio (M(u0) and J(u0) frozen): storage parts times ratio, copies refreshed,
// coarsest level refactored.
tpf_status rescale_stage(tpf_grid *g, double ratio, hipStream_t s);
// The finest FP32 matrix in the [offset][vertex] layout of the ABI (dst: nst*4*N floats).
tpf_status untile_matrix32(tpf_grid *g, float *dst, hipStream_t s);
// A coarse level's FP16 matrix as floats (entries times row scales), [offset][vertex][4].
tpf_status expand_matrix16(tpf_grid *g, int level, float *dst, hipStream_t s);
// staged: (mixed precision) the FP32 copy of b is already in the level-0 right-hand side
tpf_status vcycle(tpf_grid *g, const double *b, double *x, hipStream_t s, bool staged = false);
// y = A x (FP64, level l); if dot_with != null also block partials of (dot_with, y)
// and, if second != null, (second, y) and (y, y) as selected by mode.
tpf_status spmv64(tpf_grid *g, int level, const double *x, double *y, hipStream_t s);

// ---- krylov.hip ----
tpf_status bicgstab(tpf_grid *g, const double *f, double *x, double rtol, int maxit,
                    tpf_solve_stats *st, hipStream_t s);
// TPF_SMOOTH_LINE: TPF_EBREAKDOWN (with the error text) if the last line LU met a
// singular pivot block (synchronises s once per factorisation), else TPF_OK.
tpf_status check_line_factors(tpf_grid *g, hipStream_t s);

// ---- ie.hip ----
tpf_status ie_step(tpf_grid *g, double *u, double tau, const tpf_newton_opts *o, tpf_newton_stats *st,
                   hipStream_t s);
tpf_status project_pressure(tpf_grid *g, double *u, double h_p, const tpf_newton_opts *o, tpf_newton_stats *st,
                            hipStream_t s);

// ---- shared small kernels (krylov.hip) ----
tpf_status fill_zero(double *p, long long n, hipStream_t s);
tpf_status copy_vec(double *dst, const double *src, long long n, hipStream_t s);

}  // namespace tpf
