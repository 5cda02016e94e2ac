// C ABI of the stage-solver library: descriptor validation, arena layout, grid
// creation and the thin entry points over the device paths.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <new>

#include "tpf_internal.h"

namespace tpf {

static thread_local char g_err[1024] = {0};

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

tpf_status limex_step(tpf_grid *g, double *u, double *t, double *dt, const tpf_limex_opts *o,
                      tpf_limex_stats *stats, hipStream_t s);

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

bool finite(double x) { return std::isfinite(x); }

struct Layout {
  long long N, ncells;
  int L, nst, nc;
  int n[MAXL][3];
  long long Nl[MAXL];
  size_t off_cells, off_vert, off_lv[MAXL], off_coarse, off_rapb, off_kry, off_part, off_scal, off_flags, off_lx,
      total;
  long long npart;
};

#define BAD(...)              \
  do {                        \
    set_error(__VA_ARGS__);   \
    return TPF_EINVAL;        \
  } while (0)

tpf_status validate(const tpf_grid_desc *d) {
  if (!d) BAD("descriptor is NULL");
  if (d->dim != 2 && d->dim != 3) BAD("dim must be 2 or 3 (got %d)", d->dim);
  for (int a = 0; a < d->dim; ++a) {
    if (d->n[a] < 2) BAD("n[%d] = %d: need at least 2 vertices per axis", a, d->n[a]);
    if (!(d->extent[a] > 0.0) || !finite(d->extent[a])) BAD("extent[%d] must be positive and finite", a);
  }
  if (d->dim == 2 && d->n[2] != 1) BAD("2D grids need n[2] = 1");
  const double nv = (double)d->n[0] * d->n[1] * d->n[2];
  if (nv > 2147483647.0) BAD("grid too large (at most 2^31 - 1 vertices)");
  for (int a = 0; a < 3; ++a)
    if (!finite(d->gravity[a])) BAD("gravity must be finite");
  for (int k = 0; k < 2; ++k) {
    if (!(d->rho[k] > 0.0) || !finite(d->rho[k])) BAD("rho[%d] must be positive", k);
    if (!(d->mu[k] > 0.0) || !finite(d->mu[k])) BAD("mu[%d] must be positive", k);
    if (!(d->s_res[k] >= 0.0) || !finite(d->s_res[k])) BAD("s_res[%d] must be >= 0", k);
  }
  if (!(d->s_res[0] + d->s_res[1] < 1.0)) BAD("S_wr + S_nr must be < 1");
  if (!d->perm || !d->poro || !d->entry_p || !d->bc_lambda) BAD("cell arrays must not be NULL");
  if (!d->dir_mask) BAD("dir_mask must not be NULL");
  const long long nc = (long long)(d->n[0] - 1) * (d->n[1] - 1) * (d->dim == 3 ? d->n[2] - 1 : 1);
  for (long long c = 0; c < nc; ++c) {
    if (!(d->perm[c] > 0.0) || !finite(d->perm[c])) BAD("perm[%lld] must be positive and finite", c);
    if (!(d->poro[c] > 0.0 && d->poro[c] <= 1.0)) BAD("poro[%lld] must be in (0, 1]", c);
    if (!(d->entry_p[c] >= 0.0) || !finite(d->entry_p[c])) BAD("entry_p[%lld] must be >= 0 and finite", c);
    if (!(d->bc_lambda[c] > 0.0) || !finite(d->bc_lambda[c])) BAD("bc_lambda[%lld] must be positive", c);
  }
  const long long N = (long long)nv;
  for (long long v = 0; v < N; ++v) {
    const uint8_t m = d->dir_mask[v];
    if (m & ~3u) BAD("dir_mask[%lld] has bits other than 0 and 1", v);
    if (m) {
      if (!d->dir_value) BAD("dir_value is NULL but dir_mask has set bits");
      if (((m & 1) && !finite(d->dir_value[2 * v])) || ((m & 2) && !finite(d->dir_value[2 * v + 1])))
        BAD("dir_value[%lld] is not finite", v);
    }
  }
  if (d->n_patches < 0 || d->n_patches > TPF_MAX_PATCHES) BAD("n_patches must be in [0, %d]", TPF_MAX_PATCHES);
  if (d->n_patches > 0 && !d->patches) BAD("patches is NULL");
  for (int k = 0; k < d->n_patches; ++k) {
    const tpf_patch &p = d->patches[k];
    if (p.axis < 0 || p.axis >= d->dim) BAD("patch %d: axis out of range", k);
    if (p.side != 0 && p.side != 1) BAD("patch %d: side must be 0 or 1", k);
    if (p.phase != 0 && p.phase != 1) BAD("patch %d: phase must be 0 or 1", k);
    if (!finite(p.rate)) BAD("patch %d: rate not finite", k);
    for (int j = 0; j < d->dim - 1; ++j)
      if (!(p.lo[j] <= p.hi[j]) || !finite(p.lo[j]) || !finite(p.hi[j])) BAD("patch %d: need lo <= hi", k);
  }
  if (d->levels < 1 || d->levels > MAXL) BAD("levels must be in [1, %d]", MAXL);
  int n[3] = {d->n[0], d->n[1], d->n[2]};
  for (int l = 1; l < d->levels; ++l)
    for (int a = 0; a < d->dim; ++a) {
      if ((n[a] - 1) % 2 != 0 || (n[a] - 1) / 2 + 1 < 2)
        BAD("n[%d] = %d cannot be coarsened %d times (need (n-1) divisible by 2^(levels-1))", a, d->n[a],
            d->levels - 1);
      n[a] = (n[a] - 1) / 2 + 1;
    }
  const long long ncoarse = 2LL * n[0] * n[1] * n[2];
  if (ncoarse > 4096) BAD("coarsest level has %lld unknowns (max 4096): use more levels", ncoarse);
  if (d->precision != TPF_FP64 && d->precision != TPF_MIXED && d->precision != TPF_MIXED16)
    BAD("precision must be TPF_FP64, TPF_MIXED or TPF_MIXED16");
  if (d->nu_pre < 1 || d->nu_post < 0 || d->nu_pre > 16 || d->nu_post > 16) BAD("need 1 <= nu_pre <= 16, 0 <= nu_post <= 16");
  if (!(d->omega > 0.0 && d->omega < 2.0)) BAD("omega must be in (0, 2)");
  if (d->limex_stages < 0 || d->limex_stages > MAXK) BAD("limex_stages must be in [0, %d]", MAXK);
  if (d->kr_model != TPF_KR_BURDINE && d->kr_model != TPF_KR_POLY) BAD("kr_model must be TPF_KR_BURDINE or TPF_KR_POLY");
  if (d->smoother != TPF_SMOOTH_POINT && d->smoother != TPF_SMOOTH_LINE)
    BAD("smoother must be TPF_SMOOTH_POINT or TPF_SMOOTH_LINE");
  if (d->kr_model == TPF_KR_POLY)
    for (int k = 0; k < 2; ++k)
      if (!(d->kr_coef[k] > 0.0) || !finite(d->kr_coef[k])) BAD("kr_coef[%d] must be positive and finite", k);
  if (d->vertex_source)
    for (long long v = 0; v < 2 * N; ++v)
      if (!finite(d->vertex_source[v])) BAD("vertex_source[%lld] is not finite", v);
  return TPF_OK;
}

void layout(const tpf_grid_desc *d, Layout &L) {
  L.nst = d->dim == 3 ? 27 : 9;
  L.L = d->levels;
  L.N = (long long)d->n[0] * d->n[1] * d->n[2];
  L.ncells = (long long)(d->n[0] - 1) * (d->n[1] - 1) * (d->dim == 3 ? d->n[2] - 1 : 1);
  for (int a = 0; a < 3; ++a) L.n[0][a] = d->n[a];
  L.Nl[0] = L.N;
  for (int l = 1; l < L.L; ++l) {
    for (int a = 0; a < 3; ++a) L.n[l][a] = (a < d->dim) ? (L.n[l - 1][a] - 1) / 2 + 1 : 1;
    L.Nl[l] = (long long)L.n[l][0] * L.n[l][1] * L.n[l][2];
  }
  L.nc = (int)(2 * L.Nl[L.L - 1]);
  const size_t vsz = d->precision != TPF_FP64 ? sizeof(float) : sizeof(double);
  size_t o = 0;
  L.off_cells = o;
  o += align_up(4 * L.ncells * sizeof(double));
  L.off_vert = o;
  o += align_up(L.N * sizeof(double)) * 2;       // pdmin, lamref
  o += align_up(2 * L.N * sizeof(double)) * 3;   // pv, dval, Q
  o += align_up(L.N);                            // dmask
  for (int l = 0; l < L.L; ++l) {
    L.off_lv[l] = o;
    o += align_up((size_t)L.nst * 4 * L.Nl[l] * sizeof(double));
    if (d->precision == TPF_MIXED || (d->precision == TPF_MIXED16 && l == 0))  // finest FP32 copy tiled
      o += align_up((size_t)(l == 0 ? tiled_blocks(L.Nl[0], L.nst) : L.nst * L.Nl[l]) * 4 * sizeof(float));
    if (d->precision == TPF_MIXED16 && l > 0)  // FP16 blocks + two FP32 row scales per vertex
      o += align_up((size_t)L.nst * 4 * L.Nl[l] * sizeof(uint16_t)) + align_up(2 * L.Nl[l] * sizeof(float));
    o += align_up(2 * L.Nl[l] * sizeof(double));
    o += 4 * align_up(2 * L.Nl[l] * vsz);
    if (d->smoother == TPF_SMOOTH_LINE && l + 1 < L.L) o += align_up(12 * L.Nl[l] * vsz);  // line LU
  }
  L.off_coarse = o;
  o += 2 * align_up((size_t)L.nc * L.nc * sizeof(double)) + align_up(L.nc * sizeof(int));
  L.off_rapb = o;  // A P of the Galerkin product, one level at a time (finest fine grid largest)
  o += L.L > 1 ? align_up((size_t)L.nst * 4 * L.N * sizeof(double)) : 0;
  L.off_kry = o;
  o += 10 * align_up(2 * L.N * sizeof(double));
  L.npart = std::max<long long>(RED_BLOCKS, (L.N + BS - 1) / BS);
  L.off_part = o;
  o += align_up(4 * L.npart * sizeof(double));
  L.off_scal = o;
  o += align_up(NSCAL * sizeof(double));
  L.off_flags = o;  // device flags (line LU)
  o += align_up(sizeof(int));
  L.off_lx = o;
  o += align_up(2 * L.N * sizeof(double)) * (4 + (d->limex_stages > 0 ? 1 + d->limex_stages : 0));
  L.total = o;
}

}  // namespace
}  // namespace tpf

namespace tpf {

// ---- the solve without caller-provided Krylov workspace -----------------------
// Workspace of tpf_solve_stage_static: the BiCGSTAB vectors, block partials and device
// scalars of one solve, in a device array of fixed size (each GPU the library runs on
// holds its own copy until the process ends).  Host code never uses the array's name
// as an address: it takes the device address once per device from the runtime.
constexpr size_t STATIC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {nullptr};

// The device address of this device's scratch array (looked up on first use, with the
// device current).
tpf_status scratch_for_current_device(void **out) {
  int dev = -1;
  TPF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("device %d out of range", dev);
    return TPF_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      return TPF_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TPF_OK;
}

// Bytes of the static workspace a solve on g needs: nine Krylov vectors (the tenth of
// the arena's set, the LIMEX update, is not used by a solve), the block partials and
// the device scalars.
size_t static_solve_bytes(const tpf_grid *g) {
  return 9 * align_up(2 * (size_t)g->P.N * sizeof(double)) + align_up(4 * (size_t)g->npart * sizeof(double)) +
         align_up(NSCAL * sizeof(double));
}
}  // namespace

}  // namespace tpf

using namespace tpf;

extern "C" {

const char *tpf_last_error(void) { return g_err; }

tpf_status tpf_validate(const tpf_grid_desc *desc) {
  g_err[0] = 0;
  return validate(desc);
}

size_t tpf_grid_bytes(const tpf_grid_desc *desc) {
  g_err[0] = 0;
  if (validate(desc) != TPF_OK) return 0;
  Layout L;
  layout(desc, L);
  return L.total;
}

tpf_status tpf_create_grid(const tpf_grid_desc *d, void *arena, size_t arena_bytes, tpf_stream stream,
                           tpf_grid **out) {
  g_err[0] = 0;
  if (!out) { set_error("out is NULL"); return TPF_EINVAL; }
  *out = nullptr;
  tpf_status st = validate(d);
  if (st != TPF_OK) return st;
  Layout L;
  layout(d, L);
  if (!arena) { set_error("arena is NULL"); return TPF_EINVAL; }
  if (reinterpret_cast<uintptr_t>(arena) % ALIGN) { set_error("arena must be 256-byte aligned"); return TPF_ENOMEM; }
  if (arena_bytes < L.total) {
    set_error("arena too small: %zu bytes given, %zu needed", arena_bytes, L.total);
    return TPF_ENOMEM;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  tpf_grid *g = new (std::nothrow) tpf_grid();
  if (!g) { set_error("host allocation failed"); return TPF_ENOMEM; }
  std::memset(g, 0, sizeof(*g));
  TPF_HIP(hipGetDevice(&g->device));
  g->dim = d->dim;
  g->nst = L.nst;
  g->L = L.L;
  g->prec = d->precision;
  g->nu_pre = d->nu_pre;
  g->nu_post = d->nu_post;
  g->kmax = d->limex_stages;
  g->omega = d->omega;
  g->smoother = d->smoother;
  g->line_pair_max = TPF_LINE_PAIR_MAX_LINES;
  g->ncells = L.ncells;
  g->bytes = L.total;
  Phys &P = g->P;
  P.nx = d->n[0]; P.ny = d->n[1]; P.nz = d->n[2];
  P.N = L.N;
  P.ncx = d->n[0] - 1; P.ncy = d->n[1] - 1; P.ncz = d->dim == 3 ? d->n[2] - 1 : 1;
  for (int a = 0; a < 3; ++a) {
    P.h[a] = (a < d->dim) ? d->extent[a] / (d->n[a] - 1) : 1.0;
    P.g[a] = a < d->dim ? d->gravity[a] : 0.0;
  }
  P.rho_w = d->rho[0]; P.rho_n = d->rho[1]; P.mu_w = d->mu[0]; P.mu_n = d->mu[1];
  P.swr = d->s_res[0]; P.snr = d->s_res[1];
  P.D = (1.0 - P.swr) - P.snr;
  P.kr_model = d->kr_model;
  P.pad_ = 0;
  P.kr_aw = d->kr_model == TPF_KR_POLY ? d->kr_coef[0] : 0.0;
  P.kr_an = d->kr_model == TPF_KR_POLY ? d->kr_coef[1] : 0.0;
  P.vol = P.h[0] * P.h[1] * (d->dim == 3 ? P.h[2] : 1.0);
  P.scv = P.vol / (1 << d->dim);
  for (int a = 0; a < 3; ++a) P.area[a] = (a < d->dim) ? P.vol / ((1 << (d->dim - 1)) * P.h[a]) : 0.0;

  char *base = static_cast<char *>(arena);
  size_t o = L.off_cells;
  const size_t cb = align_up(L.ncells * sizeof(double));
  (void)cb;
  g->K = reinterpret_cast<double *>(base + o);
  g->phi = g->K + L.ncells;
  g->pd = g->phi + L.ncells;
  g->lam = g->pd + L.ncells;
  o = L.off_vert;
  g->pdmin = reinterpret_cast<double *>(base + o); o += align_up(L.N * sizeof(double));
  g->lamref = reinterpret_cast<double *>(base + o); o += align_up(L.N * sizeof(double));
  g->pv = reinterpret_cast<double *>(base + o); o += align_up(2 * L.N * sizeof(double));
  g->dval = reinterpret_cast<double *>(base + o); o += align_up(2 * L.N * sizeof(double));
  g->Q = reinterpret_cast<double *>(base + o); o += align_up(2 * L.N * sizeof(double));
  g->dmask = reinterpret_cast<uint8_t *>(base + o); o += align_up(L.N);
  const size_t vsz = d->precision != TPF_FP64 ? sizeof(float) : sizeof(double);
  for (int l = 0; l < L.L; ++l) {
    Level &lv = g->lv[l];
    for (int a = 0; a < 3; ++a) lv.n[a] = L.n[l][a];
    lv.N = L.Nl[l];
    o = L.off_lv[l];
    lv.A64 = reinterpret_cast<double *>(base + o); o += align_up((size_t)L.nst * 4 * lv.N * sizeof(double));
    lv.A32 = nullptr;
    lv.A16 = nullptr;
    lv.s16 = nullptr;
    if (d->precision == TPF_MIXED || (d->precision == TPF_MIXED16 && l == 0)) {
      lv.A32 = reinterpret_cast<float *>(base + o);
      o += align_up((size_t)(l == 0 ? tiled_blocks(lv.N, L.nst) : L.nst * lv.N) * 4 * sizeof(float));
    }
    if (d->precision == TPF_MIXED16 && l > 0) {
      lv.A16 = reinterpret_cast<uint16_t *>(base + o);
      o += align_up((size_t)L.nst * 4 * lv.N * sizeof(uint16_t));
      lv.s16 = reinterpret_cast<float *>(base + o);
      o += align_up(2 * lv.N * sizeof(float));
    }
    lv.mst = reinterpret_cast<double *>(base + o); o += align_up(2 * lv.N * sizeof(double));
    lv.x = base + o; o += align_up(2 * lv.N * vsz);
    lv.y = base + o; o += align_up(2 * lv.N * vsz);
    lv.b = base + o; o += align_up(2 * lv.N * vsz);
    lv.r = base + o; o += align_up(2 * lv.N * vsz);
    lv.lf = nullptr;
    if (d->smoother == TPF_SMOOTH_LINE && l + 1 < L.L) {
      lv.lf = base + o;
      o += align_up(12 * lv.N * vsz);
    }
  }
  g->nc = L.nc;
  o = L.off_coarse;
  g->lu = reinterpret_cast<double *>(base + o); o += align_up((size_t)L.nc * L.nc * sizeof(double));
  g->ainv = reinterpret_cast<double *>(base + o); o += align_up((size_t)L.nc * L.nc * sizeof(double));
  g->piv = reinterpret_cast<int *>(base + o);
  g->rapb = reinterpret_cast<double *>(base + L.off_rapb);
  o = L.off_kry;
  double **kv[10] = {&g->r, &g->rh, &g->p, &g->v, &g->s, &g->t, &g->ph, &g->sh, &g->w, &g->xb};
  for (int k = 0; k < 10; ++k) { *kv[k] = reinterpret_cast<double *>(base + o); o += align_up(2 * L.N * sizeof(double)); }
  g->part = reinterpret_cast<double *>(base + L.off_part);
  g->npart = L.npart;
  g->scal = reinterpret_cast<double *>(base + L.off_scal);
  g->line_bad = reinterpret_cast<int *>(base + L.off_flags);
  o = L.off_lx;
  g->u0 = reinterpret_cast<double *>(base + o); o += align_up(2 * L.N * sizeof(double));
  g->f0 = reinterpret_cast<double *>(base + o); o += align_up(2 * L.N * sizeof(double));
  g->fv = reinterpret_cast<double *>(base + o); o += align_up(2 * L.N * sizeof(double));
  g->ua = reinterpret_cast<double *>(base + o); o += align_up(2 * L.N * sizeof(double));
  if (d->limex_stages > 0) {
    g->Tp = reinterpret_cast<double *>(base + o); o += align_up(2 * L.N * sizeof(double));
    for (int k = 0; k < d->limex_stages; ++k) {
      g->T[k] = reinterpret_cast<double *>(base + o);
      o += align_up(2 * L.N * sizeof(double));
    }
  }
  hipError_t he = hipHostMalloc(reinterpret_cast<void **>(&g->hscal), NSCAL * sizeof(double), hipHostMallocDefault);
  if (he != hipSuccess) {
    set_error("hipHostMalloc failed: %s", hipGetErrorString(he));
    delete g;
    return TPF_EDEVICE;
  }
  he = hipEventCreateWithFlags(&g->scal_ev, hipEventDisableTiming);
  if (he != hipSuccess) {
    set_error("hipEventCreate failed: %s", hipGetErrorString(he));
    (void)hipHostFree(g->hscal);
    delete g;
    return TPF_EDEVICE;
  }
  auto fail = [&](tpf_status e) {
    (void)hipEventDestroy(g->scal_ev);
    (void)hipHostFree(g->hscal);
    delete g;
    return e;
  };
#define UP(dst, src, bytes)                                                                   \
  do {                                                                                        \
    hipError_t e_ = hipMemcpyAsync((dst), (src), (bytes), hipMemcpyHostToDevice, s);          \
    if (e_ != hipSuccess) {                                                                   \
      set_error("upload failed: %s", hipGetErrorString(e_));                                  \
      return fail(TPF_EDEVICE);                                                               \
    }                                                                                         \
  } while (0)
  UP(g->K, d->perm, L.ncells * sizeof(double));
  UP(g->phi, d->poro, L.ncells * sizeof(double));
  UP(g->pd, d->entry_p, L.ncells * sizeof(double));
  UP(g->lam, d->bc_lambda, L.ncells * sizeof(double));
  UP(g->dmask, d->dir_mask, L.N);
  if (d->dir_value) {
    UP(g->dval, d->dir_value, 2 * L.N * sizeof(double));
  } else {
    st = fill_zero(g->dval, 2 * L.N, s);
    if (st != TPF_OK) return fail(st);
  }
  // vertex sources first; the setup kernel adds the integrated patches to them
  if (d->vertex_source) {
    UP(g->Q, d->vertex_source, 2 * L.N * sizeof(double));
  } else {
    st = fill_zero(g->Q, 2 * L.N, s);
    if (st != TPF_OK) return fail(st);
  }
#undef UP
  Patches pt{};
  pt.n = d->n_patches;
  for (int k = 0; k < d->n_patches; ++k) {
    const tpf_patch &p = d->patches[k];
    pt.p[k] = PatchDev{p.axis, p.side, p.phase, 0, {p.lo[0], p.lo[1]}, {p.hi[0], p.hi[1]}, p.rate};
  }
  st = setup_vertices(g, pt, s);
  if (st != TPF_OK) return fail(st);
  he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    set_error("create_grid: %s", hipGetErrorString(he));
    return fail(TPF_EDEVICE);
  }
  *out = g;
  return TPF_OK;
}

static void prof_release(tpf_grid *g);

void tpf_destroy_grid(tpf_grid *g) {
  if (!g) return;
  prof_release(g);
  if (g->vgraph_exec) (void)hipGraphExecDestroy(g->vgraph_exec);
  if (g->vgraph) (void)hipGraphDestroy(g->vgraph);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  if (g->lu_pending) (void)hipEventSynchronize(g->lu_done);  // the arena is freed after this call
  if (g->lu_stream) (void)hipStreamDestroy(g->lu_stream);
  if (g->lu_fork) (void)hipEventDestroy(g->lu_fork);
  if (g->lu_done) (void)hipEventDestroy(g->lu_done);
  if (g->scal_ev) (void)hipEventDestroy(g->scal_ev);
  if (g->hscal) (void)hipHostFree(g->hscal);
  delete g;
}

tpf_status tpf_apply_dirichlet(tpf_grid *g, double *u, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !u) { set_error("NULL argument"); return TPF_EINVAL; }
  return launch_apply_dirichlet(g, u, reinterpret_cast<hipStream_t>(stream));
}

tpf_status tpf_residual(tpf_grid *g, const double *u, double *f, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !u || !f) { set_error("NULL argument"); return TPF_EINVAL; }
  if (u == f) { set_error("u and f may not alias"); return TPF_EINVAL; }
  return launch_residual(g, u, f, reinterpret_cast<hipStream_t>(stream));
}

tpf_status tpf_assemble_stage(tpf_grid *g, const double *u0, double h, double *f0_out, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !u0) { set_error("NULL argument"); return TPF_EINVAL; }
  if (!(h > 0.0) || !std::isfinite(h)) { set_error("h must be positive and finite"); return TPF_EINVAL; }
  if (f0_out == u0) { set_error("u0 and f0_out may not alias"); return TPF_EINVAL; }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  tpf_status st = launch_assemble(g, u0, h, f0_out ? f0_out : g->f0, s);
  if (st != TPF_OK) return st;
  st = build_hierarchy(g, s);
  if (st != TPF_OK) return st;
  g->assembled = true;
  g->has_f0 = true;
  return TPF_OK;
}

tpf_status tpf_solve_stage_static(tpf_grid *g, const double *f, double *x, double rtol, int32_t maxit,
                                  tpf_solve_stats *stats, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !f || !x) { set_error("NULL argument"); return TPF_EINVAL; }
  if (f == x) { set_error("f and x may not alias"); return TPF_EINVAL; }
  if (!(rtol > 0.0) || maxit < 1) { set_error("need rtol > 0 and maxit >= 1"); return TPF_EINVAL; }
  if (!g->assembled) { set_error("solve_stage before assemble_stage"); return TPF_ESTATE; }
  const size_t need = static_solve_bytes(g);
  if (need > STATIC_SCRATCH_BYTES) {
    set_error("tpf_solve_stage_static: the grid needs %zu bytes of workspace, the static array holds %zu "
              "(at most about %lld vertices); use tpf_solve_stage", need, STATIC_SCRATCH_BYTES,
              (long long)(STATIC_SCRATCH_BYTES / (9 * 16 + 1)));
    return TPF_EINVAL;
  }
  int dev = -1;
  TPF_HIP(hipGetDevice(&dev));
  if (dev != g->device) {
    set_error("the grid lives on device %d but device %d is current", g->device, dev);
    return TPF_EINVAL;
  }
  void *base = nullptr;
  tpf_status st = scratch_for_current_device(&base);
  if (st != TPF_OK) return st;
  // point the grid's solve workspace into the static array for this call
  double **kv[9] = {&g->r, &g->rh, &g->p, &g->v, &g->s, &g->t, &g->ph, &g->sh, &g->w};
  double *saved[9];
  double *saved_part = g->part, *saved_scal = g->scal;
  char *c = static_cast<char *>(base);
  for (int k = 0; k < 9; ++k) {
    saved[k] = *kv[k];
    *kv[k] = reinterpret_cast<double *>(c);
    c += align_up(2 * (size_t)g->P.N * sizeof(double));
  }
  g->part = reinterpret_cast<double *>(c);
  c += align_up(4 * (size_t)g->npart * sizeof(double));
  g->scal = reinterpret_cast<double *>(c);
  // a coarse-level graph is replayed if one exists; capturing one would allocate
  const int saved_graph = g->coarse_graph;
  if (!g->vgraph_exec) g->coarse_graph = 0;
  st = bicgstab(g, f, x, rtol, maxit, stats, reinterpret_cast<hipStream_t>(stream));
  g->coarse_graph = saved_graph;
  for (int k = 0; k < 9; ++k) *kv[k] = saved[k];
  g->part = saved_part;
  g->scal = saved_scal;
  return st;
}

tpf_status tpf_rescale_stage(tpf_grid *g, double h, tpf_stream stream) {
  g_err[0] = 0;
  if (!g) { set_error("NULL argument"); return TPF_EINVAL; }
  if (!(h > 0.0) || !std::isfinite(h)) { set_error("h must be positive and finite"); return TPF_EINVAL; }
  if (!g->assembled) { set_error("rescale_stage before assemble_stage"); return TPF_ESTATE; }
  const tpf_status st = rescale_stage(g, g->h_stage / h, reinterpret_cast<hipStream_t>(stream));
  if (st == TPF_OK) g->h_stage = h;
  return st;
}

tpf_status tpf_solve_stage(tpf_grid *g, const double *f, double *x, double rtol, int32_t maxit,
                           tpf_solve_stats *stats, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !f || !x) { set_error("NULL argument"); return TPF_EINVAL; }
  if (f == x) { set_error("f and x may not alias"); return TPF_EINVAL; }
  if (!(rtol > 0.0) || maxit < 1) { set_error("need rtol > 0 and maxit >= 1"); return TPF_EINVAL; }
  if (!g->assembled) { set_error("solve_stage before assemble_stage"); return TPF_ESTATE; }
  return bicgstab(g, f, x, rtol, maxit, stats, reinterpret_cast<hipStream_t>(stream));
}

tpf_status tpf_limex_step(tpf_grid *g, double *u, double *t, double *dt, const tpf_limex_opts *opts,
                          tpf_limex_stats *stats, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !u || !t || !dt || !opts) { set_error("NULL argument"); return TPF_EINVAL; }
  if (opts->stages < 1 || opts->stages > g->kmax) {
    set_error("stages = %d but the grid was created with limex_stages = %d", opts->stages, g->kmax);
    return TPF_EINVAL;
  }
  if (!(*dt > 0.0) || !std::isfinite(*dt) || !(opts->tol > 0.0) || !(opts->safety > 0.0) ||
      !(opts->dt_max > 0.0) || !(opts->rtol > 0.0) || opts->maxit < 1) {
    set_error("invalid LIMEX options or step");
    return TPF_EINVAL;
  }
  return limex_step(g, u, t, dt, opts, stats, reinterpret_cast<hipStream_t>(stream));
}

tpf_status tpf_storage(tpf_grid *g, const double *u, double *m, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !u || !m) { set_error("NULL argument"); return TPF_EINVAL; }
  if (u == m) { set_error("u and m may not alias"); return TPF_EINVAL; }
  return launch_storage(g, u, m, reinterpret_cast<hipStream_t>(stream));
}

tpf_status tpf_ie_step(tpf_grid *g, double *u, double tau, const tpf_newton_opts *opts, tpf_newton_stats *stats,
                       tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !u || !opts) { set_error("NULL argument"); return TPF_EINVAL; }
  if (!(tau > 0.0) || !std::isfinite(tau)) { set_error("tau must be positive and finite"); return TPF_EINVAL; }
  if (opts->max_newton < 1 || opts->max_halvings < 0 || opts->maxit < 1 || !(opts->atol >= 0.0) ||
      !(opts->rtol >= 0.0) || !(opts->lin_rtol > 0.0) || !(opts->xtol >= 0.0) || !std::isfinite(opts->xtol)) {
    set_error("invalid Newton options");
    return TPF_EINVAL;
  }
  return ie_step(g, u, tau, opts, stats, reinterpret_cast<hipStream_t>(stream));
}

tpf_status tpf_project_pressure(tpf_grid *g, double *u, double h_p, const tpf_newton_opts *opts,
                                tpf_newton_stats *stats, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !u || !opts) { set_error("NULL argument"); return TPF_EINVAL; }
  if (!(h_p > 0.0) || !std::isfinite(h_p)) { set_error("h_p must be positive and finite"); return TPF_EINVAL; }
  if (opts->max_newton < 1 || opts->maxit < 1 || !(opts->atol >= 0.0) || !(opts->rtol >= 0.0) ||
      !(opts->lin_rtol > 0.0)) {
    set_error("invalid Newton options");
    return TPF_EINVAL;
  }
  return project_pressure(g, u, h_p, opts, stats, reinterpret_cast<hipStream_t>(stream));
}

tpf_status tpf_set_coarse_graph(tpf_grid *g, int32_t enable) {
  g_err[0] = 0;
  if (!g) { set_error("NULL argument"); return TPF_EINVAL; }
  g->coarse_graph = enable ? 1 : 0;
  return TPF_OK;
}

tpf_status tpf_set_line_pairs(tpf_grid *g, int64_t max_lines) {
  if (!g || max_lines < 0) {
    set_error("need a grid and max_lines >= 0");
    return TPF_EINVAL;
  }
  g->line_pair_max = max_lines;
  return TPF_OK;
}

int32_t tpf_levels(const tpf_grid *g) { return g ? g->L : 0; }

tpf_status tpf_level_dims(const tpf_grid *g, int32_t level, int32_t n_out[3]) {
  if (!g || !n_out || level < 0 || level >= g->L) { set_error("bad level"); return TPF_EINVAL; }
  for (int a = 0; a < 3; ++a) n_out[a] = g->lv[level].n[a];
  return TPF_OK;
}

tpf_status tpf_copy_matrix(tpf_grid *g, int32_t level, int32_t precision, void *dst, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !dst || level < 0 || level >= g->L) { set_error("bad argument"); return TPF_EINVAL; }
  if (!g->assembled) { set_error("no assembled matrix"); return TPF_ESTATE; }
  const Level &lv = g->lv[level];
  const size_t cnt = (size_t)g->nst * 4 * lv.N;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (precision == TPF_FP64) {
    TPF_HIP(hipMemcpyAsync(dst, lv.A64, cnt * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else if (precision == TPF_MIXED && (g->prec == TPF_MIXED || (g->prec == TPF_MIXED16 && level == 0))) {
    if (level == 0) return untile_matrix32(g, reinterpret_cast<float *>(dst), s);
    TPF_HIP(hipMemcpyAsync(dst, lv.A32, cnt * sizeof(float), hipMemcpyDeviceToDevice, s));
  } else if (precision == TPF_MIXED16 && g->prec == TPF_MIXED16 && level > 0) {
    return expand_matrix16(g, level, reinterpret_cast<float *>(dst), s);
  } else {
    set_error("no matrix of that precision on this level");
    return TPF_EINVAL;
  }
  return TPF_OK;
}

tpf_status tpf_spmv(tpf_grid *g, int32_t level, const double *x, double *y, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !x || !y || x == y || level < 0 || level >= g->L) { set_error("bad argument"); return TPF_EINVAL; }
  if (!g->assembled) { set_error("no assembled matrix"); return TPF_ESTATE; }
  return spmv64(g, level, x, y, reinterpret_cast<hipStream_t>(stream));
}

tpf_status tpf_precondition(tpf_grid *g, const double *b, double *x, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !b || !x || b == x) { set_error("bad argument"); return TPF_EINVAL; }
  if (!g->assembled) { set_error("no assembled matrix"); return TPF_ESTATE; }
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const tpf_status lc = check_line_factors(g, s);  // a singular line pivot: no V-cycle
  if (lc != TPF_OK) return lc;
  return vcycle(g, b, x, s);
}

tpf_status tpf_copy_coarse_inverse(tpf_grid *g, double *dst, tpf_stream stream) {
  g_err[0] = 0;
  if (!g || !dst) { set_error("bad argument"); return TPF_EINVAL; }
  if (!g->assembled) { set_error("no assembled matrix"); return TPF_ESTATE; }
  const tpf_status lj = lu_join(g, reinterpret_cast<hipStream_t>(stream));
  if (lj != TPF_OK) return lj;
  TPF_HIP(hipMemcpyAsync(dst, g->ainv, (size_t)g->nc * g->nc * sizeof(double), hipMemcpyDeviceToDevice,
                         reinterpret_cast<hipStream_t>(stream)));
  return TPF_OK;
}

const double *tpf_pdmin_ptr(const tpf_grid *g) { return g ? g->pdmin : nullptr; }

static void prof_release(tpf_grid *g) {
  Prof &p = g->prof;
  if (p.ev) {
    for (int i = 0; i < 2 * p.cap; ++i) (void)hipEventDestroy(p.ev[i]);
    delete[] p.ev;
  }
  delete[] p.cls;
  p = Prof();
}

tpf_status tpf_profile_begin(tpf_grid *g, int32_t max_launches, uint32_t class_mask) {
  g_err[0] = 0;
  if (!g || max_launches < 1 || max_launches > (1 << 20)) { set_error("bad argument"); return TPF_EINVAL; }
  prof_release(g);
  Prof &p = g->prof;
  p.ev = new (std::nothrow) hipEvent_t[2 * (size_t)max_launches];
  p.cls = new (std::nothrow) int[max_launches];
  if (!p.ev || !p.cls) { prof_release(g); set_error("host allocation failed"); return TPF_ENOMEM; }
  for (int i = 0; i < 2 * max_launches; ++i) {
    if (hipEventCreate(&p.ev[i]) != hipSuccess) {
      p.cap = i / 2;
      prof_release(g);
      set_error("hipEventCreate failed");
      return TPF_EDEVICE;
    }
    p.cap = (i + 1) / 2;
  }
  p.cap = max_launches;
  p.used = 0;
  p.mask = class_mask ? class_mask : ~0u;
  p.active = 1;
  return TPF_OK;
}

tpf_status tpf_profile_end(tpf_grid *g, tpf_kernel_time *out) {
  g_err[0] = 0;
  if (!g || !out) { set_error("bad argument"); return TPF_EINVAL; }
  Prof &p = g->prof;
  for (int c = 0; c < TPF_K_COUNT; ++c) out[c] = tpf_kernel_time{0, 0, 0.0};
  tpf_status st = TPF_OK;
  for (int i = 0; i < p.used; ++i) {
    if (hipEventSynchronize(p.ev[2 * i + 1]) != hipSuccess) { st = TPF_EDEVICE; break; }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.ev[2 * i], p.ev[2 * i + 1]) != hipSuccess) { st = TPF_EDEVICE; break; }
    out[p.cls[i]].count += 1;
    out[p.cls[i]].total_ms += ms;
  }
  if (st != TPF_OK) set_error("event timing failed");
  prof_release(g);
  return st;
}

}  // extern "C"
