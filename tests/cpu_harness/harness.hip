// CPU build of the library's per-thread kernel bodies (test infrastructure).
//
// The assembly, constitutive-law and Galerkin-product bodies of the HIP library are
// __host__ __device__ functions; this program includes their sources and runs every
// thread of a launch on the host, over buffers of exactly the sizes the kernels are
// given, so that an AddressSanitizer build (host side) catches any access outside
// them.  It reads one binary input file and writes one binary output file (layouts in
// tests/test_cpu_harness.py); the test compares the results with the FP64 oracle.
//
//   harness math     in out   log_pos / exp_fin on given arguments
//   harness assemble in out   residual and stage-matrix rows (inline laws, the corner
//                             pass, and in 3D the two-thread split of the row)
//   harness rap      in out   the two-pass Galerkin product over the launch's thread
//                             mapping, with a count of the writes to every block
//   harness line     in out   the line-block Jacobi bodies: the block LU of every line
//                             and one sweep per line (in place, or from a zero guess)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "assemble.hip"
#include "line.h"
#include "rap.hip"

namespace tpf {
void set_error(const char *, ...) {}
}  // namespace tpf

using namespace tpf;

namespace {

struct Reader {
  FILE *f;
  double d() {
    double v;
    if (fread(&v, sizeof v, 1, f) != 1) { fprintf(stderr, "short input\n"); exit(2); }
    return v;
  }
  int i() { return (int)d(); }
  std::vector<double> vec(size_t n) {
    std::vector<double> v(n);
    if (n && fread(v.data(), sizeof(double), n, f) != n) { fprintf(stderr, "short input\n"); exit(2); }
    return v;
  }
};

void put(FILE *f, const std::vector<double> &v) { fwrite(v.data(), sizeof(double), v.size(), f); }

int run_math(Reader &r, FILE *out) {
  const int n = r.i();
  std::vector<double> x = r.vec(n), y = r.vec(n), lg(n), ex(n);
  for (int k = 0; k < n; ++k) {
    lg[k] = log_pos(x[k]);
    ex[k] = exp_fin(y[k]);
  }
  put(out, lg);
  put(out, ex);
  return 0;
}

// Phys of a grid, filled as tpf_create_grid fills it.
Phys make_phys(Reader &r, int &dim) {
  Phys P{};
  dim = r.i();
  int n[3];
  for (int a = 0; a < 3; ++a) n[a] = r.i();
  double h[3], g[3], rho[2], mu[2], sres[2], coef[2];
  for (int a = 0; a < 3; ++a) h[a] = r.d();
  for (int a = 0; a < 3; ++a) g[a] = r.d();
  for (int k = 0; k < 2; ++k) rho[k] = r.d();
  for (int k = 0; k < 2; ++k) mu[k] = r.d();
  for (int k = 0; k < 2; ++k) sres[k] = r.d();
  const int kr_model = r.i();
  for (int k = 0; k < 2; ++k) coef[k] = r.d();
  P.nx = n[0]; P.ny = n[1]; P.nz = n[2];
  P.N = (long long)n[0] * n[1] * n[2];
  P.ncx = n[0] - 1; P.ncy = n[1] - 1; P.ncz = dim == 3 ? n[2] - 1 : 1;
  for (int a = 0; a < 3; ++a) {
    P.h[a] = a < dim ? h[a] : 1.0;
    P.g[a] = a < dim ? g[a] : 0.0;
  }
  P.rho_w = rho[0]; P.rho_n = rho[1]; P.mu_w = mu[0]; P.mu_n = mu[1];
  P.swr = sres[0]; P.snr = sres[1];
  P.D = (1.0 - P.swr) - P.snr;
  P.kr_model = kr_model;
  P.kr_aw = kr_model == TPF_KR_POLY ? coef[0] : 0.0;
  P.kr_an = kr_model == TPF_KR_POLY ? coef[1] : 0.0;
  P.vol = P.h[0] * P.h[1] * (dim == 3 ? P.h[2] : 1.0);
  P.scv = P.vol / (1 << dim);
  for (int a = 0; a < 3; ++a) P.area[a] = a < dim ? P.vol / ((1 << (dim - 1)) * P.h[a]) : 0.0;
  return P;
}

template <int DIM>
void assemble_all(const Phys &P, const CellIn &in_inline, const CellIn &in_pairs, const uint8_t *dmask,
                  const double *Q, double inv_h, FILE *out) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  const long long N = P.N;
  std::vector<double> A(NST * 4 * N), F(2 * N), mst(2 * N);
  for (long long v = 0; v < N; ++v)
    assemble_vertex<DIM, true, false, false>(v, P, in_inline, dmask, Q, inv_h, A.data(), nullptr, F.data(),
                                             mst.data());
  put(out, A);
  put(out, F);
  put(out, mst);
  std::fill(A.begin(), A.end(), -7.0);
  std::fill(F.begin(), F.end(), -7.0);
  for (long long v = 0; v < N; ++v)
    assemble_vertex<DIM, true, false, true>(v, P, in_pairs, dmask, Q, inv_h, A.data(), nullptr, F.data(),
                                            mst.data());
  put(out, A);
  put(out, F);
  if constexpr (DIM == 3) {
    // the two-thread split of k_assemble3_split: cells below (slots 0..17) and above
    // (slots 9..26), the shared plane added to the upper half's accumulators
    std::fill(A.begin(), A.end(), -7.0);
    std::fill(F.begin(), F.end(), -7.0);
    for (long long v = 0; v < N; ++v) {
      double a1[18][4] = {}, a0[18][4] = {};
      double Fw1 = 0, Fn1 = 0, mw1 = 0, mn1 = 0, Fw0 = 0, Fn0 = 0, mw0 = 0, mn0 = 0;
      accumulate_cells<3, true, 1, 0, 18, true>(v, P, in_pairs, a1, Fw1, Fn1, mw1, mn1);
      accumulate_cells<3, true, 0, 9, 18, true>(v, P, in_pairs, a0, Fw0, Fn0, mw0, mn0);
      for (int k = 0; k < 9; ++k)
        for (int e = 0; e < 4; ++e) a0[k][e] += a1[9 + k][e];
      Fw0 += Fw1; Fn0 += Fn1; mw0 += mw1; mn0 += mn1;
      finish_vertex<3, true, false, true, 9, 18>(v, P, dmask, Q, inv_h, a0, Fw0, Fn0, mw0, mn0, A.data(), nullptr,
                                                 F.data(), mst.data());
      double low[9][4];
      for (int k = 0; k < 9; ++k)
        for (int e = 0; e < 4; ++e) low[k][e] = a1[k][e];
      finish_vertex<3, true, false, false, 0, 9>(v, P, dmask, Q, inv_h, low, 0.0, 0.0, 0.0, 0.0, A.data(), nullptr,
                                                 nullptr, nullptr);
    }
    put(out, A);
    put(out, F);
  }
}

int run_assemble(Reader &r, FILE *out) {
  int dim = 0;
  const Phys P = make_phys(r, dim);
  const double inv_h = r.d();
  const long long N = P.N, nc = (long long)P.ncx * P.ncy * P.ncz;
  std::vector<double> K = r.vec(nc), phi = r.vec(nc), pd = r.vec(nc), lam = r.vec(nc);
  std::vector<double> pdmin = r.vec(N), lamref = r.vec(N), maskd = r.vec(N), Q = r.vec(2 * N), u = r.vec(2 * N);
  std::vector<uint8_t> dmask(N);
  for (long long v = 0; v < N; ++v) dmask[v] = (uint8_t)maskd[v];
  std::vector<double> pv(2 * N);
  for (long long v = 0; v < N; ++v) vertex_pc(v, P, u.data(), pdmin.data(), lamref.data(), pv.data());
  const int NC = 1 << dim;
  std::vector<double> cp(nc * NC * CP);  // the corner pass's (cell, corner) laws, exactly sized
  CellIn in{u.data(), K.data(), phi.data(), pd.data(), lam.data(), pdmin.data(), pv.data(), nullptr};
  CellIn inp = in;
  inp.cp = cp.data();
  for (long long c = 0; c < nc; ++c) {
    if (dim == 3)
      corner_pass<3>(c, P, in, cp.data());
    else
      corner_pass<2>(c, P, in, cp.data());
  }
  if (dim == 3)
    assemble_all<3>(P, in, inp, dmask.data(), Q.data(), inv_h, out);
  else
    assemble_all<2>(P, in, inp, dmask.data(), Q.data(), inv_h, out);
  return 0;
}

template <int DIM>
int rap_all(Reader &r, FILE *out) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  int nf[3], ncv[3];
  for (int a = 0; a < 3; ++a) nf[a] = r.i();
  for (int a = 0; a < 3; ++a) ncv[a] = r.i();
  const bool mask = r.i() != 0;
  const double vr = r.d();
  const long long Nf = (long long)nf[0] * nf[1] * nf[2], Nc = (long long)ncv[0] * ncv[1] * ncv[2];
  const Geo F = geo_of(nf, Nf), C = geo_of(ncv, Nc);
  std::vector<double> Af = r.vec(NST * 4 * Nf), mf = r.vec(2 * Nf), maskd = r.vec(Nf);
  std::vector<uint8_t> fmask(Nf);
  for (long long v = 0; v < Nf; ++v) fmask[v] = (uint8_t)maskd[v];
  const uint8_t *fm = mask ? fmask.data() : nullptr;
  std::vector<double> B(NST * 4 * Nf), Ac(NST * 4 * Nc), mc(2 * Nc), cntB(NST * Nf, 0.0), cntA(NST * Nc, 0.0);
  // the launch geometry of launch_rap: one wavefront per (tile of 64 vertices, slot)
  const long long wf = ((Nf + 63) / 64) * NST, wc = ((Nc + 63) / 64) * NST;
  const unsigned nbf = (unsigned)((wf + BS / 64 - 1) / (BS / 64)), nbc = (unsigned)((wc + BS / 64 - 1) / (BS / 64));
  std::vector<char> seen(std::max(nbf, nbc), 0);
  for (int pass = 0; pass < 2; ++pass) {
    const unsigned nb = pass == 0 ? nbf : nbc;
    std::fill(seen.begin(), seen.end(), 0);
    for (unsigned bid = 0; bid < nb; ++bid) {
      const unsigned blk = xcd_block(bid, nb);
      if (blk >= nb || seen[blk]) { fprintf(stderr, "xcd_block is not a permutation\n"); return 3; }
      seen[blk] = 1;
      for (int t = 0; t < BS; ++t) {
        const long long wave = (long long)blk * (BS / 64) + (t >> 6);
        long long I;
        int T;
        if (pass == 0) {
          if (!rap_thread<DIM>(wave, t & 63, Nf, I, T)) continue;
          double b[4];
          if (mask)
            rap_ap_entry<DIM, true>(I, T, F, C, Af.data(), fm, mf.data(), vr, b);
          else
            rap_ap_entry<DIM, false>(I, T, F, C, Af.data(), fm, mf.data(), vr, b);
          std::memcpy(&B[((long long)T * Nf + I) * 4], b, sizeof b);
          cntB[(long long)T * Nf + I] += 1.0;
        } else {
          if (!rap_thread<DIM>(wave, t & 63, Nc, I, T)) continue;
          if (mask)
            rap_block<DIM, true>(I, T, F, C, B.data(), fm, mf.data(), vr, Ac.data(), nullptr, mc.data());
          else
            rap_block<DIM, false>(I, T, F, C, B.data(), fm, mf.data(), vr, Ac.data(), nullptr, mc.data());
          cntA[(long long)T * Nc + I] += 1.0;
        }
      }
    }
  }
  put(out, Ac);
  put(out, mc);
  put(out, cntB);
  put(out, cntA);
  return 0;
}

int run_rap(Reader &r, FILE *out) {
  const int dim = r.i();
  return dim == 3 ? rap_all<3>(r, out) : rap_all<2>(r, out);
}

}  // namespace

// Line smoother of one level: factors every line from the FP64 stencil A into a
// buffer of exactly 12 N values of T, then runs one sweep per line.  first: rin = b,
// c kept in a separate buffer, no previous iterate; otherwise rin is the residual,
// overwritten in place by c, and xi the previous iterate.  Writes xo (2N), the count
// of lines with a singular pivot, and the factor buffer.
template <int DIM, typename T>
int line_level(Reader &r, FILE *out, const Geo &G, double omega, int first) {
  constexpr int NST = DIM == 3 ? 27 : 9;
  const long long N = G.N;
  std::vector<double> A = r.vec((size_t)NST * 4 * N), rin = r.vec(2 * N), xi = r.vec(2 * N);
  std::vector<T> lf(12 * N), rv(2 * N), cb(2 * N), xv(2 * N), xo(2 * N);
  for (long long i = 0; i < 2 * N; ++i) {
    rv[i] = (T)rin[i];
    xv[i] = (T)xi[i];
  }
  const LineGeo lg = line_geo<DIM>(G);
  double bad = 0;
  for (long long l = 0; l < lg.S; ++l)
    if (!line_factor<DIM, T>(G, A.data(), lf.data(), l)) bad += 1;
  for (long long l = 0; l < lg.S; ++l) {
    if (first)
      line_solve<DIM, T, T, 8>(G, lf.data(), rv.data(), cb.data(), nullptr, xo.data(), (T)omega, l);
    else
      line_solve<DIM, T, T, 8>(G, lf.data(), rv.data(), rv.data(), xv.data(), xo.data(), (T)omega, l);
  }
  std::vector<double> o(xo.begin(), xo.end()), f(lf.begin(), lf.end());
  put(out, o);
  put(out, std::vector<double>{bad});
  put(out, f);
  return 0;
}

int run_line(Reader &r, FILE *out) {
  const int dim = r.i();
  int n[3];
  for (int a = 0; a < 3; ++a) n[a] = r.i();
  const double omega = r.d();
  const int first = r.i();
  const int single = r.i();
  const Geo G{n[0], n[1], n[2], (long long)n[0] * n[1] * n[2]};
  if (dim == 3) return single ? line_level<3, float>(r, out, G, omega, first) : line_level<3, double>(r, out, G, omega, first);
  return single ? line_level<2, float>(r, out, G, omega, first) : line_level<2, double>(r, out, G, omega, first);
}

int main(int argc, char **argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: harness math|assemble|rap|line in out\n");
    return 2;
  }
  FILE *in = fopen(argv[2], "rb");
  FILE *out = fopen(argv[3], "wb");
  if (!in || !out) {
    fprintf(stderr, "cannot open files\n");
    return 2;
  }
  Reader r{in};
  int rc = 2;
  if (!strcmp(argv[1], "math")) rc = run_math(r, out);
  else if (!strcmp(argv[1], "assemble")) rc = run_assemble(r, out);
  else if (!strcmp(argv[1], "rap")) rc = run_rap(r, out);
  else if (!strcmp(argv[1], "line")) rc = run_line(r, out);
  fclose(in);
  fclose(out);
  return rc;
}
