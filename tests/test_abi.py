"""Host-only checks of the C ABI: the library loads, exports every symbol the header
declares, sizes the arena and rejects invalid descriptors (no compute calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2506_04763_amd import _lib as L
import paper_2506_04763_amd as tpf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "tpf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L._SIGS), set(names) ^ set(L._SIGS)


def test_struct_layouts_match_header():
    # offsets follow natural C alignment of the header's field order
    assert C.sizeof(L.Patch) == 56
    assert L.GridDesc.omega.offset == 192 and L.GridDesc.kr_model.offset == 200
    assert L.GridDesc.kr_coef.offset == 208 and L.GridDesc.vertex_source.offset == 224
    assert C.sizeof(L.GridDesc) == 232
    assert C.sizeof(L.SolveStats) == 32
    assert C.sizeof(L.LimexOpts) == 40
    assert C.sizeof(L.LimexStats) == 40


def _bytes_expected(scn, prec, limex=0, smoother="point"):
    """Independent re-derivation of the arena size from the documented layout."""
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    nst = 27 if scn.dim == 3 else 9
    vb = 8 if prec == "fp64" else 4  # level-vector entry bytes
    N = scn.nverts
    n = list(scn.n)
    sizes = [tuple(n)]
    for _ in range(scn.levels - 1):
        n = [(v - 1) // 2 + 1 if a < scn.dim else 1 for a, v in enumerate(n)]
        sizes.append(tuple(n))
    tot = al(4 * scn.ncells * 8) + 2 * al(N * 8) + 3 * al(2 * N * 8) + al(N)
    for lvl, s in enumerate(sizes):
        Nl = s[0] * s[1] * s[2]
        tot += al(nst * 4 * Nl * 8)
        if prec == "mixed" or (prec == "mixed16" and lvl == 0):
            # FP32 copy; the finest one is stored in whole tiles of 64 vertices
            n32 = (Nl + 63) // 64 * 64 if lvl == 0 else Nl
            tot += al(nst * 4 * n32 * 4)
        if prec == "mixed16" and lvl > 0:  # FP16 blocks and two FP32 row scales per vertex
            tot += al(nst * 4 * Nl * 2) + al(2 * Nl * 4)
        tot += al(2 * Nl * 8)
        tot += 4 * al(2 * Nl * vb)
        if smoother == "line" and lvl + 1 < len(sizes):  # line LU: three 2x2 blocks per vertex
            tot += al(12 * Nl * vb)
    nc = 2 * sizes[-1][0] * sizes[-1][1] * sizes[-1][2]
    tot += 2 * al(nc * nc * 8) + al(nc * 4)
    tot += al(nst * 4 * N * 8) if scn.levels > 1 else 0   # Galerkin-product scratch
    tot += 10 * al(2 * N * 8)
    tot += al(4 * max(1024, (N + 255) // 256) * 8) + al(32 * 8) + al(4)  # partials, scalars, flags
    # step vectors: u0, F0, F(v) and the Newton base point, then the LIMEX tableau
    tot += al(2 * N * 8) * (4 + (1 + limex if limex else 0))
    return tot


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed16"])
def test_grid_bytes(prec):
    scn = W.small_cube(17, levels=3)
    nb = tpf.grid_bytes(scn, precision=prec)
    assert nb == _bytes_expected(scn, prec)
    scn2 = W.lens_2d()
    assert tpf.grid_bytes(scn2, precision=prec, limex_stages=2) == _bytes_expected(scn2, prec, 2)
    for s_ in (scn, scn2):
        assert tpf.grid_bytes(s_, precision=prec, smoother="line") == _bytes_expected(s_, prec, smoother="line")


def test_grid_bytes_c3_fits_hbm():
    # 129^3 mixed: matrices dominate (27 blocks x 4 x (8 + 4) bytes per vertex)
    scn = W._empty("c3", 3, (129, 129, 129), (1, 1, 1), (0, 0, -9.81))
    nb_per_vertex = 27 * 4 * 12
    est = 129 ** 3 * nb_per_vertex
    assert est < 3e9


def _desc_ok():
    scn = W.small_cube(9, levels=3)
    return scn


@pytest.mark.parametrize("mutate,msg", [
    (lambda s: setattr(s, "levels", 5), "coarsened"),
    (lambda s: s.perm.__setitem__(3, -1.0), "perm"),
    (lambda s: s.perm.__setitem__(0, np.nan), "perm"),
    (lambda s: s.poro.__setitem__(1, 0.0), "poro"),
    (lambda s: s.bc_lambda.__setitem__(2, 0.0), "bc_lambda"),
    (lambda s: setattr(s, "mu", (0.0, 1e-3)), "mu"),
    (lambda s: setattr(s, "s_res", (0.6, 0.5)), "S_wr"),
    (lambda s: s.dir_value.__setitem__((0, 0), np.inf), "dir_value"),
    (lambda s: setattr(s, "n", (9, 9, 8)), ""),
    (lambda s: setattr(s, "kr_model", "poly") or setattr(s, "kr_coef", (0.9, 0.0)), "kr_coef[1]"),
    (lambda s: setattr(s, "kr_model", "poly") or setattr(s, "kr_coef", (np.nan, 0.5)), "kr_coef[0]"),
    (lambda s: setattr(s, "vertex_source", np.full((s.nverts, 2), np.inf)), "vertex_source"),
])
def test_invalid_descriptors_rejected(mutate, msg):
    scn = _desc_ok()
    assert tpf.validate(scn) == L.TPF_OK
    try:
        mutate(scn)
    except Exception:
        pytest.skip("mutation not applicable")
    st = tpf.validate(scn)
    assert st == L.TPF_EINVAL
    assert msg in L.last_error()


def test_invalid_options_rejected():
    scn = _desc_ok()
    assert tpf.validate(scn, omega=2.5) == L.TPF_EINVAL
    assert tpf.validate(scn, nu_pre=0) == L.TPF_EINVAL
    assert tpf.validate(scn, precision=7) == L.TPF_EINVAL
    assert tpf.validate(scn, limex_stages=9) == L.TPF_EINVAL
    assert tpf.validate(scn, smoother=2) == L.TPF_EINVAL
    assert tpf.validate(scn, smoother="line") == L.TPF_OK
    big = W.small_cube(9, levels=1)   # 729 vertices -> 1458 unknowns on the only level: allowed
    assert tpf.validate(big) == L.TPF_OK
    huge = W.small_cube(65, levels=2)  # 33^3 coarsest -> too many unknowns for the dense solve
    assert tpf.validate(huge) == L.TPF_EINVAL
    assert "coarsest" in L.last_error()


def test_create_grid_rejects_small_arena_without_gpu_work():
    lib = L.load()
    scn = _desc_ok()
    dd = tpf.make_desc(scn)
    h = C.c_void_p()
    # a NULL arena and a misaligned one are rejected before any HIP call
    assert lib.tpf_create_grid(C.byref(dd.desc), None, 0, None, C.byref(h)) == L.TPF_EINVAL
    assert lib.tpf_create_grid(C.byref(dd.desc), C.c_void_p(8), 1 << 40, None, C.byref(h)) == L.TPF_ENOMEM
    assert lib.tpf_create_grid(C.byref(dd.desc), C.c_void_p(1 << 20), 16, None, C.byref(h)) == L.TPF_ENOMEM
    assert "too small" in L.last_error()


def test_product_path_does_not_import_oracle():
    import subprocess
    import sys
    code = ("import sys; import paper_2506_04763_amd, paper_2506_04763_amd._lib as L; L.load(); "
            "bad=[m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]; print(bad); "
            "assert not bad")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
