"""Python binding of the gfx950 two-phase stage solver (libtpf.so).

Argument marshalling only: every step of the path runs in the HIP library.  PyTorch
provides device memory (the grid arena and the state vectors) and streams.

    g = Grid(scenario, precision="mixed")
    g.assemble_stage(u0, h)
    x, stats = g.solve_stage(f, rtol=1e-8)
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import (TPF_EBREAKDOWN, TPF_EINVAL, TPF_ENOMEM, TPF_ESTATE, TPF_FP64, TPF_MIXED,  # noqa: F401
                   TPF_NOT_CONVERGED, TPF_OK, TPF_STEP_REJECTED, TPFError)

__all__ = ["Grid", "make_desc", "grid_bytes", "validate", "TPFError"]

PRECISIONS = {"fp64": TPF_FP64, "mixed": TPF_MIXED, "mixed16": L.TPF_MIXED16}
SMOOTHERS = {"point": 0, "line": 1}  # TPF_SMOOTH_POINT, TPF_SMOOTH_LINE


class _Desc:
    """A tpf_grid_desc plus the host arrays it points to (kept alive together)."""

    def __init__(self, scn, precision="fp64", levels=None, nu_pre=2, nu_post=2, omega=2.0 / 3.0,
                 limex_stages=0, smoother="point"):
        self.keep = []
        d = L.GridDesc()
        d.dim = int(scn.dim)
        for a in range(3):
            d.n[a] = int(scn.n[a])
            d.extent[a] = float(scn.extent[a])
            d.gravity[a] = float(scn.gravity[a])
        for k in range(2):
            d.rho[k] = float(scn.rho[k])
            d.mu[k] = float(scn.mu[k])
            d.s_res[k] = float(scn.s_res[k])

        def arr(a, dtype, ctype):
            a = np.ascontiguousarray(np.asarray(a, dtype=dtype).ravel())
            self.keep.append(a)
            return a.ctypes.data_as(C.POINTER(ctype))

        d.perm = arr(scn.perm, np.float64, C.c_double)
        d.poro = arr(scn.poro, np.float64, C.c_double)
        d.entry_p = arr(scn.entry_p, np.float64, C.c_double)
        d.bc_lambda = arr(scn.bc_lambda, np.float64, C.c_double)
        d.dir_mask = arr(scn.dir_mask, np.uint8, C.c_uint8)
        d.dir_value = arr(scn.dir_value, np.float64, C.c_double)
        pats = (L.Patch * max(1, len(scn.patches)))()
        for k, p in enumerate(scn.patches):
            pats[k].axis, pats[k].side, pats[k].phase = int(p.axis), int(p.side), int(p.phase)
            for j in range(2):
                pats[k].lo[j] = float(p.lo[j])
                pats[k].hi[j] = float(p.hi[j])
            pats[k].rate = float(p.rate)
        self.keep.append(pats)
        d.patches = C.cast(pats, C.POINTER(L.Patch))
        d.n_patches = len(scn.patches)
        d.levels = int(scn.levels if levels is None else levels)
        d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        d.nu_pre, d.nu_post = int(nu_pre), int(nu_post)
        d.omega = float(omega)
        d.smoother = SMOOTHERS[smoother] if isinstance(smoother, str) else int(smoother)
        d.limex_stages = int(limex_stages)
        model = getattr(scn, "kr_model", "burdine")
        d.kr_model = {"burdine": L.TPF_KR_BURDINE, "poly": L.TPF_KR_POLY}[model]
        coef = getattr(scn, "kr_coef", (1.0, 1.0))
        d.kr_coef[0], d.kr_coef[1] = float(coef[0]), float(coef[1])
        src = getattr(scn, "vertex_source", None)
        if src is not None:
            d.vertex_source = arr(src, np.float64, C.c_double)
        self.desc = d


def make_desc(scn, **kw) -> _Desc:
    return _Desc(scn, **kw)


def validate(scn, **kw) -> int:
    lib = L.load()
    dd = _Desc(scn, **kw)
    return lib.tpf_validate(C.byref(dd.desc))


def grid_bytes(scn, **kw) -> int:
    lib = L.load()
    dd = _Desc(scn, **kw)
    n = lib.tpf_grid_bytes(C.byref(dd.desc))
    if n == 0:
        raise TPFError(TPF_EINVAL, "tpf_grid_bytes")
    return int(n)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Grid:
    """One scenario resident on one GPU (all device state in a torch-owned arena)."""

    def __init__(self, scn, precision="fp64", levels=None, nu_pre=2, nu_post=2, omega=2.0 / 3.0,
                 limex_stages=0, device=None, stream=None, arena=None, smoother="point"):
        import torch
        self.torch = torch
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the stage solver needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.scn = scn
        self.N = int(scn.nverts)
        self.dim = int(scn.dim)
        self.nst = 27 if self.dim == 3 else 9
        self._dd = _Desc(scn, precision=precision, levels=levels, nu_pre=nu_pre, nu_post=nu_post,
                         omega=omega, limex_stages=limex_stages, smoother=smoother)
        self.smoother = smoother
        self.precision = self._dd.desc.precision
        nbytes = self.lib.tpf_grid_bytes(C.byref(self._dd.desc))
        if nbytes == 0:
            raise TPFError(TPF_EINVAL, "tpf_grid_bytes")
        self.nbytes = int(nbytes)
        self._stream = stream
        with torch.cuda.device(self.device):
            self.arena = arena if arena is not None else torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            h = C.c_void_p()
            st = self.lib.tpf_create_grid(C.byref(self._dd.desc), _ptr(self.arena), self.nbytes,
                                          self._sptr(), C.byref(h))
        L.check(st, "tpf_create_grid")
        self.handle = h
        self.levels = self.lib.tpf_levels(self.handle)

    # -- helpers ------------------------------------------------------------------
    def _sptr(self):
        s = self._stream if self._stream is not None else self.torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def _vec(self, t, n=None):
        torch = self.torch
        n = 2 * self.N if n is None else n
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(np.ascontiguousarray(t, dtype=np.float64).ravel())
        if t.device != self.device or t.dtype != torch.float64 or not t.is_contiguous():
            t = t.to(device=self.device, dtype=torch.float64).contiguous()
        t = t.reshape(-1)
        if t.numel() != n:
            raise ValueError(f"expected {n} entries, got {t.numel()}")
        return t

    def empty(self, n=None):
        return self.torch.empty(2 * self.N if n is None else n, dtype=self.torch.float64, device=self.device)

    @property
    def stream(self):
        return self._stream if self._stream is not None else self.torch.cuda.current_stream(self.device)

    # -- the path -----------------------------------------------------------------
    def initial_state(self):
        return self._vec(self.scn.u0)

    def apply_dirichlet(self, u):
        u = self._vec(u)
        L.check(self.lib.tpf_apply_dirichlet(self.handle, _ptr(u), self._sptr()), "tpf_apply_dirichlet")
        return u

    def residual(self, u, out=None):
        u = self._vec(u)
        f = self.empty() if out is None else out
        L.check(self.lib.tpf_residual(self.handle, _ptr(u), _ptr(f), self._sptr()), "tpf_residual")
        return f

    def assemble_stage(self, u0, h, f0_out=None):
        """A = M(u0)/h - J(u0) and the hierarchy; if f0_out (a float64 device tensor of
        2N entries) is given it receives F(u0), computed by the same kernel."""
        u0 = self._vec(u0)
        fp = None if f0_out is None else _ptr(self._vec(f0_out))
        if f0_out is not None and fp.value != f0_out.data_ptr():
            raise ValueError("f0_out must be a contiguous float64 tensor on the grid's device")
        L.check(self.lib.tpf_assemble_stage(self.handle, _ptr(u0), float(h), fp, self._sptr()),
                "tpf_assemble_stage")
        return f0_out

    def rescale_stage(self, h):
        """Moves the assembled stage operator (M, J frozen) and its hierarchy to the step h."""
        L.check(self.lib.tpf_rescale_stage(self.handle, float(h), self._sptr()), "tpf_rescale_stage")

    def solve_stage(self, f, rtol=1e-10, maxit=500, out=None, raise_on_soft=False):
        f = self._vec(f)
        x = self.empty() if out is None else out
        st = L.SolveStats()
        status = self.lib.tpf_solve_stage(self.handle, _ptr(f), _ptr(x), float(rtol), int(maxit), C.byref(st),
                                          self._sptr())
        L.check(status, "tpf_solve_stage", soft_ok=not raise_on_soft)
        d = st.as_dict()
        d["status"] = L.STATUS_NAMES.get(status, status)
        return x, d

    def limex_step(self, u, t, dt, stages=2, tol=5e-3, safety=0.75, dt_max=8.64e6, rtol=1e-10, maxit=500):
        """One LIMEX step in place on the device tensor u; returns (accepted, t, dt_next, stats)."""
        if not (isinstance(u, self.torch.Tensor) and u.device == self.device and u.dtype == self.torch.float64):
            raise TypeError("u must be a float64 tensor on the grid's device")
        o = L.LimexOpts(int(stages), int(maxit), float(tol), float(safety), float(dt_max), float(rtol))
        st = L.LimexStats()
        tt = C.c_double(float(t))
        dd = C.c_double(float(dt))
        status = self.lib.tpf_limex_step(self.handle, _ptr(u), C.byref(tt), C.byref(dd), C.byref(o), C.byref(st),
                                         self._sptr())
        L.check(status, "tpf_limex_step", soft_ok=True)
        return status == TPF_OK, tt.value, dd.value, st.as_dict()

    def storage(self, u, out=None):
        """m(u): the storage of both phases per control volume (kg), interleaved (w, n)."""
        u = self._vec(u)
        m = self.empty() if out is None else out
        L.check(self.lib.tpf_storage(self.handle, _ptr(u), _ptr(m), self._sptr()), "tpf_storage")
        return m

    def ie_step(self, u, tau, atol=1e-8, rtol=1e-6, lin_rtol=1e-6, max_newton=30, max_halvings=8, maxit=500,
                xtol=1e-10):
        """One implicit Euler step with Newton in place on the device tensor u; returns
        (converged, stats).  On failure u is unchanged."""
        if not (isinstance(u, self.torch.Tensor) and u.device == self.device and u.dtype == self.torch.float64):
            raise TypeError("u must be a float64 tensor on the grid's device")
        o = L.NewtonOpts(int(max_newton), int(max_halvings), int(maxit), 0, float(atol), float(rtol),
                         float(lin_rtol), float(xtol))
        st = L.NewtonStats()
        status = self.lib.tpf_ie_step(self.handle, _ptr(u), float(tau), C.byref(o), C.byref(st), self._sptr())
        L.check(status, "tpf_ie_step", soft_ok=True)
        return status == TPF_OK, st.as_dict()

    def project_pressure(self, u, h_p=1e-6, rtol=1e-10, atol=0.0, lin_rtol=1e-10, max_newton=20, maxit=500):
        """Newton at fixed saturation onto the volume-balance constraint, in place on the
        device tensor u (pressure components only); returns (converged, stats)."""
        if not (isinstance(u, self.torch.Tensor) and u.device == self.device and u.dtype == self.torch.float64):
            raise TypeError("u must be a float64 tensor on the grid's device")
        o = L.NewtonOpts(int(max_newton), 0, int(maxit), 0, float(atol), float(rtol), float(lin_rtol))
        st = L.NewtonStats()
        status = self.lib.tpf_project_pressure(self.handle, _ptr(u), float(h_p), C.byref(o), C.byref(st),
                                               self._sptr())
        L.check(status, "tpf_project_pressure", soft_ok=True)
        return status == TPF_OK, st.as_dict()

    def set_coarse_graph(self, enable=True):
        """Replay the V-cycle's coarse levels as one captured HIP graph (or not)."""
        L.check(self.lib.tpf_set_coarse_graph(self.handle, int(bool(enable))), "tpf_set_coarse_graph")

    def set_line_pairs(self, max_lines=32768):
        """Line smoother: levels with fewer lines use two threads per line (identical results)."""
        L.check(self.lib.tpf_set_line_pairs(self.handle, int(max_lines)), "tpf_set_line_pairs")

    # -- inspection ------------------------------------------------------------------
    def level_dims(self, level):
        n = (C.c_int32 * 3)()
        L.check(self.lib.tpf_level_dims(self.handle, int(level), n), "tpf_level_dims")
        return tuple(int(v) for v in n)

    def matrix(self, level=0, precision="fp64"):
        torch = self.torch
        n = self.level_dims(level)
        Nl = n[0] * n[1] * n[2]
        dt = torch.float64 if precision == "fp64" else torch.float32
        out = torch.empty((self.nst, Nl, 4), dtype=dt, device=self.device)
        L.check(self.lib.tpf_copy_matrix(self.handle, int(level), PRECISIONS[precision], _ptr(out), self._sptr()),
                "tpf_copy_matrix")
        return out

    def spmv(self, x, level=0):
        n = self.level_dims(level)
        Nl = n[0] * n[1] * n[2]
        x = self._vec(x, 2 * Nl)
        y = self.empty(2 * Nl)
        L.check(self.lib.tpf_spmv(self.handle, int(level), _ptr(x), _ptr(y), self._sptr()), "tpf_spmv")
        return y

    def precondition(self, b):
        b = self._vec(b)
        x = self.empty()
        L.check(self.lib.tpf_precondition(self.handle, _ptr(b), _ptr(x), self._sptr()), "tpf_precondition")
        return x

    def pdmin(self):
        """p_dmin per vertex (Eq. pdmin): a float64 view of the arena at the address
        tpf_pdmin_ptr reports."""
        ptr = self.lib.tpf_pdmin_ptr(self.handle)
        off = int(ptr) - self.arena.data_ptr()
        if ptr is None or off < 0 or off % 8 or off + 8 * self.N > self.nbytes:
            raise RuntimeError("tpf_pdmin_ptr is outside the grid's arena")
        return self.arena[off:off + 8 * self.N].view(self.torch.float64)

    def coarse_inverse(self):
        n = self.level_dims(self.levels - 1)
        nc = 2 * n[0] * n[1] * n[2]
        out = self.torch.empty(nc * nc, dtype=self.torch.float64, device=self.device)
        L.check(self.lib.tpf_copy_coarse_inverse(self.handle, _ptr(out), self._sptr()), "tpf_copy_coarse_inverse")
        return out.reshape(nc, nc)  # row-major storage

    def profile_begin(self, max_launches=65536, classes=None):
        """Times every launch of the named kernel classes (all when None) with HIP events."""
        mask = 0
        for c in (classes or []):
            mask |= 1 << L.KERNEL_CLASSES.index(c)
        L.check(self.lib.tpf_profile_begin(self.handle, int(max_launches), mask), "tpf_profile_begin")

    def profile_end(self):
        arr = (L.KernelTime * len(L.KERNEL_CLASSES))()
        L.check(self.lib.tpf_profile_end(self.handle, arr), "tpf_profile_end")
        return {name: (arr[i].count, arr[i].total_ms) for i, name in enumerate(L.KERNEL_CLASSES)}

    def close(self):
        if getattr(self, "handle", None):
            # all of the grid's device work is on its stream: wait for it, then free
            self.stream.synchronize()
            self.lib.tpf_destroy_grid(self.handle)
            self.handle = None
            self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
