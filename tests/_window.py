"""Sub-grid windows of a scenario, for oracle checks of sampled rows of full-size grids.

A window keeps the cells, vertex data and state of a box of vertices of the full grid.
A row of the box-method residual or stage matrix at vertex v depends on the cells
adjacent to v and on the p_dmin / reference medium of the vertices of those cells,
i.e. on cells at most two cells away from v: on a window reaching two cells past v
(clipped at the domain boundary) the oracle reproduces the full grid's row exactly.
The window's own cut faces are no-flux boundaries, which only changes rows of the
window's boundary vertices.  Injection patches are kept, translated, on the faces the
window shares with the domain.  No arithmetic of the method is done here.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np


def window(scn, lo, hi, u=None, levels=1):
    """Vertices lo[a]..hi[a] (inclusive) of each axis; u: full-grid state (N, 2)."""
    dim = scn.dim
    lo = [int(lo[a]) if a < dim else 0 for a in range(3)]
    hi = [int(hi[a]) if a < dim else 0 for a in range(3)]
    n = tuple(hi[a] - lo[a] + 1 for a in range(3))
    sp = scn.spacing
    extent = tuple((n[a] - 1) * sp[a] if a < dim else scn.extent[a] for a in range(3))
    vs = (slice(lo[2], hi[2] + 1), slice(lo[1], hi[1] + 1), slice(lo[0], hi[0] + 1))
    cs = (slice(lo[2], hi[2]) if dim == 3 else slice(0, 1), slice(lo[1], hi[1]), slice(lo[0], hi[0]))

    def cell(a):
        return np.ascontiguousarray(np.asarray(a).reshape(scn.cell_shape)[cs]).ravel()

    def vert(a):
        return np.ascontiguousarray(np.asarray(a).reshape(scn.vert_shape)[vs]).ravel()

    def vert2(a):
        return np.ascontiguousarray(np.asarray(a).reshape(scn.vert_shape + (2,))[vs]).reshape(-1, 2)

    origin = [lo[a] * sp[a] for a in range(3)]
    patches = []
    for p in scn.patches:
        a = p.axis
        if (p.side == 1 and hi[a] != scn.n[a] - 1) or (p.side == 0 and lo[a] != 0):
            continue
        others = [b for b in range(dim) if b != a]
        plo = list(p.lo)
        phi = list(p.hi)
        for k, b in enumerate(others):
            plo[k] = p.lo[k] - origin[b]
            phi[k] = p.hi[k] - origin[b]
        patches.append(replace(p, lo=tuple(plo), hi=tuple(phi)))
    return replace(scn, name=f"{scn.name}[{lo}:{hi}]", n=n, extent=extent, perm=cell(scn.perm),
                   poro=cell(scn.poro), entry_p=cell(scn.entry_p), bc_lambda=cell(scn.bc_lambda),
                   dir_mask=vert(scn.dir_mask), dir_value=vert2(scn.dir_value), patches=patches,
                   u0=vert2(scn.u0 if u is None else u), levels=levels,
                   vertex_source=None if scn.vertex_source is None else vert2(scn.vertex_source))


def row_window(scn, v, reach=2):
    """Window bounds reaching `reach` cells past vertex v (a 3-tuple) on every axis."""
    lo = [max(v[a] - reach, 0) if a < scn.dim else 0 for a in range(3)]
    hi = [min(v[a] + reach, scn.n[a] - 1) if a < scn.dim else 0 for a in range(3)]
    return lo, hi


def local_index(lo, hi, v):
    nx, ny = hi[0] - lo[0] + 1, hi[1] - lo[1] + 1
    return (v[0] - lo[0]) + nx * ((v[1] - lo[1]) + ny * (v[2] - lo[2]))


def sample_vertices(scn, n_random, seed):
    """Corners, edge and face midpoints, vertices on the injection patch edges and next
    to the Dirichlet faces, and n_random seeded interior vertices."""
    nx, ny, nz = scn.n
    dim = scn.dim
    zs = (0, nz // 2, nz - 1) if dim == 3 else (0,)
    out = set()
    for z in zs:
        for y in (0, ny // 2, ny - 1):
            for x in (0, 1, nx // 2, nx - 2, nx - 1):
                out.add((x, y, z))
    sp = scn.spacing
    for p in scn.patches:
        others = [b for b in range(dim) if b != p.axis]
        fixed = 0 if p.side == 0 else scn.n[p.axis] - 1
        for k, b in enumerate(others):
            for edge in (p.lo[k], p.hi[k]):
                i = int(round(edge / sp[b]))
                for di in (-1, 0, 1):
                    v = [nx // 2, ny // 2, nz // 2 if dim == 3 else 0]
                    v[p.axis] = fixed
                    v[b] = min(max(i + di, 0), scn.n[b] - 1)
                    out.add(tuple(v))
    rng = np.random.default_rng(seed)
    for _ in range(n_random):
        out.add((int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz)) if dim == 3 else 0))
    return sorted(out)


def vertex_index(scn, v):
    return v[0] + scn.n[0] * (v[1] + scn.n[1] * v[2])
