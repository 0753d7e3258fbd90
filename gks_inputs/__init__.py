"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates* meshes and initial cell averages.  It holds none
of the scheme's arithmetic (no geometry of the finite-volume method, no
reconstruction, no flux); both the CPU oracle and the HIP path consume the
arrays it returns, each with its own code.

Mesh family "jittered split squares" (JSS): an Nx x Ny lattice of squares,
each split into two counter-clockwise triangles along a seeded random
diagonal, with interior lattice vertices moved by a seeded uniform offset of
at most 0.2 of the local spacing in each direction.  Vertices on the box
boundary are never moved, so periodic identification and wall lines stay
exact.

Initial data are exact cell averages (up to rounding) of the analytic fields
of the paper's test cases, obtained with a collapsed (Duffy) tensor Gauss rule
on each triangle.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Mesh", "jss_mesh", "cell_average", "density_advection_ic",
    "density_advection_exact", "shock_vortex_ic", "cavity_ic",
    "prim_to_cons", "random_coefficients", "serving_specs", "serving_case", "serving_cells", "BC_NONE", "BC_SLIP",
    "BC_NOSLIP", "BC_INFLOW", "BC_OUTFLOW",
]

# Boundary-edge kinds (the value stored per boundary edge is an index into a
# per-mesh table of (kind, state) rows; kinds are fixed here).
BC_NONE = 0      # interior edge
BC_SLIP = 1      # inviscid reflecting wall
BC_NOSLIP = 2    # no-slip wall with a prescribed wall velocity (lid or fixed)
BC_INFLOW = 3    # supersonic inflow: fixed state, zero gradients
BC_OUTFLOW = 4   # extrapolation outflow


@dataclass
class Mesh:
    """Plain arrays describing a triangle mesh.

    xy       float64 [nv, 2]  vertex coordinates
    tri      int32   [nt, 3]  counter-clockwise vertex indices
    edge_tag int32   [nt, 3]  0 for an interior/periodic edge, else a 1-based
                              row of ``bc_table``; edge e runs from vertex
                              tri[t, e] to tri[t, (e + 1) % 3]
    periodic (px, py) and box lengths (Lx, Ly) for minimum-image unwrapping
    bc_table list of (kind, (rho, u, v, p)) rows for tagged edges; for a
             no-slip wall only (u, v), the wall velocity, is used
    """

    xy: np.ndarray
    tri: np.ndarray
    edge_tag: np.ndarray
    periodic: tuple
    L: tuple
    origin: tuple = (0.0, 0.0)
    bc_table: list = field(default_factory=list)
    nx: int = 0
    ny: int = 0

    @property
    def nt(self) -> int:
        return int(self.tri.shape[0])

    @property
    def nv(self) -> int:
        return int(self.xy.shape[0])

    def unwrapped_vertices(self) -> np.ndarray:
        """[nt, 3, 2] vertex coordinates, each triangle unwrapped about its
        first vertex by the minimum image (identity on non-periodic axes)."""
        v = self.xy[self.tri]                      # [nt, 3, 2]
        d = v - v[:, :1, :]
        for ax in range(2):
            if self.periodic[ax]:
                Lx = self.L[ax]
                d[..., ax] -= Lx * np.round(d[..., ax] / Lx)
        return v[:, :1, :] + d


def _lines(n: int, length: float, stretch: float) -> np.ndarray:
    s = np.arange(n + 1, dtype=np.float64) / n
    if stretch > 0.0:
        s = 0.5 * (1.0 + np.tanh(stretch * (2.0 * s - 1.0)) / math.tanh(stretch))
    return s * length


def jss_mesh(nx: int, ny: int, seed: int, Lx: float = 2.0, Ly: float = 2.0,
             periodic: bool = True, stretch: float = 0.0, jitter: float = 0.2,
             walls: tuple | None = None, origin=(0.0, 0.0)) -> Mesh:
    """Jittered split-square mesh with ``2 * nx * ny`` triangles.

    periodic  True: both axes periodic (no boundary edges); requires nx, ny >= 3
    stretch   tanh clustering strength toward both ends of each axis (0 = uniform)
    walls     for non-periodic meshes: ((kind, state) for x = x0, x = x1,
              y = y0, y = y1); default all slip walls
    Triangles are ordered square by square (row-major, x fastest), the lower
    triangle of each square first.
    """
    if periodic and (nx < 3 or ny < 3):
        raise ValueError("periodic JSS meshes need nx, ny >= 3")
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = _lines(nx, Lx, stretch) + origin[0]
    ys = _lines(ny, Ly, stretch) + origin[1]
    X, Y = np.meshgrid(xs, ys)                 # [ny+1, nx+1]
    P = np.stack([X, Y], axis=-1).copy()
    hx = np.diff(xs)
    hy = np.diff(ys)
    hloc_x = np.minimum(hx[:-1], hx[1:])       # interior vertex lines 1..nx-1
    hloc_y = np.minimum(hy[:-1], hy[1:])
    off = rng.uniform(-1.0, 1.0, (ny - 1, nx - 1, 2))
    P[1:ny, 1:nx, 0] += off[..., 0] * jitter * hloc_x[None, :]
    P[1:ny, 1:nx, 1] += off[..., 1] * jitter * hloc_y[:, None]
    diag = rng.integers(0, 2, (ny, nx))

    if periodic:
        xy = P[:ny, :nx].reshape(-1, 2).copy()

        def vid(i, j):
            return (j % ny) * nx + (i % nx)
    else:
        xy = P.reshape(-1, 2).copy()

        def vid(i, j):
            return j * (nx + 1) + i

    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    I = I.ravel()
    J = J.ravel()
    d = diag.ravel()
    v00 = vid(I, J)
    v10 = vid(I + 1, J)
    v11 = vid(I + 1, J + 1)
    v01 = vid(I, J + 1)
    lower = np.where(d[:, None] == 0, np.stack([v00, v10, v11], 1), np.stack([v00, v10, v01], 1))
    upper = np.where(d[:, None] == 0, np.stack([v00, v11, v01], 1), np.stack([v10, v11, v01], 1))
    tri = np.empty((2 * nx * ny, 3), dtype=np.int32)
    tri[0::2] = lower
    tri[1::2] = upper

    edge_tag = np.zeros_like(tri)
    bc_table = []
    if not periodic:
        if walls is None:
            walls = ((BC_SLIP, None),) * 4
        bc_table = [(int(k), None if s is None else tuple(float(q) for q in s)) for k, s in walls]
        # Tag every triangle edge whose two vertices lie on the same box side.
        vx = xy[tri][..., 0]
        vy = xy[tri][..., 1]
        x0, x1 = xs[0], xs[-1]
        y0, y1 = ys[0], ys[-1]
        for e in range(3):
            a, b = e, (e + 1) % 3
            for side, (coord, val) in enumerate(((vx, x0), (vx, x1), (vy, y0), (vy, y1))):
                on = (coord[:, a] == val) & (coord[:, b] == val)
                edge_tag[on, e] = side + 1

    mesh = Mesh(xy=xy, tri=tri, edge_tag=edge_tag, periodic=(periodic, periodic),
                L=(float(Lx), float(Ly)), origin=(float(origin[0]), float(origin[1])),
                bc_table=bc_table, nx=nx, ny=ny)
    v = mesh.unwrapped_vertices()
    area2 = ((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1])
             - (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1]))
    if not np.all(area2 > 0):
        raise RuntimeError("JSS generator produced a non-positive triangle")
    return mesh


# --- quadrature used only to form exact initial cell averages -------------

def _duffy_rule(order: int = 8):
    g, w = np.polynomial.legendre.leggauss(order)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    s, t = np.meshgrid(g, g, indexing="ij")
    ws, wt = np.meshgrid(w, w, indexing="ij")
    # (s, t) in the unit square -> barycentric (l1, l2) = (s, t (1 - s));
    # the Jacobian of the collapse is (1 - s); the reference triangle has area 1/2.
    l1 = s.ravel()
    l2 = (t * (1.0 - s)).ravel()
    wq = (ws * wt * (1.0 - s)).ravel() * 2.0  # weights sum to 1 (area fraction)
    return l1, l2, wq


def cell_average(mesh: Mesh, fn, order: int = 8) -> np.ndarray:
    """Average over each triangle of ``fn(x, y) -> [k, ...]`` arrays.

    fn receives point arrays of shape [nt, q] and returns an array of shape
    [m, nt, q]; the result has shape [m, nt].
    """
    l1, l2, wq = _duffy_rule(order)
    v = mesh.unwrapped_vertices()
    x = v[:, 0, 0, None] + l1[None] * (v[:, 1, 0] - v[:, 0, 0])[:, None] + l2[None] * (v[:, 2, 0] - v[:, 0, 0])[:, None]
    y = v[:, 0, 1, None] + l1[None] * (v[:, 1, 1] - v[:, 0, 1])[:, None] + l2[None] * (v[:, 2, 1] - v[:, 0, 1])[:, None]
    vals = np.asarray(fn(x, y), dtype=np.float64)
    return np.einsum("mtq,q->mt", vals, wq)


def prim_to_cons(rho, u, v, p, gamma):
    rho = np.asarray(rho, dtype=np.float64)
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def density_advection_ic(mesh: Mesh, gamma: float = 1.4, amp: float = 0.2,
                         u: float = 1.0, v: float = 1.0, p: float = 1.0,
                         t: float = 0.0) -> np.ndarray:
    """Cell averages [4, nt] of the density-perturbation advection field.

    The field is rho(x, y, t) = 1 + amp * sin(pi * ((x - u t) + (y - v t))),
    with constant velocity and pressure, i.e. the exact solution of the
    density-perturbation advection test at time t (paper section 4.1, in its
    two-dimensional diagonal form on the periodic square [0, 2]^2).
    """
    def rho_fn(x, y):
        return (1.0 + amp * np.sin(np.pi * ((x - u * t) + (y - v * t))))[None]

    rho = cell_average(mesh, rho_fn)[0]
    W = np.empty((4, mesh.nt))
    W[0] = rho
    W[1] = rho * u
    W[2] = rho * v
    W[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return W


def density_advection_exact(mesh: Mesh, t: float, **kw) -> np.ndarray:
    return density_advection_ic(mesh, t=t, **kw)


def acoustic_pulse_ic(mesh: Mesh, gamma: float = 1.4, amp: float = 0.01, half_width: float = 0.04,
                      center=(0.5, 0.5)) -> np.ndarray:
    """Cell averages [4, nt] of the acoustic pressure pulse (paper section
    4.4): rho = 1, u = v = 0, p = 1 + amp * exp(-alpha eta^2) with
    eta = |x - center| and alpha = ln 2 / half_width^2."""
    alpha = math.log(2.0) / half_width ** 2
    cx, cy = center

    def p_fn(x, y):
        return (1.0 + amp * np.exp(-alpha * ((x - cx) ** 2 + (y - cy) ** 2)))[None]

    p = cell_average(mesh, p_fn)[0]
    rho = np.ones_like(p)
    return prim_to_cons(rho, np.zeros_like(p), np.zeros_like(p), p, gamma)


def shock_vortex_states(gamma: float = 1.4, mach: float = 1.1):
    """Pre-shock (rho, u, v, p) = (1, Ma sqrt(gamma), 0, 1) and the post-shock
    state from the Rankine-Hugoniot relations of a stationary normal shock."""
    M2 = mach * mach
    u1 = mach * math.sqrt(gamma)
    r2 = (gamma + 1.0) * M2 / ((gamma - 1.0) * M2 + 2.0)
    p2 = 1.0 + 2.0 * gamma / (gamma + 1.0) * (M2 - 1.0)
    return (1.0, u1, 0.0, 1.0), (r2, u1 / r2, 0.0, p2)


def shock_vortex_ic(mesh: Mesh, gamma: float = 1.4, mach: float = 1.1,
                    x_shock: float = 0.5, kappa: float = 0.3, mu_v: float = 0.204,
                    rc: float = 0.05, center=(0.25, 0.5)) -> np.ndarray:
    """Shock-vortex initial cell averages [4, nt] (paper section 4.6).

    Cells whose centroid lies left of the shock get the exact average of the
    pre-shock state with the isentropic vortex superposed; the others get the
    uniform post-shock state.  The vortex temperature perturbation is read as a
    scalar (the paper's stray direction vector on dT is dropped).
    """
    left, right = shock_vortex_states(gamma, mach)

    def fn(x, y):
        dx = x - center[0]
        dy = y - center[1]
        r = np.sqrt(dx * dx + dy * dy)
        eta = r / rc
        th = np.arctan2(dy, dx)
        amp = kappa * eta * np.exp(mu_v * (1.0 - eta * eta))
        du = amp * np.sin(th)
        dv = -amp * np.cos(th)
        dT = -(gamma - 1.0) * kappa * kappa / (4.0 * mu_v * gamma) * np.exp(2.0 * mu_v * (1.0 - eta * eta))
        T = left[3] / left[0] + dT
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        return prim_to_cons(rho, left[1] + du, left[2] + dv, p, gamma)

    v = mesh.unwrapped_vertices()
    cx = v[..., 0].mean(axis=1)
    cy = v[..., 1].mean(axis=1)
    Wl = prim_to_cons(np.full(mesh.nt, left[0]), left[1], left[2], left[3], gamma)
    # the perturbation is below 1e-17 beyond r = 14 rc: average only near the vortex
    near = np.hypot(cx - center[0], cy - center[1]) < 14.0 * rc + 2.0 * np.sqrt(
        np.max(np.abs(v[..., 0] - cx[:, None]) + np.abs(v[..., 1] - cy[:, None]), axis=1) ** 2)
    if np.any(near):
        sub = Mesh(xy=mesh.xy, tri=mesh.tri[near], edge_tag=mesh.edge_tag[near], periodic=mesh.periodic,
                   L=mesh.L, origin=mesh.origin, bc_table=mesh.bc_table)
        Wl[:, near] = cell_average(sub, fn)
    Wr = prim_to_cons(np.full(mesh.nt, right[0]), right[1], right[2], right[3], gamma)
    return np.where((cx < x_shock)[None], Wl, Wr)


def cavity_ic(mesh: Mesh, gamma: float = 1.4, mach: float = 0.15) -> np.ndarray:
    """Fluid at rest: rho = 1, p = 1 / (gamma Ma^2) so a unit lid speed has Mach Ma."""
    p = 1.0 / (gamma * mach * mach)
    return prim_to_cons(np.ones(mesh.nt), 0.0, 0.0, p, gamma)


def serving_specs(n_requests: int = 2000, rate: float = 40.0, seed: int = 5, nt_range=(2e3, 2e5),
                  steps_range=(50, 500)) -> list:
    """Seeded request stream: Poisson arrivals at `rate` per second; each
    request is density advection or shock-vortex (50/50) on a JSS mesh whose
    triangle count is log-uniform in nt_range, runs a uniform integer number
    of steps in steps_range, in the FP64 or mixed form (50/50)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    kinds = rng.integers(0, 2, n_requests)
    nts = np.exp(rng.uniform(np.log(nt_range[0]), np.log(nt_range[1]), n_requests))
    steps = rng.integers(steps_range[0], steps_range[1] + 1, n_requests)
    mixed = rng.integers(0, 2, n_requests)
    seeds = rng.integers(1, 2 ** 31 - 1, n_requests)
    return [{"rid": i, "kind": "advection" if kinds[i] == 0 else "shock_vortex", "nt": float(nts[i]),
             "steps": int(steps[i]), "mixed": bool(mixed[i]), "seed": int(seeds[i]), "arrival": float(arrivals[i])}
            for i in range(n_requests)]


def serving_cells(spec: dict) -> int:
    """Triangles of the mesh serving_case builds for spec (without building it)."""
    if spec["kind"] == "advection":
        n = max(3, int(round(np.sqrt(spec["nt"] / 2.0))))
        return 2 * n * n
    ny = max(2, int(round(np.sqrt(spec["nt"] / 4.0))))
    return 4 * ny * ny


def serving_case(spec: dict):
    """(mesh, W0) of one request of serving_specs."""
    if spec["kind"] == "advection":
        n = max(3, int(round(np.sqrt(spec["nt"] / 2.0))))
        m = jss_mesh(n, n, spec["seed"])
        return m, density_advection_ic(m)
    ny = max(2, int(round(np.sqrt(spec["nt"] / 4.0))))
    left, _ = shock_vortex_states()
    walls = ((BC_INFLOW, left), (BC_OUTFLOW, None), (BC_SLIP, None), (BC_SLIP, None))
    m = jss_mesh(2 * ny, ny, spec["seed"], Lx=2.0, Ly=1.0, periodic=False, walls=walls)
    return m, shock_vortex_ic(m)


def random_coefficients(nt: int, seed: int, scale: float = 0.05) -> np.ndarray:
    """Seeded reconstruction coefficients [4, 5, nt] for flux-only tests
    (independent of any solve)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, (4, 5, nt))
