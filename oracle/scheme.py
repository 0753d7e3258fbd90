"""Oracle finite-volume step: Gauss-point states, face fluxes, update.

* Gauss-point states evaluate the cell quadratic of Eq. quadRCP and its
  derivatives at the two Gauss points of each face (Eq. fluxgauss) and rotate
  them into the face frame (normal, tangent).
* The face flux is sum_l (S/2) F_l of the time-integrated Gauss-point fluxes
  (two-point Gauss-Legendre rule: the paper leaves the number of points
  open), rotated back.
* The update is Eq. fvm3: W_i <- W_i - (1/|Omega_i|) sum_f s_if F_f with
  s = +1 for the owner and -1 for the neighbour.
* The time step (the paper gives none) is
  dt = CFL min_i |Omega_i| / sum_{f in i} S_f (|U_i . n_f| + c_i).
* Boundary faces use a ghost state: walls mirror the interior one-sided
  polynomial at the Gauss point, inflow takes a fixed state, and outflow
  (transmissive) takes the boundary cell's average with zero derivatives;
  boundary faces add no CLS rows.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cls as cls_mod
from . import kinetic
from .mesh import Geometry, build_geometry

BC_SLIP, BC_NOSLIP, BC_INFLOW, BC_OUTFLOW = 1, 2, 3, 4


@dataclass
class Params:
    gamma: float = 1.4
    mu: float = 0.0
    eps: float = 0.01          # coefficient of dt in the inviscid collision time
    cls_w: float = 0.3
    cfl: float = 0.5
    exact_time: bool = False
    fallback: bool = False     # non-physical Gauss-point state -> cell average
    reading: str = "G"
    all_quadratic: bool = False
    solve: str = "auto"        # CLS solve: "direct", "cg", or "auto" (direct up to
                               # cls.DIRECT_MAX_UNKNOWNS unknowns, CG beyond)


def gp_states(geo: Geometry, W, X, cells, pts):
    """Value, gradient and Hessian in (x, y) of the cell polynomials of
    ``cells`` [m] at points ``pts`` [m, 2]; returns (Q, Qx, Qy, Qxx, Qxy, Qyy),
    each [4, m]."""
    h = geo.h[cells]
    d = geo.minimg(pts - geo.cen[cells]) / h[:, None]
    dx, dy = d[:, 0], d[:, 1]
    phi = np.stack([dx, dy,
                    0.5 * (dx * dx - geo.Ixx[cells] / h ** 2),
                    dx * dy - geo.Ixy[cells] / h ** 2,
                    0.5 * (dy * dy - geo.Iyy[cells] / h ** 2)])
    Xc = X[:, :, cells]                                   # [4, 5, m]
    Q = W[:, cells] + np.einsum("vlm,lm->vm", Xc, phi)
    Qx = (Xc[:, 0] + Xc[:, 2] * dx + Xc[:, 3] * dy) / h
    Qy = (Xc[:, 1] + Xc[:, 3] * dx + Xc[:, 4] * dy) / h
    Qxx = Xc[:, 2] / h ** 2
    Qxy = Xc[:, 3] / h ** 2
    Qyy = Xc[:, 4] / h ** 2
    return Q, Qx, Qy, Qxx, Qxy, Qyy


def to_local(vec, nx, ny):
    """Rotate the momentum pair of conserved vectors [4, m] into (n, t)."""
    out = vec.copy()
    out[1] = vec[1] * nx + vec[2] * ny
    out[2] = -vec[1] * ny + vec[2] * nx
    return out


def local_derivs(Q, Qx, Qy, Qxx, Qxy, Qyy, nx, ny):
    """States and derivatives along n = (nx, ny) and t = (-ny, nx)."""
    tx, ty = -ny, nx
    Wn = nx * Qx + ny * Qy
    Wt = tx * Qx + ty * Qy
    Wnn = nx * nx * Qxx + 2.0 * nx * ny * Qxy + ny * ny * Qyy
    Wnt = nx * tx * Qxx + (nx * ty + ny * tx) * Qxy + ny * ty * Qyy
    Wtt = tx * tx * Qxx + 2.0 * tx * ty * Qxy + ty * ty * Qyy
    W = to_local(Q, nx, ny)
    d = {key: to_local(val, nx, ny) for key, val in
         (("n", Wn), ("t", Wt), ("nn", Wnn), ("nt", Wnt), ("tt", Wtt))}
    return W, d


def physical(W, gamma):
    return (W[0] > 0.0) & (kinetic.pressure(W, gamma) > 0.0)


def ghost(WL, dL, kind, state, gamma, nx, ny, Wc):
    """Ghost state and derivatives (face frame) beyond a boundary face.

    Walls mirror the interior polynomial across the face line, so each ghost
    derivative picks up (-1) per normal differentiation, combined with a
    linear map of the conserved variables: slip reflects the normal momentum;
    no-slip sets the ghost velocity to 2 U_wall - U with even density and
    pressure, which is linear in (rho, rho U, E).  Inflow uses the fixed
    state with zero derivatives (the kinetic flux then takes from it only
    what enters).  Outflow uses Wc, the boundary cell's average in the face
    frame, with zero derivatives: zeroth-order extrapolation.  A ghost that
    copied the interior Gauss-point state would make the face flux purely
    one-sided, so a characteristic entering through a subsonic outflow would
    be taken downwind; the linearised step then grows at the boundary.
    """
    m = WL.shape[1]
    if kind in (BC_SLIP, BC_NOSLIP):
        Lm = np.zeros((4, 4, m))
        Lm[0, 0] = 1.0
        Lm[3, 3] = 1.0
        if kind == BC_SLIP:
            Lm[1, 1] = -1.0
            Lm[2, 2] = 1.0
        else:
            uw, vw = state[1], state[2]
            wn = uw * nx + vw * ny
            wt = -uw * ny + vw * nx
            Lm[1, 0] = 2.0 * wn
            Lm[1, 1] = -1.0
            Lm[2, 0] = 2.0 * wt
            Lm[2, 2] = -1.0
            Lm[3, 0] = 2.0 * (wn * wn + wt * wt)
            Lm[3, 1] = -2.0 * wn
            Lm[3, 2] = -2.0 * wt
        ap = lambda q: np.einsum("abm,bm->am", Lm, q)
        WR = ap(WL)
        dR = {"n": -ap(dL["n"]), "t": ap(dL["t"]), "nn": ap(dL["nn"]),
              "nt": -ap(dL["nt"]), "tt": ap(dL["tt"])}
        return WR, dR
    if kind == BC_INFLOW:
        rho, u, v, p = state
        Wg = np.array([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])
        WR = to_local(np.repeat(Wg[:, None], m, axis=1), nx, ny)
        dR = {key: np.zeros((4, m)) for key in dL}
        return WR, dR
    if kind == BC_OUTFLOW:
        return Wc.copy(), {key: np.zeros_like(val) for key, val in dL.items()}
    raise ValueError("unknown boundary kind %r" % (kind,))


class NonPhysical(RuntimeError):
    pass


def face_fluxes(geo: Geometry, W, X, dt, prm: Params, bc_table=(), counters=None, faces=None):
    """Time-integrated face fluxes F [4, nf] (x-y frame, owner -> neighbour),
    or F [4, len(faces)] for a subset of faces."""
    fs = np.arange(geo.nf) if faces is None else np.asarray(faces)
    own, nbr, tag = geo.own[fs], geo.nbr[fs], geo.tag[fs]
    nfs = fs.size
    F = np.zeros((4, nfs))
    nx, ny = geo.normal[fs, 0], geo.normal[fs, 1]
    inner = nbr >= 0
    for g in range(2):
        pts = geo.gp[fs, g]
        Q = gp_states(geo, W, X, own, pts)
        WL, dL = local_derivs(*Q, nx, ny)
        WR = np.empty_like(WL)
        dR = {key: np.empty_like(val) for key, val in dL.items()}
        fi = np.nonzero(inner)[0]
        if fi.size:
            Qr = gp_states(geo, W, X, nbr[fi], pts[fi])
            wr, dr = local_derivs(*Qr, nx[fi], ny[fi])
            WR[:, fi] = wr
            for key in dR:
                dR[key][:, fi] = dr[key]
        for side_W, side_d, cells, sel in ((WL, dL, own, np.arange(nfs)), (WR, dR, nbr, fi)):
            ok = physical(side_W[:, sel], prm.gamma)
            if not np.all(ok):
                bad = sel[~ok]
                if counters is not None:
                    counters["nonphys"] = counters.get("nonphys", 0) + int(bad.size)
                if not prm.fallback:
                    raise NonPhysical("non-physical reconstructed state at %d Gauss points" % bad.size)
                side_W[:, bad] = to_local(W[:, cells[bad]], nx[bad], ny[bad])
                for key in side_d:
                    side_d[key][:, bad] = 0.0
        for row, (kind, state) in enumerate(bc_table, start=1):
            fb = np.nonzero((~inner) & (tag == row))[0]
            if fb.size:
                Wc = to_local(W[:, own[fb]], nx[fb], ny[fb])
                wg, dg = ghost(WL[:, fb], {key: val[:, fb] for key, val in dL.items()},
                               kind, state, prm.gamma, nx[fb], ny[fb], Wc)
                WR[:, fb] = wg
                for key in dR:
                    dR[key][:, fb] = dg[key]
        Fl = kinetic.gp_flux(WL, dL, WR, dR, dt, prm.gamma, prm.mu, prm.eps, prm.exact_time)
        # rotate the momentum back to (x, y)
        Fx = Fl.copy()
        Fx[1] = Fl[1] * nx - Fl[2] * ny
        Fx[2] = Fl[1] * ny + Fl[2] * nx
        F += 0.5 * geo.S[fs] * Fx
    return F


def update(geo: Geometry, W, F):
    """Eq. fvm3 with F already integrated over the step and the face."""
    dW = np.zeros_like(W)
    for v in range(4):
        np.add.at(dW[v], geo.own, -F[v])
        inner = geo.nbr >= 0
        np.add.at(dW[v], geo.nbr[inner], F[v, inner])
    return W + dW / geo.area[None]


def cfl_dt(geo: Geometry, W, prm: Params):
    rho = W[0]
    u = W[1] / rho
    v = W[2] / rho
    p = (prm.gamma - 1.0) * (W[3] - 0.5 * rho * (u * u + v * v))
    c = np.sqrt(prm.gamma * p / rho)
    den = np.zeros(geo.nt)
    for cells in (geo.own, geo.nbr):
        m = cells >= 0
        cc = cells[m]
        un = np.abs(u[cc] * geo.normal[m, 0] + v[cc] * geo.normal[m, 1])
        np.add.at(den, cc, geo.S[m] * (un + c[cc]))
    return prm.cfl * float(np.min(geo.area / den))


class Solver:
    """Holds the geometry and the factorised CLS system of one mesh."""

    def __init__(self, mesh, prm: Params | None = None):
        self.mesh = mesh
        self.prm = prm or Params()
        self.geo = build_geometry(mesh)
        self.k = cls_mod.cell_orders(self.geo, self.prm.all_quadratic)
        self.K, self.pairs = cls_mod.assemble(self.geo, self.k, self.prm.cls_w, self.prm.reading)
        self._lu = None
        self.bc_table = mesh.bc_table
        self.counters = {}

    def rhs(self, W):
        return cls_mod.rhs(self.geo, self.pairs, W)

    def reconstruct(self, W):
        R = self.rhs(W)
        nt = self.geo.nt
        mode = self.prm.solve
        if mode == "auto":
            mode = "direct" if 5 * nt <= cls_mod.DIRECT_MAX_UNKNOWNS or self.prm.reading != "G" else "cg"
        if mode == "cg":
            return cls_mod.solve_cg(self.K, R)
        b = R.reshape(4, 5 * nt).T
        if self._lu is None:
            self._lu = cls_mod.factorize(self.K, spd=self.prm.reading == "G")
        Xf = self._lu.solve(b)
        return np.ascontiguousarray(Xf.T.reshape(4, nt, 5).transpose(0, 2, 1))

    def flux(self, W, X, dt, faces=None):
        return face_fluxes(self.geo, W, X, dt, self.prm, self.bc_table, self.counters, faces)

    def step(self, W, dt=None):
        if dt is None or dt <= 0:
            dt = cfl_dt(self.geo, W, self.prm)
        X = self.reconstruct(W)
        F = self.flux(W, X, dt)
        return update(self.geo, W, F), dt

    def run(self, W, steps, dt=None):
        t = 0.0
        for _ in range(steps):
            W, d = self.step(W, dt)
            t += d
        return W, t
