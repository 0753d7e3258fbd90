"""Oracle geometry: cells, faces and face Gauss points.

Follows section 2.1 (Eq. fvm3: cell measure, interface measure S; Eq.
fluxgauss: Gauss quadrature along each interface) and section 3.1 (Eq. RCP:
the basis is centred at the cell centroid and scaled by h_i; Eq. h:
h_i = max(circumradius, sqrt(area))).

Face convention (shared by contract with the library, not by code): face f
is emitted while scanning triangles t = 0..nt-1 and their local edges
e = 0, 1, 2 (edge e runs from vertex e to vertex e+1 mod 3), whenever the
triangle across the edge has a larger index or the edge lies on the
boundary.  The owner is t, the unit normal points out of the owner, and the
two Gauss points are m -/+ (b - a) / (2 sqrt(3)) for edge a -> b, each with
weight S / 2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Geometry:
    nt: int
    area: np.ndarray        # [nt]
    cen: np.ndarray         # [nt, 2] centroid in the triangle's unwrapped frame
    Ixx: np.ndarray         # [nt] area-mean of (x - cx)^2
    Ixy: np.ndarray         # [nt] area-mean of (x - cx)(y - cy)
    Iyy: np.ndarray         # [nt]
    h: np.ndarray           # [nt] length scale of Eq. h
    boundary_cell: np.ndarray  # [nt] bool, cell has a boundary edge
    # faces
    own: np.ndarray         # [nf]
    nbr: np.ndarray         # [nf] neighbour cell, -1 on the boundary
    tag: np.ndarray         # [nf] boundary tag (0 interior)
    normal: np.ndarray      # [nf, 2] unit normal out of the owner
    S: np.ndarray           # [nf] face length
    gp: np.ndarray          # [nf, 2, 2] Gauss points (owner frame)
    periodic: tuple
    L: tuple

    @property
    def nf(self) -> int:
        return int(self.own.shape[0])

    def minimg(self, d: np.ndarray) -> np.ndarray:
        """Minimum-image displacement on periodic axes; d has trailing dim 2."""
        d = np.array(d, dtype=np.float64, copy=True)
        for ax in range(2):
            if self.periodic[ax]:
                d[..., ax] -= self.L[ax] * np.round(d[..., ax] / self.L[ax])
        return d


def triangle_geometry(v: np.ndarray):
    """Area, centroid, central second moments (per unit area) and
    circumradius of triangles v [nt, 3, 2].

    The second moments use the exact identity for a triangle: the covariance
    of the uniform distribution equals (1/12) sum_k (v_k - c)(v_k - c)^T.
    """
    x = v[..., 0]
    y = v[..., 1]
    area = 0.5 * ((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    cx = x.mean(axis=1)
    cy = y.mean(axis=1)
    dx = x - cx[:, None]
    dy = y - cy[:, None]
    Ixx = (dx * dx).sum(axis=1) / 12.0
    Ixy = (dx * dy).sum(axis=1) / 12.0
    Iyy = (dy * dy).sum(axis=1) / 12.0
    a = np.hypot(x[:, 1] - x[:, 0], y[:, 1] - y[:, 0])
    b = np.hypot(x[:, 2] - x[:, 1], y[:, 2] - y[:, 1])
    c = np.hypot(x[:, 0] - x[:, 2], y[:, 0] - y[:, 2])
    rad = a * b * c / (4.0 * area)
    return area, np.stack([cx, cy], axis=1), Ixx, Ixy, Iyy, rad


def build_geometry(mesh) -> Geometry:
    """Geometry of a ``gks_inputs.Mesh`` (section 2.1 and section 3.1)."""
    v = mesh.unwrapped_vertices()
    nt = v.shape[0]
    area, cen, Ixx, Ixy, Iyy, rad = triangle_geometry(v)
    if np.any(area <= 0.0):
        raise ValueError("triangles must be counter-clockwise and non-degenerate")
    h = np.maximum(rad, np.sqrt(area))

    # edge -> (triangle, local edge) map through sorted vertex pairs
    tri = mesh.tri
    edges = {}
    for t in range(nt):
        for e in range(3):
            a, b = int(tri[t, e]), int(tri[t, (e + 1) % 3])
            key = (a, b) if a < b else (b, a)
            edges.setdefault(key, []).append((t, e))
    for key, lst in edges.items():
        if len(lst) > 2:
            raise ValueError("non-manifold edge %r" % (key,))

    own, nbr, tag, loc = [], [], [], []
    for t in range(nt):
        for e in range(3):
            a, b = int(tri[t, e]), int(tri[t, (e + 1) % 3])
            key = (a, b) if a < b else (b, a)
            lst = edges[key]
            if len(lst) == 1:
                own.append(t); nbr.append(-1); tag.append(int(mesh.edge_tag[t, e])); loc.append(e)
                if mesh.edge_tag[t, e] == 0:
                    raise ValueError("open edge without a boundary tag")
            else:
                other = lst[0][0] if lst[0][0] != t else lst[1][0]
                if other > t:
                    own.append(t); nbr.append(other); tag.append(0); loc.append(e)
    own = np.array(own, dtype=np.int64)
    nbr = np.array(nbr, dtype=np.int64)
    tag = np.array(tag, dtype=np.int64)
    loc = np.array(loc, dtype=np.int64)

    pa = v[own, loc]
    pb = v[own, (loc + 1) % 3]
    d = pb - pa
    S = np.hypot(d[:, 0], d[:, 1])
    normal = np.stack([d[:, 1], -d[:, 0]], axis=1) / S[:, None]
    mid = 0.5 * (pa + pb)
    off = d / (2.0 * np.sqrt(3.0))
    gp = np.stack([mid - off, mid + off], axis=1)

    bcell = np.zeros(nt, dtype=bool)
    bcell[own[nbr < 0]] = True
    return Geometry(nt=nt, area=area, cen=cen, Ixx=Ixx, Ixy=Ixy, Iyy=Iyy, h=h,
                    boundary_cell=bcell, own=own, nbr=nbr, tag=tag, normal=normal,
                    S=S, gp=gp, periodic=tuple(mesh.periodic), L=tuple(mesh.L))
