"""Oracle: DWBAP limiter and shock detector for the reconstruction.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and
bench.py's CPU-baseline leg, never by the library.

Follows section 3.3 of the paper: the limited value is the inverse of a
biased function (arctan) applied to a weighted mean of the biased candidates
(Eq. DWBAP); the weights are inverse powers of the mean distance between a
candidate's centroid and the cell's face centroids, with an exponent S that
falls as the local pressure variation grows (Eqs. DWBAP_w, DWBAP_S,
epsilon = 1e-8); a cell is limited only where the shock indicator IS_i
reaches 1 (Eqs. ISD1, ISD2).

The paper leaves several points open; the readings taken (the library takes
the same ones):
  L1  Each conserved variable is limited separately, one derivative at a
      time: u_x, u_y, u_xx, u_xy, u_yy at the centroid (the coefficients
      X1..X5 divided by h_i and h_i^2).
  L2  Hierarchical candidates (highest derivatives first).  j = 0 is always
      the cell's own value.  Second derivatives: j = 1..J are the face
      neighbours' second derivatives.  First derivatives: candidate j is the
      gradient of the plane through the cell averages, at the centroids, of
      the remainder u - q_i, where q_i is cell i's quadratic part with its
      limited second derivatives, taken over cell i and the neighbour pair
      (j, j+1), neighbours taken in the cell's local-edge order
      (counter-clockwise, boundary edges skipped, cyclic; minimum image on
      periodic axes); a pair's candidate carries the mean of its two
      neighbours' weights, so the result does not depend on where the cycle
      starts.  The remainder is linear for quadratic data, so these
      candidates are exact there; across a jump the pairs on the smooth side
      give small slopes.  Cells with fewer than three face neighbours (at a
      boundary) take instead, per neighbour, the gradient along the
      neighbour's direction alone, rem_j d_j / |d_j|^2: the plane through a
      wall cell and its two neighbours would turn a jump between them into
      a spurious wall-normal slope (it made the Sod tube's wall cells blow
      up, where the directional candidates keep them bounded).
      (Derivatives of the neighbours' own polynomials would not do: the
      compact least-squares reconstruction is global, and near a jump the
      neighbours on the smooth side carry large slopes too.)
  L3  The biased function acts on the derivative values themselves, as the
      equation is written (the paper's test cases are dimensionless): across
      a discontinuity derivatives of order jump/h and jump/h^2 fall where
      arctan saturates, so outlying candidates are compressed, while small
      smooth-flow derivatives are averaged almost linearly.
  L4  Distances are measured in units of h_i; r_0 is cell i's centroid, r_j
      neighbour j's, r_m the midpoints of cell i's J faces shared with a
      neighbour.
  L5  chi = sigma / mean of the J neighbours' cell-average pressures, sigma
      their population standard deviation.
  L6  The indicator uses the density; u_j(r_i) is neighbour j's
      reconstructed density at cell i's centroid; k_i = 2 (k_i = 1 for cells
      with a boundary face); the maximum runs over the cell and its face
      neighbours.
  L7  All cells are limited at once from the unlimited coefficients; the
      limited coefficients feed the flux, the solver keeps the unlimited ones.
  L8  Linear (boundary) cells keep X3..X5 = 0 and limit X1, X2.
  L9  Limiting in characteristic variables (the variant of section 4.2):
      each derivative's four candidates, one per conserved variable, are
      mapped to characteristic variables with the left eigenvectors of the
      Euler flux Jacobian along a direction n, at cell i's average state;
      each characteristic field is limited by Eq. DWBAP with the same
      weights; the result is mapped back with the right eigenvectors.  One
      basis serves all five derivatives of the cell.  n is the direction of
      cell i's unlimited density gradient (the normal of a shock or contact
      through the cell), the x axis where that gradient vanishes.
"""
from __future__ import annotations

import numpy as np

from .cls import cell_orders

EPS = 1e-8


def smoothness_exponent(chi):
    """S(chi) of Eq. DWBAP_S."""
    return 1.0 / (np.sqrt(chi + EPS) + 0.05)


def dwbap(cands, weights):
    """Eq. DWBAP with B = arctan (reading L3).  cands [J+1], weights [J+1]
    summing to one."""
    return np.tan(np.dot(weights, np.arctan(np.asarray(cands))))


def cell_stencils(geo, mesh):
    """For each cell, its face neighbours in local-edge order (edge e runs
    from vertex e to vertex e+1, counter-clockwise), boundary edges skipped:
    a list of (neighbour, midpoint of the shared edge minus the centroid)."""
    tri = mesh.tri
    v = mesh.unwrapped_vertices()
    owners = {}
    for t in range(geo.nt):
        for e in range(3):
            a, b = int(tri[t, e]), int(tri[t, (e + 1) % 3])
            owners.setdefault((min(a, b), max(a, b)), []).append(t)
    st = []
    for t in range(geo.nt):
        row = []
        for e in range(3):
            a, b = int(tri[t, e]), int(tri[t, (e + 1) % 3])
            others = [u for u in owners[(min(a, b), max(a, b))] if u != t]
            if others:
                row.append((others[0], 0.5 * (v[t, e] + v[t, (e + 1) % 3]) - geo.cen[t]))
        st.append(row)
    return st


def _poly_at(geo, W, X, j, d):
    """Value (4), gradient (4, 2) and Hessian entries (4, 3) of cell j's
    polynomials at displacement d (2,) from its centroid."""
    h = geo.h[j]
    dx, dy = d / h
    phi = np.array([dx, dy, 0.5 * (dx * dx - geo.Ixx[j] / h ** 2), dx * dy - geo.Ixy[j] / h ** 2,
                    0.5 * (dy * dy - geo.Iyy[j] / h ** 2)])
    Xj = X[:, :, j]                                            # [4, 5]
    val = W[:, j] + Xj @ phi
    gx = (Xj[:, 0] + Xj[:, 2] * dx + Xj[:, 3] * dy) / h
    gy = (Xj[:, 1] + Xj[:, 3] * dx + Xj[:, 4] * dy) / h
    hes = Xj[:, 2:5] / h ** 2
    return val, np.stack([gx, gy], axis=1), hes


def shock_indicator(geo, W, X, mesh, stencils=None, k=None):
    """IS_i of Eq. ISD1 for every cell (reading L6); k: cell orders."""
    st = cell_stencils(geo, mesh) if stencils is None else stencils
    k = cell_orders(geo) if k is None else k
    IS = np.zeros(geo.nt)
    for i in range(geo.nt):
        J = len(st[i])
        if J == 0:
            continue
        own, _, _ = _poly_at(geo, W, X, i, np.zeros(2))
        num = 0.0
        umax = W[0, i]
        for j, _f in st[i]:
            d = geo.minimg(geo.cen[i] - geo.cen[j])
            vj, _, _ = _poly_at(geo, W, X, j, d)
            num += abs(own[0] - vj[0])
            umax = max(umax, W[0, j])
        IS[i] = num / (J * geo.h[i] ** ((k[i] + 1) / 2.0) * umax)
    return IS


def limiter_weights(geo, W, i, stencil, gamma):
    """omega_j, j = 0..J, of Eq. DWBAP_w for cell i (readings L4, L5)."""
    h = geo.h[i]
    mids = []
    cents = [np.zeros(2)]
    for j, mid in stencil:
        mids.append(mid)                           # relative to cell i
        cents.append(geo.minimg(geo.cen[j] - geo.cen[i]))
    mids = np.array(mids) / h
    cents = np.array(cents) / h
    p = np.array([(gamma - 1.0) * (W[3, j] - 0.5 * (W[1, j] ** 2 + W[2, j] ** 2) / W[0, j]) for j, _ in stencil])
    pbar = p.mean()
    chi = np.sqrt(np.mean((p - pbar) ** 2)) / pbar
    S = smoothness_exponent(chi)
    D = np.array([np.mean(np.linalg.norm(c[None, :] - mids, axis=1)) for c in cents])
    beta = D ** (-S)
    return beta / beta.sum()


def characteristic_basis(Wc, gamma, n):
    """Right eigenvectors [4, 4] (columns) of the Jacobian of the Euler flux
    F(W) . n with respect to the conserved variables, at state Wc, for unit
    n; eigenvalues u_n - c, u_n, u_n, u_n + c.  Columns: the acoustic wave
    against n, the entropy wave, the shear wave, the acoustic wave along n."""
    rho = Wc[0]
    u, v = Wc[1] / rho, Wc[2] / rho
    p = (gamma - 1.0) * (Wc[3] - 0.5 * rho * (u * u + v * v))
    c = np.sqrt(gamma * p / rho)
    H = (Wc[3] + p) / rho
    nx, ny = n
    un = u * nx + v * ny
    ut = -u * ny + v * nx
    return np.array([[1.0, 1.0, 0.0, 1.0],
                     [u - c * nx, u, -ny, u + c * nx],
                     [v - c * ny, v, nx, v + c * ny],
                     [H - c * un, 0.5 * (u * u + v * v), ut, H + c * un]])


def limiting_direction(X, i):
    """Unit direction of cell i's unlimited density gradient (reading L9)."""
    g = X[0, 0:2, i]
    nrm = np.hypot(g[0], g[1])
    return np.array([1.0, 0.0]) if nrm == 0.0 else g / nrm


def first_derivative_candidates(geo, W, X, Xl, i, stencil, w):
    """Candidates [J+1, 4, 2] for u_x, u_y of cell i and their weights
    (reading L2): Xl holds cell i's limited second derivatives."""
    h = geo.h[i]
    J = len(stencil)
    d = np.array([geo.minimg(geo.cen[j] - geo.cen[i]) for j, _ in stencil]) / h   # [J, 2]
    rem = np.zeros((J, 4))
    for n, (j, _f) in enumerate(stencil):
        dx, dy = d[n]
        # averages over cell j of cell i's quadratic basis functions
        a3 = 0.5 * (dx * dx + (geo.Ixx[j] - geo.Ixx[i]) / h ** 2)
        a4 = dx * dy + (geo.Ixy[j] - geo.Ixy[i]) / h ** 2
        a5 = 0.5 * (dy * dy + (geo.Iyy[j] - geo.Iyy[i]) / h ** 2)
        rem[n] = (W[:, j] - W[:, i]) - (Xl[:, 2, i] * a3 + Xl[:, 3, i] * a4 + Xl[:, 4, i] * a5)
    c1 = np.zeros((J + 1, 4, 2))
    c1[0] = X[:, 0:2, i] / h
    w1 = w.copy()
    for n in range(J):
        if J < 3:
            # wall cell: the gradient along the neighbour's direction alone
            c1[n + 1] = np.outer(rem[n], d[n]) / (d[n] @ d[n]) / h
            continue
        m2 = (n + 1) % J
        A = np.array([d[n], d[m2]])
        if abs(np.linalg.det(A)) < 1e-12:
            c1[n + 1] = c1[0]
        else:
            G = np.linalg.solve(A, np.stack([rem[n], rem[m2]]))   # [2, 4]: h-scaled gradient
            c1[n + 1] = G.T / h
        # a pair candidate carries the mean weight of its two neighbours
        w1[n + 1] = 0.5 * (w[n + 1] + w[m2 + 1])
    return c1, w1


def limit(geo, W, X, mesh, gamma=1.4, threshold=1.0, k=None, variables="conservative"):
    """Limited coefficients (reading L7) and the mask of limited cells.
    threshold: IS_i at or above which a cell is limited (1 per Eq. ISD2;
    tests lower it to force limiting everywhere); k: cell orders (default:
    linear boundary cells); variables: "conservative" (reading L1) or
    "characteristic" (reading L9)."""
    if variables not in ("conservative", "characteristic"):
        raise ValueError(variables)
    st = cell_stencils(geo, mesh)
    k = cell_orders(geo) if k is None else k
    IS = shock_indicator(geo, W, X, mesh, st, k)
    Xl = X.copy()
    mask = IS >= threshold
    for i in np.nonzero(mask)[0]:
        stencil = st[i]
        if not stencil:
            continue
        h = geo.h[i]
        J = len(stencil)
        w = limiter_weights(geo, W, i, stencil, gamma)
        if variables == "characteristic":
            R = characteristic_basis(W[:, i], gamma, limiting_direction(X, i))
            Lft = np.linalg.inv(R)

        def limited(cands, wts):
            # cands [J+1, 4]: one candidate vector of conserved variables per row
            if variables == "conservative":
                return np.array([dwbap(cands[:, q], wts) for q in range(4)])
            ch = cands @ Lft.T
            return R @ np.array([dwbap(ch[:, q], wts) for q in range(4)])

        # second derivatives u_xx, u_xy, u_yy: own and the neighbours'
        if k[i] == 2:
            c2 = np.zeros((J + 1, 4, 3))
            c2[0] = X[:, 2:5, i] / h ** 2
            for n, (j, _f) in enumerate(stencil, start=1):
                c2[n] = X[:, 2:5, j] / geo.h[j] ** 2
            for l in range(3):
                Xl[:, 2 + l, i] = limited(c2[:, :, l], w) * h * h
        # first derivatives from remainder averages (readings L2)
        c1, w1 = first_derivative_candidates(geo, W, X, Xl, i, stencil, w)
        for l in range(2):
            Xl[:, l, i] = limited(c1[:, :, l], w1) * h
    return Xl, mask
