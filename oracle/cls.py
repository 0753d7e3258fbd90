"""Oracle compact least-squares (CLS) reconstruction, section 3.

Each cell i carries the quadratic of Eq. quadRCP,

    u^i(x, y) = ubar_i + u1 dx + u2 dy + u3 (dx^2 - mean_i dx^2) / 2
                + u4 (dx dy - mean_i dx dy) + u5 (dy^2 - mean_i dy^2) / 2,

with dx = (x - x_i) / h_i, dy = (y - y_i) / h_i centred at the centroid
(Eq. RCP), or only its linear part on cells with a boundary edge (Eq. k_i).
For every ordered pair of face neighbours (i, j) the mean over cell j of each
derivative of order p = m + n <= M = k_i of u^i must equal that of u^j
(Eqs. spdConserved:1-2), giving the rows A^i_j u^i - B^i_j u^j = b^i_j
(Eqs. spdConserved:3, A:B:b:2), each scaled by w_{i,p} = (w h_i)^p with
w = 0.3 (Eq. A:B:b:3).  All rows over all pairs form one over-determined
system C u = b (Eq. spdConserved:4), solved in the least-squares sense
through its normal equations C^T C u = C^T b (Eq. spdConserved:5).

Reading of the paper used here: the normal equations are those of the
single global system ("reading G"), as Eq. spdConserved:5 is written.  ``reading='P'``
switches to the per-cell reading (only A^T applied), which has the same
right-hand side and sparsity.

The solution is obtained with a library sparse direct solver; RCM, ILU and
GMRES only accelerate reaching it and are not part of the oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import Geometry

CLS_W = 0.3


def cell_orders(geo: Geometry, all_quadratic: bool = False) -> np.ndarray:
    """k_i of Eq. k_i: 1 on cells touching the boundary, 2 inside."""
    k = np.full(geo.nt, 2, dtype=np.int64)
    if not all_quadratic:
        k[geo.boundary_cell] = 1
    return k


def pair_blocks(geo: Geometry, i: np.ndarray, j: np.ndarray, k: np.ndarray, w: float = CLS_W):
    """Weighted condition blocks for ordered neighbour pairs (i, j).

    Returns A [np, 6, 5], B [np, 6, 5] and a0 [np, 5] (row p = 0 of A).
    Row order: p = 0; p = 1: d/dx, d/dy; p = 2: d2/dx2, d2/dxdy, d2/dy2.
    Columns follow the basis of Eq. quadRCP.  Rows with p > k_i and columns
    beyond DOF(k_i) (for A) or DOF(k_j) (for B) are zero.

    Entries are the cell-j means of the basis derivatives (Eq. A:B:b):
      mean_j phi_{l,i}   uses mean_j (x - x_i)^2 = (x_j - x_i)^2 + Ixx_j, ...
      mean_j d phi_{l,i} / dx = (1, 0, dx, dy, 0) / h_i, ...
      mean_j d^2 phi_{l,i} = unit vectors / h_i^2
    and the basis of cell j has zero mean over cell j, so row p = 0 of B is 0.
    """
    hi = geo.h[i]
    hj = geo.h[j]
    d = geo.minimg(geo.cen[j] - geo.cen[i]) / hi[:, None]
    dx, dy = d[:, 0], d[:, 1]
    r = hi / hj
    n = i.shape[0]
    a0 = np.stack([
        dx,
        dy,
        0.5 * (dx * dx + (geo.Ixx[j] - geo.Ixx[i]) / hi ** 2),
        dx * dy + (geo.Ixy[j] - geo.Ixy[i]) / hi ** 2,
        0.5 * (dy * dy + (geo.Iyy[j] - geo.Iyy[i]) / hi ** 2),
    ], axis=1)
    A = np.zeros((n, 6, 5))
    B = np.zeros((n, 6, 5))
    # p = 0, weight (w h_i)^0 = 1
    A[:, 0, :] = a0
    # p = 1, weight w h_i; the derivative brings 1/h_i (cell i) or 1/h_j (cell j)
    A[:, 1, 0] = w
    A[:, 1, 2] = w * dx
    A[:, 1, 3] = w * dy
    A[:, 2, 1] = w
    A[:, 2, 3] = w * dx
    A[:, 2, 4] = w * dy
    B[:, 1, 0] = w * r
    B[:, 2, 1] = w * r
    # p = 2, weight (w h_i)^2
    for q, col in ((3, 2), (4, 3), (5, 4)):
        A[:, q, col] = w * w
        B[:, q, col] = w * w * r * r
    ki = k[i]
    kj = k[j]
    lin_i = ki == 1
    lin_j = kj == 1
    A[lin_i, 3:, :] = 0.0      # M = k_i = 1: no second-derivative rows
    B[lin_i, 3:, :] = 0.0
    A[lin_i, :, 2:] = 0.0      # DOF(1) = 2 unknowns on cell i
    B[lin_j, :, 2:] = 0.0      # DOF(1) = 2 unknowns on cell j
    return A, B, a0


def interior_pairs(geo: Geometry):
    m = geo.nbr >= 0
    o = geo.own[m]
    nb = geo.nbr[m]
    return np.concatenate([o, nb]), np.concatenate([nb, o])


def assemble(geo: Geometry, k: np.ndarray | None = None, w: float = CLS_W, reading: str = "G"):
    """Normal-equation matrix K (sparse, 5 nt x 5 nt) of Eq. spdConserved:5.

    Unknown (i, l) sits at row 5 i + l.  Unused quadratic unknowns of linear
    cells get an identity row so the matrix stays square and regular.
    Returns (K, pairs) where pairs = (i, j, a0) feeds ``rhs``.
    """
    if k is None:
        k = cell_orders(geo)
    i, j = interior_pairs(geo)
    A, B, a0 = pair_blocks(geo, i, j, k, w)
    AtA = np.einsum("prk,prl->pkl", A, A)
    AtB = np.einsum("prk,prl->pkl", A, B)
    BtB = np.einsum("prk,prl->pkl", B, B)
    rows, cols, vals = [], [], []

    def put(bi, bj, blk):
        r = (5 * bi)[:, None, None] + np.arange(5)[None, :, None]
        c = (5 * bj)[:, None, None] + np.arange(5)[None, None, :]
        rows.append(np.broadcast_to(r, blk.shape).ravel())
        cols.append(np.broadcast_to(c, blk.shape).ravel())
        vals.append(blk.ravel())

    put(i, i, AtA)
    put(i, j, -AtB)
    if reading == "G":
        put(j, j, BtB)
        put(j, i, -np.transpose(AtB, (0, 2, 1)))
    elif reading != "P":
        raise ValueError("reading must be 'G' or 'P'")
    lin = np.nonzero(k == 1)[0]
    for l in range(2, 5):
        rows.append(5 * lin + l)
        cols.append(5 * lin + l)
        vals.append(np.ones(lin.shape[0]))
    n = 5 * geo.nt
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K, (i, j, a0, A)


def rhs(geo: Geometry, pairs, W: np.ndarray) -> np.ndarray:
    """Right-hand side C^T b of Eq. spdConserved:5 for the four conserved
    variables: R_i = sum_j A_ij^T b_ij with b_ij = (ubar_j - ubar_i) e_0
    (Eq. A:B:b).  B^T b vanishes because row 0 of B is zero.

    Returns R [4, nt, 5]."""
    i, j, a0, A = pairs
    R = np.zeros((4, geo.nt, 5))
    for v in range(4):
        diff = W[v, j] - W[v, i]
        contrib = A[:, 0, :] * diff[:, None]
        np.add.at(R[v], i, contrib)
    return R


def factorize(K, spd: bool = True):
    """SuperLU factorisation of K.  Under reading G, K is symmetric positive
    definite (the normal equations of one global least-squares system), so
    the factorisation takes a symmetric fill-reducing order (minimum degree
    on K + K^T) and keeps the diagonal pivots (no pivoting is needed for an
    SPD matrix); this changes the rounding order of the direct solve, not
    what it computes, and keeps the fill of meshes with 10^6 cells within
    host memory.  Reading P's matrix is not symmetric and takes SuperLU's
    default column order with partial pivoting."""
    if spd:
        return spla.splu(K.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                         options=dict(SymmetricMode=True))
    return spla.splu(K.tocsc())


# Above this many unknowns the SuperLU factorisation's fill passes the
# 32-bit index range of SciPy's build (the 10^6-cell shock-vortex mesh, 5e6
# unknowns, fails; 524,288 cells, 2.6e6 unknowns, fits), so the oracle
# solves iteratively instead.
DIRECT_MAX_UNKNOWNS = 3_000_000


def block_jacobi(K):
    """Inverses of the 5 x 5 diagonal blocks of K as a block-diagonal sparse
    matrix (the preconditioner of solve_cg)."""
    n = K.shape[0] // 5
    B = K.tobsr(blocksize=(5, 5))
    rows = np.repeat(np.arange(n), np.diff(B.indptr))
    diag = B.data[B.indices == rows]
    if diag.shape[0] != n:
        raise ValueError("K lacks a diagonal block")
    return sp.bsr_matrix((np.linalg.inv(diag), np.arange(n), np.arange(n + 1)), shape=K.shape).tocsr()


def solve_cg(K, R: np.ndarray, rtol: float = 1e-14) -> np.ndarray:
    """K X = R for the four columns by conjugate gradients (K is symmetric
    positive definite under reading G) with the block-Jacobi preconditioner,
    from X = 0 to a relative residual of rtol per column (1e-14 reaches the
    direct solve's solution to about 1e-13 relative); X [4, 5, nt]."""
    nt = R.shape[1]
    rhs_mat = R.reshape(4, 5 * nt).T
    Kc = K.tocsr()
    P = block_jacobi(Kc)
    X = np.zeros_like(rhs_mat)
    for c in range(4):
        if not np.any(rhs_mat[:, c]):
            continue
        x, info = spla.cg(Kc, rhs_mat[:, c], rtol=rtol, atol=0.0, maxiter=10000, M=P)
        if info != 0:
            raise RuntimeError("CG did not reach the relative residual %g (column %d)" % (rtol, c))
        X[:, c] = x
    return np.ascontiguousarray(X.T.reshape(4, nt, 5).transpose(0, 2, 1))


def solve(K, R: np.ndarray, spd: bool = True) -> np.ndarray:
    """Direct solve of K X = R for the four columns; returns X [4, 5, nt]
    in the layout of the library (variable, coefficient, cell)."""
    nt = R.shape[1]
    rhs_mat = R.reshape(4, 5 * nt).T
    if 5 * nt <= 4000:
        Xf = np.linalg.solve(K.toarray(), rhs_mat)
    else:
        Xf = factorize(K, spd).solve(rhs_mat)
    return np.ascontiguousarray(Xf.T.reshape(4, nt, 5).transpose(0, 2, 1))


def reconstruct(geo: Geometry, W: np.ndarray, k=None, reading: str = "G", w: float = CLS_W):
    """Coefficients X [4, 5, nt] of the CLS reconstruction of W [4, nt]."""
    K, pairs = assemble(geo, k, w, reading)
    return solve(K, rhs(geo, pairs, W), spd=reading == "G")


def residual(K, R: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Relative residual ||R - K X|| / ||R|| per column (0 for a zero R)."""
    nt = R.shape[1]
    out = np.zeros(4)
    for v in range(4):
        x = X[v].T.reshape(-1)
        b = R[v].reshape(-1)
        nb = np.linalg.norm(b)
        out[v] = np.linalg.norm(b - K @ x) / nb if nb > 0 else np.linalg.norm(K @ x)
    return out
