"""Seeded sparse SPD matrices that do not come from the ocean grid.

Sec. 5 of the paper also compares the preconditioners on a matrix from
outside the ocean model.  That matrix is not available here; these generators
stand in for it with the same kind of object: the stiffness-like matrix of an
unstructured point cloud (irregular degrees, no grid structure), symmetric
positive definite, stored in CSR with the columns of each row ascending.

Construction (all seeded):
  - points: a mixture of Gaussian clusters and a uniform background in the
    unit square, so the point density (and the node degree) varies;
  - graph: each point joined to its k nearest neighbours, symmetrised;
  - couplings: w_ij = 1 / (|p_i - p_j| + h), h a small length, so close
    pairs couple strongly;
  - ordering: reverse Cuthill-McKee of the graph (a usual numbering of
    unstructured meshes);
  - "laplacian": A_ij = -w_ij, A_ii = sum_j w_ij + sigma_i with sigma_i > 0
    only on points near the square's boundary (a Dirichlet-like condition)
    and on one point of every connected component that has none: each block
    is an irreducibly diagonally dominant M-matrix, hence SPD;
  - "mixed": the same magnitudes with seeded signs on the couplings and
    A_ii = sum_j |w_ij| + sigma_i: SPD by diagonal dominance, not an
    M-matrix.
The right-hand side is N(0, 1), seeded.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class CsrProblem:
    n: int
    rowptr: np.ndarray     # int64 [n+1]
    col: np.ndarray        # int64 [nnz], ascending within each row
    val: np.ndarray        # float64 [nnz]
    b: np.ndarray          # float64 [n]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def dense(self) -> np.ndarray:
        """Dense matrix (small problems only; for tests)."""
        M = np.zeros((self.n, self.n))
        for k in range(self.n):
            a, e = self.rowptr[k], self.rowptr[k + 1]
            M[k, self.col[a:e]] = self.val[a:e]
        return M

    def diag(self) -> np.ndarray:
        d = np.zeros(self.n)
        for k in range(self.n):
            a, e = self.rowptr[k], self.rowptr[k + 1]
            m = self.col[a:e] == k
            d[k] = self.val[a:e][m][0]
        return d


def _points(npts, rng):
    nc = max(3, npts // 4000)
    centres = rng.uniform(0.1, 0.9, size=(nc, 2))
    widths = rng.uniform(0.02, 0.12, size=nc)
    n_bg = npts // 3
    lab = rng.integers(0, nc, size=npts - n_bg)
    pts = centres[lab] + rng.standard_normal((npts - n_bg, 2)) * widths[lab, None]
    pts = np.vstack([pts, rng.uniform(0.0, 1.0, size=(n_bg, 2))])
    return np.clip(pts, 0.0, 1.0)


def unstructured_problem(npts: int, seed: int, k: int = 6, kind: str = "laplacian") -> CsrProblem:
    """Stiffness-like SPD matrix of a seeded point cloud (see module doc)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    from scipy.spatial import cKDTree

    if kind not in ("laplacian", "mixed"):
        raise ValueError("kind must be 'laplacian' or 'mixed'")
    rng = np.random.default_rng(seed)
    pts = _points(int(npts), rng)
    n = pts.shape[0]
    tree = cKDTree(pts)
    kk = min(k + 1, n)
    dist, nb = tree.query(pts, k=kk)
    rows = np.repeat(np.arange(n), kk - 1)
    cols = nb[:, 1:].ravel()
    G = coo_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n)).tocsr()
    G = ((G + G.T) > 0).astype(np.float64).tocsr()
    perm = reverse_cuthill_mckee(G, symmetric_mode=True)
    pts = pts[perm]
    G = G[perm][:, perm].tocoo()
    i, j = G.row, G.col
    keep = i < j
    i, j = i[keep], j[keep]
    h = 0.1 / np.sqrt(n)
    w = 1.0 / (np.linalg.norm(pts[i] - pts[j], axis=1) + h)
    w = w / np.mean(w)
    if kind == "mixed":
        sign = np.where(rng.random(w.size) < 0.5, -1.0, 1.0)
    else:
        sign = -np.ones(w.size)
    off = sign * w
    deg = np.zeros(n)
    np.add.at(deg, i, w)
    np.add.at(deg, j, w)
    edge = np.minimum.reduce([pts[:, 0], pts[:, 1], 1.0 - pts[:, 0], 1.0 - pts[:, 1]])
    sigma = np.where(edge < 2.0 / np.sqrt(n), 1.0, 0.0)
    # every connected component of the graph needs one shifted point, or its
    # block of A is singular (a kNN graph of clustered points can fall apart)
    from scipy.sparse.csgraph import connected_components
    ncomp, comp = connected_components(G.tocsr(), directed=False)
    has = np.zeros(ncomp, dtype=bool)
    has[comp[sigma > 0]] = True
    for cidx in np.nonzero(~has)[0]:
        sigma[np.argmax(comp == cidx)] = 1.0
    diag = deg + sigma
    r = np.concatenate([i, j, np.arange(n)])
    c = np.concatenate([j, i, np.arange(n)])
    v = np.concatenate([off, off, diag])
    A = coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    A.sort_indices()
    b = rng.standard_normal(n)
    return CsrProblem(n, A.indptr.astype(np.int64), A.indices.astype(np.int64),
                      A.data.astype(np.float64), b, name=f"unstructured{n}_{kind}")


def csr_from_grid(p) -> CsrProblem:
    """The five-point operator of a grid Problem written as CSR (zero
    couplings omitted, columns ascending), with the same right-hand side."""
    n = p.n
    nx, ny = p.nx, p.ny
    rowptr = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for kcell in range(n):
        ii, jj = kcell % nx, kcell // nx
        e = []
        if jj > 0 and p.an[kcell - nx] != 0.0:
            e.append((kcell - nx, p.an[kcell - nx]))
        if ii > 0:
            if p.ae[kcell - 1] != 0.0:
                e.append((kcell - 1, p.ae[kcell - 1]))
        elif p.periodic and p.ae[kcell + nx - 1] != 0.0:
            e.append((kcell + nx - 1, p.ae[kcell + nx - 1]))
        e.append((kcell, p.diag[kcell]))
        if ii < nx - 1 or p.periodic:
            if p.ae[kcell] != 0.0:
                e.append((kcell + 1 if ii < nx - 1 else kcell - nx + 1, p.ae[kcell]))
        if jj < ny - 1 and p.an[kcell] != 0.0:
            e.append((kcell + nx, p.an[kcell]))
        e.sort()
        cols.extend(c for c, _ in e)
        vals.extend(v for _, v in e)
        rowptr[kcell + 1] = len(cols)
    return CsrProblem(n, rowptr, np.array(cols, dtype=np.int64), np.array(vals), p.b.copy(),
                      name=f"csr_{p.name}")
