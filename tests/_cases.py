"""Hand-built operators with known structure, for pins (no solver arithmetic)."""
import numpy as np

from gen import Problem


def tridiag_problem(diag, off, b=None):
    """1-D operator (ny = 1, no wrap): A = tridiag(off, diag, off).

    `off[k]` is A[k, k+1]; its last entry must be 0 (no east neighbour).
    """
    n = len(diag)
    off = np.asarray(off, dtype=np.float64).copy()
    off[-1] = 0.0
    b = np.ones(n) if b is None else np.asarray(b, dtype=np.float64)
    return Problem(n, 1, False, np.asarray(diag, dtype=np.float64), off, np.zeros(n),
                   np.ones(n, dtype=bool), b, name=f"tri{n}")


def laplace1d(n):
    """tridiag(-1, 2, -1)."""
    return tridiag_problem(np.full(n, 2.0), np.full(n, -1.0))


def const_periodic(nx, ny, b=None):
    """Constant-coefficient 5-point operator, periodic in i, Dirichlet in j:
    (A x)_k = 4 x_k - x_E - x_W - x_N - x_S with x = 0 beyond the j edges."""
    n = nx * ny
    diag = np.full(n, 4.0)
    ae = np.full(n, -1.0)
    an = np.full(n, -1.0)
    an[(ny - 1) * nx:] = 0.0
    b = np.ones(n) if b is None else b
    return Problem(nx, ny, True, diag, ae, an, np.ones(n, dtype=bool), b, name="cper")


def stencil_reference(nx, ny, periodic, x):
    """Textbook constant 5-point Laplacian applied with array shifts."""
    X = x.reshape(ny, nx)
    P = np.zeros((ny + 2, nx + 2))
    P[1:-1, 1:-1] = X
    if periodic:
        P[1:-1, 0] = X[:, -1]
        P[1:-1, -1] = X[:, 0]
    y = 4 * X - P[1:-1, 2:] - P[1:-1, :-2] - P[2:, 1:-1] - P[:-2, 1:-1]
    return y.ravel()


def cholesky_ainv(M):
    """Unit-upper Z and D with M^-1 = Z D^-1 Z^T, from a dense Cholesky
    M = L L^T:  M^-1 = L^-T L^-1, so Z = L^-T diag(L), D = diag(L)^2."""
    L = np.linalg.cholesky(M)
    Linv = np.linalg.inv(L)
    dl = np.diag(L)
    Z = Linv.T * dl[None, :]
    return Z, dl ** 2


def mixed_sign_dominant(nx, ny, periodic, seed):
    """Five-point operator with couplings of both signs, U(-1, 1) seeded, and
    a strictly dominant diagonal (1.05 x the row's absolute coupling sum plus
    1e-3): symmetric positive definite but not an M-matrix."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    ae = rng.uniform(-1.0, 1.0, n)
    an = rng.uniform(-1.0, 1.0, n)
    if not periodic:
        ae[nx - 1::nx] = 0.0
    an[(ny - 1) * nx:] = 0.0
    A = np.abs(ae).reshape(ny, nx)
    west = np.roll(A, 1, axis=1)
    if not periodic:
        west[:, 0] = 0.0
    N = np.abs(an).reshape(ny, nx)
    south = np.zeros_like(N)
    south[1:] = N[:-1]
    diag = (A + west + N + south).ravel() * 1.05 + 1e-3
    return Problem(nx, ny, periodic, diag, ae, an, np.ones(n, dtype=bool), np.ones(n),
                   name=f"mixed{nx}x{ny}")
