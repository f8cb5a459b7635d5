"""Synthetic ORCA-shaped elliptic problems (seeded, deterministic).

Operator (paper Sec. 3, eq. (8) and eq. (10)).  The five-point system couples
cell (i, j) to its four neighbours through face coefficients; the diagonal is
the sum of the four faces of the cell.  Eq. (10) is written with -d on the
diagonal (negative definite); we store its negation, which is symmetric
positive definite: A[k,k] = sum of the 4 face coefficients (faces towards land
or a domain edge included, i.e. Dirichlet), A[k,nbr] = -c_face between two
ocean cells.  Land cells are identity rows with a zero right-hand side.

Face coefficients on the sphere (Sec. 2, metric factors e1 = r cos(phi),
e2 = r; Sec. 3, C^EW ~ H e2/e1 and C^NS ~ H e1/e2).  For a face between cells
of a lon/lat grid with spacings dlam, dphi (radians):

  east-west face (i+1/2, j):   c = H_f * dphi / (cos(phi_j) * dlam)
  north-south face (i, j+1/2): c = H_f * cos(phi_{j+1/2}) * dlam / dphi

The radius cancels; the uniform factor 2*dt^2 of eq. (8) is dropped (a global
scale changes neither the Krylov iterates nor the preconditioner pattern in
exact arithmetic).  H_f is the mean depth of the two cells.

Storage ("A5"): three row-major arrays over the nx*ny grid, cell k = j*nx + i
(i runs west->east fastest, then j south->north, the natural ordering of
Sec. 3):
  diag[k] = A[k, k]
  ae[k]   = A[k, east(k)]   (east(k) wraps to i=0 when periodic)
  an[k]   = A[k, k + nx]
The west/south entries of row k are ae[west(k)] and an[k - nx] (symmetry).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Seeds: base + configuration index (0: box, 1: 182x149, 2: 1442x1021,
# 3: ensemble, 4: serving catalogue).
CONFIG_SEED_BASE = 1878


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    periodic: bool
    diag: np.ndarray          # float64 [ny*nx]
    ae: np.ndarray            # float64 [ny*nx]
    an: np.ndarray            # float64 [ny*nx]
    ocean: np.ndarray         # bool    [ny*nx]
    b: np.ndarray             # float64 [ny*nx]
    u_star: np.ndarray | None = None   # manufactured solution if any
    name: str = ""
    B: np.ndarray | None = None        # several right-hand sides [nrhs, n]

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def dense(self) -> np.ndarray:
        """Dense n x n matrix (tiny grids only; for tests)."""
        n = self.n
        nx, ny = self.nx, self.ny
        M = np.zeros((n, n))
        for k in range(n):
            M[k, k] = self.diag[k]
            i, j = k % nx, k // nx
            if i < nx - 1 or self.periodic:
                e = j * nx + (i + 1) % nx
                if self.ae[k] != 0.0:
                    M[k, e] += self.ae[k]
                    M[e, k] += self.ae[k]
            if j < ny - 1 and self.an[k] != 0.0:
                M[k, k + nx] += self.an[k]
                M[k + nx, k] += self.an[k]
        return M

    def footprint(self) -> int:
        return 8 * 4 * self.n


def _assemble(nx, ny, periodic, cE, cN, cW0, cS0, ocean):
    """Assemble A5 from face coefficients.

    cE[j, i]: face between (i, j) and (i+1, j); for i = nx-1 this is the
              periodic face to (0, j) or, without periodicity, the east edge.
    cN[j, i]: face between (i, j) and (i, j+1); j = ny-1 is the north edge.
    cW0[j]:   west edge face of (0, j) (non-periodic only, else unused).
    cS0[i]:   south edge face of (i, 0).
    ocean[j, i]: mask.
    """
    diag = np.zeros((ny, nx))
    diag += cE                                  # east face of each cell
    if periodic:
        diag += np.roll(cE, 1, axis=1)          # west face = east face of west nbr
    else:
        diag[:, 1:] += cE[:, :-1]
        diag[:, 0] += cW0
    diag += cN                                  # north face
    diag[1:, :] += cN[:-1, :]                   # south face
    diag[0, :] += cS0

    ae = -cE.copy()
    if periodic:
        east_ocean = np.roll(ocean, -1, axis=1)
    else:
        east_ocean = np.zeros_like(ocean)
        east_ocean[:, :-1] = ocean[:, 1:]
        ae[:, -1] = 0.0
    ae[~(ocean & east_ocean)] = 0.0

    an = -cN.copy()
    north_ocean = np.zeros_like(ocean)
    north_ocean[:-1, :] = ocean[1:, :]
    an[-1, :] = 0.0
    an[~(ocean & north_ocean)] = 0.0

    diag[~ocean] = 1.0
    # Off-diagonals must vanish on land rows (set above through the masks);
    # -0.0 from negating a zero face is normalised to +0.0.
    ae = ae + 0.0
    an = an + 0.0
    return (np.ascontiguousarray(diag.ravel()), np.ascontiguousarray(ae.ravel()),
            np.ascontiguousarray(an.ravel()))


def manufactured_solution(nx, ny):
    x = (np.arange(nx) + 1.0) / (nx + 1.0)
    y = (np.arange(ny) + 1.0) / (ny + 1.0)
    X, Y = np.meshgrid(x, y)
    u = np.sin(np.pi * X) * np.sin(np.pi * Y) + 0.5 * np.sin(3 * np.pi * X) * np.sin(2 * np.pi * Y)
    return u.ravel()


def apply_a5(nx, ny, periodic, diag, ae, an, x):
    """y = A x for the A5 storage (input construction only: manufactured RHS)."""
    X = x.reshape(ny, nx)
    D = diag.reshape(ny, nx)
    E = ae.reshape(ny, nx)
    N = an.reshape(ny, nx)
    y = D * X
    if periodic:
        y += E * np.roll(X, -1, axis=1)
        y += np.roll(E, 1, axis=1) * np.roll(X, 1, axis=1)
    else:
        y[:, :-1] += E[:, :-1] * X[:, 1:]
        y[:, 1:] += E[:, :-1] * X[:, :-1]
    y[:-1, :] += N[:-1, :] * X[1:, :]
    y[1:, :] += N[:-1, :] * X[:-1, :]
    return y.ravel()


def box_problem(nx=64, ny=48, seed=CONFIG_SEED_BASE + 0, perturb=0.1, constant=False):
    """Dirichlet box: every face 1 + U(-perturb, perturb); no land, no wrap.

    With constant=True every face is exactly 1 (the constant-coefficient
    5-point Laplacian, whose spectrum has a closed form).
    """
    rng = np.random.default_rng(seed)
    if constant:
        f = lambda shape: np.ones(shape)  # noqa: E731
    else:
        f = lambda shape: 1.0 + rng.uniform(-perturb, perturb, size=shape)  # noqa: E731
    cE = f((ny, nx))        # includes the east edge face at i = nx-1
    cW0 = f((ny,))
    cN = f((ny, nx))        # includes the north edge face at j = ny-1
    cS0 = f((nx,))
    ocean = np.ones((ny, nx), dtype=bool)
    diag, ae, an = _assemble(nx, ny, False, cE, cN, cW0, cS0, ocean)
    u = manufactured_solution(nx, ny)
    b = apply_a5(nx, ny, False, diag, ae, an, u)
    return Problem(nx, ny, False, diag, ae, an, ocean.ravel(), b, u_star=u,
                   name=f"box{nx}x{ny}")


def _bathymetry(nx, ny, lam, phi, rng, modes=32):
    """Smooth seeded depth field in lon/lat, min-max mapped to [500, 5500] m."""
    H = np.zeros((ny, nx))
    for _ in range(modes):
        k = rng.integers(0, 5)           # zonal wavenumber (periodic in lon)
        l = rng.uniform(0.5, 4.0)        # meridional wavenumber
        a = rng.normal() / (1.0 + k + l)
        ps, pc = rng.uniform(0, 2 * np.pi, size=2)
        H += a * np.outer(np.cos(l * phi + pc), np.cos(k * lam + ps))
    lo, hi = H.min(), H.max()
    return 500.0 + 5000.0 * (H - lo) / (hi - lo)


def _land_mask(nx, ny, lam, phi, rng, land_frac=0.35, blobs=12):
    """Thresholded sum of seeded Gaussian blobs in great-circle distance."""
    f = np.zeros((ny, nx))
    sphi, cphi = np.sin(phi)[:, None], np.cos(phi)[:, None]
    for _ in range(blobs):
        lam0 = rng.uniform(0, 2 * np.pi)
        phi0 = math.asin(rng.uniform(-1.0, 1.0))
        sig = math.radians(rng.uniform(5.0, 20.0))
        w = rng.uniform(0.5, 1.5)
        cosd = sphi * math.sin(phi0) + cphi * math.cos(phi0) * np.cos(lam[None, :] - lam0)
        d = np.arccos(np.clip(cosd, -1.0, 1.0))
        f += w * np.exp(-0.5 * (d / sig) ** 2)
    thr = np.quantile(f, 1.0 - land_frac)
    return f < thr


@dataclasses.dataclass
class Geometry:
    """Lon/lat geometry of the ORCA-shaped grid (radians)."""
    lam: np.ndarray      # [nx] cell-centre longitudes
    phi_c: np.ndarray    # [ny] cell-centre latitudes
    phi_f: np.ndarray    # [ny+1] face latitudes (j-1/2 for j = 0..ny)
    cos_f: np.ndarray    # [ny+1] cos of the face latitudes (0 at the pole)
    dlam: float
    dphi: float


def orca_geometry(nx, ny) -> Geometry:
    """phi in [-78, 90] degrees, EW periodic, uniform spacings."""
    dphi_deg = 168.0 / ny
    dlam = 2.0 * np.pi / nx
    dphi = math.radians(dphi_deg)
    lam = (np.arange(nx) + 0.5) * dlam
    phi_c = np.radians(-78.0 + (np.arange(ny) + 0.5) * dphi_deg)
    # face latitudes: j+1/2 for j = -1..ny-1; the last one is exactly the pole
    phi_f = np.radians(-78.0 + np.arange(ny + 1) * dphi_deg)
    cos_f = np.cos(phi_f)
    cos_f[-1] = 0.0        # fl(cos(pi/2)) != 0: the polar face carries nothing
    return Geometry(lam, phi_c, phi_f, cos_f, dlam, dphi)


def orca_problem(nx, ny, seed, land_frac=0.35, rhs=True):
    """ORCA-shaped lon/lat grid: phi in [-78, 90] degrees, EW periodic."""
    rng = np.random.default_rng(seed)
    geo = orca_geometry(nx, ny)
    dlam, dphi, lam, phi_c, cos_f = geo.dlam, geo.dphi, geo.lam, geo.phi_c, geo.cos_f

    H = _bathymetry(nx, ny, lam, phi_c, rng)
    ocean = _land_mask(nx, ny, lam, phi_c, rng, land_frac=land_frac)

    HE = 0.5 * (H + np.roll(H, -1, axis=1))
    cE = HE * dphi / (np.cos(phi_c)[:, None] * dlam)
    HN = np.empty_like(H)
    HN[:-1, :] = 0.5 * (H[:-1, :] + H[1:, :])
    HN[-1, :] = H[-1, :]
    cN = HN * cos_f[1:, None] * dlam / dphi
    cS0 = H[0, :] * cos_f[0] * dlam / dphi
    diag, ae, an = _assemble(nx, ny, True, cE, cN, None, cS0, ocean)
    oc = ocean.ravel()
    b = rhs_normal(oc, rng) if rhs else np.zeros(nx * ny)
    return Problem(nx, ny, True, diag, ae, an, oc, b, name=f"orca{nx}x{ny}")


def rhs_normal(ocean, rng):
    """N(0,1) on ocean cells, 0 on land."""
    if not isinstance(rng, np.random.Generator):
        rng = np.random.default_rng(rng)
    b = rng.standard_normal(ocean.shape[0])
    b[~ocean] = 0.0
    return b


def ensemble_problems(count=64, seed=CONFIG_SEED_BASE + 3, nrhs=4,
                      nx_range=(182, 362), ny_range=(149, 292)):
    """Uneven ensemble: each member has its own size, depth, land and RHS set."""
    rng = np.random.default_rng(seed)
    out = []
    for m in range(count):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        ny = int(rng.integers(ny_range[0], ny_range[1] + 1))
        p = orca_problem(nx, ny, seed=int(rng.integers(1 << 31)), rhs=False)
        rr = np.random.default_rng(int(rng.integers(1 << 31)))
        p.B = np.stack([rhs_normal(p.ocean, rr) for _ in range(nrhs)])
        out.append(p)
    return out


@dataclasses.dataclass
class TransportModes:
    """Face transports of an ORCA-shaped grid as fixed spatial fields and time
    factors: Mu(t) = base_u + sum_m (cos(w_m t) cu_m + sin(w_m t) su_m) on open
    east faces (likewise Mv on open north faces, base_v = 0), zero on faces
    that touch land or close the domain.  Fields are [n], stored at the cell
    west (east faces) or south (north faces) of the face."""
    w: list
    base_u: np.ndarray
    cu: list
    su: list
    cv: list
    sv: list
    e2u: np.ndarray           # east-face metric factor e2 = dphi (radius dropped)
    e1v: np.ndarray           # north-face metric factor e1 = cos(phi) dlam


def orca_transport_modes(p: Problem, seed: int) -> TransportModes:
    """A zonal band flow plus four planetary-scale modes travelling slowly in
    time (periods of 150-400 steps), seeded; see TransportModes."""
    nx, ny = p.nx, p.ny
    geo = orca_geometry(nx, ny)
    rng = np.random.default_rng(seed)
    ocean = p.ocean.reshape(ny, nx)
    open_e = (ocean & np.roll(ocean, -1, axis=1)).ravel()       # periodic in longitude
    open_n = np.zeros_like(ocean)
    open_n[:-1, :] = ocean[:-1, :] & ocean[1:, :]
    open_n = open_n.ravel()
    lam_e = geo.lam + 0.5 * geo.dlam                           # east-face longitudes
    phi_n = geo.phi_f[1:]                                      # north-face latitudes
    base_u = np.where(open_e, (0.8 * np.cos(3.0 * geo.phi_c)[:, None] * np.ones((1, nx))).ravel(), 0.0)
    w, cu, su, cv, sv = [], [], [], [], []
    for _ in range(4):
        k = int(rng.integers(1, 6))
        l = int(rng.integers(1, 5))
        amp = rng.uniform(0.2, 0.6)
        w.append(2.0 * np.pi / rng.uniform(150.0, 400.0))
        ps = rng.uniform(0.0, 2.0 * np.pi)
        # cos(k lam - w t + ps) = cos(w t) cos(k lam + ps) + sin(w t) sin(k lam + ps)
        # sin(k lam - w t + ps) = cos(w t) sin(k lam + ps) - sin(w t) cos(k lam + ps)
        su_amp = amp * np.sin(l * geo.phi_c)[:, None]
        sv_amp = amp * np.cos(l * phi_n)[:, None]
        ce, se = np.cos(k * lam_e + ps)[None, :], np.sin(k * lam_e + ps)[None, :]
        cc, sc = np.cos(k * geo.lam + ps)[None, :], np.sin(k * geo.lam + ps)[None, :]
        cu.append(np.where(open_e, (su_amp * ce).ravel(), 0.0))
        su.append(np.where(open_e, (su_amp * se).ravel(), 0.0))
        cv.append(np.where(open_n, (sv_amp * sc).ravel(), 0.0))
        sv.append(np.where(open_n, (-sv_amp * cc).ravel(), 0.0))
    e2u = np.full(nx * ny, geo.dphi)
    e1v = np.repeat(geo.cos_f[1:] * geo.dlam, nx)
    return TransportModes(w, base_u, cu, su, cv, sv, e2u, e1v)


def combine_transports(m: TransportModes, t: int):
    """(Mu, Mv) of time step t from the modes."""
    mu = m.base_u.copy()
    mv = np.zeros_like(m.base_u)
    for w, cu, su, cv, sv in zip(m.w, m.cu, m.su, m.cv, m.sv):
        c, s = math.cos(w * t), math.sin(w * t)
        mu += c * cu + s * su
        mv += c * cv + s * sv
    return mu, mv


def orca_transports(p: Problem, t: int, seed: int):
    """Synthetic face transports of time step t for the right-hand side of
    eq. (8) (see orca_transport_modes).  Returns (e2u, mu, e1v, mv), each
    [nx*ny]: east-face metric factor e2 = dphi and transport Mu (at the cell
    west of the face), north-face metric factor e1 = cos(phi) dlam and
    transport Mv (at the cell south of the face); the radius is dropped as in
    the operator's coefficients."""
    m = orca_transport_modes(p, seed)
    mu, mv = combine_transports(m, t)
    return m.e2u, mu, m.e1v, mv
