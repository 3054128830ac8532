"""Seeded synthetic inputs for the NLSE  i Psi_t + a Lap Psi - V Psi + s |Psi|^2 Psi = 0.

This module is shared by the CPU oracle tests and by the GPU library's tests and
benchmark.  It builds grids, potentials V(r), initial fields Psi(r, 0) and the
analytic solutions the paper tests against.  It holds none of the numerical
method (no Laplacian, no time stepping, no step-size bound): only the problem
definitions.

Grid convention: ``n`` is the number of intervals per axis; there are ``n + 1``
nodes per axis including the two boundary nodes, node ``i`` sits at
``lo + i * h`` with ``h = (hi - lo) / n`` and the same ``h`` on every axis
(Sec. 2: the 2D and 3D stencils assume square / cubic cells).  Arrays are
C-ordered ``[z][y][x]`` (x fastest).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Grid", "grid", "bright_soliton", "dark_soliton", "gaussian_ho",
    "gp2d_vortex", "gp3d_ring", "gp2d_multivortex", "batch_instances",
    "ProblemSpec", "config_soliton_1d", "config_gp2d", "config_gp3d",
    "paper_fig1", "paper_fig2", "paper_fig3", "dark_plane", "background_vortices",
    "background_ring",
]


@dataclasses.dataclass(frozen=True)
class Grid:
    dim: int
    n: int          # intervals per axis
    lo: float
    hi: float

    @property
    def h(self) -> float:
        return (self.hi - self.lo) / self.n

    @property
    def nodes(self) -> int:
        return self.n + 1

    @property
    def shape(self) -> tuple:
        return (self.n + 1,) * self.dim

    def axis(self) -> np.ndarray:
        return self.lo + self.h * np.arange(self.n + 1, dtype=np.float64)

    def coords(self):
        """Coordinate arrays broadcast to ``shape`` in [z][y][x] order.

        Returns (x,) in 1D, (x, y) in 2D and (x, y, z) in 3D."""
        ax = self.axis()
        if self.dim == 1:
            return (ax,)
        if self.dim == 2:
            y, x = np.meshgrid(ax, ax, indexing="ij")
            return (x, y)
        z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
        return (x, y, z)

    def boundary_mask(self) -> np.ndarray:
        """True on nodes that lie on the domain boundary (any axis index 0 or n)."""
        m = np.zeros(self.shape, dtype=bool)
        for ax in range(self.dim):
            idx = [slice(None)] * self.dim
            idx[ax] = 0
            m[tuple(idx)] = True
            idx[ax] = self.n
            m[tuple(idx)] = True
        return m


def grid(dim: int, n: int, lo: float, hi: float) -> Grid:
    return Grid(dim, int(n), float(lo), float(hi))


# ---------------------------------------------------------------------------
# Analytic solutions (problem definitions, used as initial data at t = 0 and,
# in the tests, as exact references at later times).
# ---------------------------------------------------------------------------

def bright_soliton(x, t, a=1.0, s=1.0, eta=1.0, c=0.0, x0=0.0):
    """Travelling bright soliton of the focusing NLSE (s > 0, V = 0).

    Psi = sqrt(2a/s) eta sech(eta (x - x0 - c t)) exp(i[c x/(2a) + (a eta^2 - c^2/(4a)) t]).
    With a = s = eta = 1, c = 0.5 it starts as sqrt(2) sech(x) exp(0.25 i x)."""
    amp = math.sqrt(2.0 * a / s) * eta
    xi = eta * (x - x0 - c * t)
    phase = c * x / (2.0 * a) + (a * eta * eta - c * c / (4.0 * a)) * t
    return amp / np.cosh(xi) * np.exp(1j * phase)


def dark_soliton(x, t, a=1.0, s=-1.0, omega=-1.0, c=0.5, x0=0.0):
    """Co-moving dark soliton of the defocusing NLSE (Sec. 4.1, Eq. 1dmds).

    Psi = sqrt(Omega/s) tanh(sqrt(|Omega|/(2a)) (x - x0 - c t)) exp(i[c x/(2a) + (Omega - c^2/(4a)) t])."""
    amp = math.sqrt(omega / s)
    xi = math.sqrt(abs(omega) / (2.0 * a)) * (x - x0 - c * t)
    phase = c * x / (2.0 * a) + (omega - c * c / (4.0 * a)) * t
    return amp * np.tanh(xi) * np.exp(1j * phase)


def gaussian_ho(coords, t, a=1.0):
    """Linear (s = 0) Gaussian eigenstate of V = r^2 / a (Sec. 4.2-4.3, Eqs. 2dexpsol / 3dexpsol).

    Psi = exp(-r^2/(2a)) exp(-i d t) in d dimensions, with potential V = r^2 / a."""
    r2 = sum(c * c for c in coords)
    d = len(coords)
    return np.exp(-r2 / (2.0 * a)) * np.exp(-1j * d * t)


def gaussian_ho_potential(coords, a=1.0):
    return sum(c * c for c in coords) / a


def harmonic_potential(coords, omega):
    """V = 0.5 omega^2 r^2 (the trap of the Gross-Pitaevskii workloads)."""
    return 0.5 * omega * omega * sum(c * c for c in coords)


def _noise(rng, shape, sigma, interior_mask):
    g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return sigma * g * interior_mask


def gp2d_vortex(g: Grid, omega=0.05, mu=1.0, noise=1e-3, seed=2):
    """Singly charged vortex in a Thomas-Fermi cloud plus seeded complex noise.

    Psi0 = sqrt(max(mu - V, 0)) tanh(r) e^{i theta} + noise, noise = sigma (g1 + i g2),
    g ~ N(0,1) i.i.d. (numpy PCG64, given seed) on interior nodes only; boundary nodes 0.
    Returns (psi0 complex128, V float64)."""
    x, y = g.coords()
    V = harmonic_potential((x, y), omega)
    r = np.sqrt(x * x + y * y)
    th = np.arctan2(y, x)
    psi = np.sqrt(np.maximum(mu - V, 0.0)) * np.tanh(r) * np.exp(1j * th)
    interior = ~g.boundary_mask()
    if noise:
        psi = psi + _noise(np.random.default_rng(seed), g.shape, noise, interior)
    psi = np.where(interior, psi, 0.0)
    return psi.astype(np.complex128), V


def gp2d_multivortex(g: Grid, omega=0.05, mu=1.0, noise=1e-3, seed=0):
    """1-8 vortices of random charge sign at seeded positions inside 0.6 R_TF, TF cloud, noise."""
    rng = np.random.default_rng(seed)
    x, y = g.coords()
    V = harmonic_potential((x, y), omega)
    rtf = math.sqrt(2.0 * mu) / omega
    k = int(rng.integers(1, 9))
    psi = np.sqrt(np.maximum(mu - V, 0.0)).astype(np.complex128)
    for _ in range(k):
        rad = 0.6 * rtf * math.sqrt(rng.uniform())
        ang = rng.uniform(0, 2 * math.pi)
        xk, yk = rad * math.cos(ang), rad * math.sin(ang)
        sgn = 1.0 if rng.uniform() < 0.5 else -1.0
        dx, dy = x - xk, y - yk
        psi = psi * np.tanh(np.sqrt(dx * dx + dy * dy)) * np.exp(1j * sgn * np.arctan2(dy, dx))
    interior = ~g.boundary_mask()
    if noise:
        psi = psi + _noise(rng, g.shape, noise, interior)
    psi = np.where(interior, psi, 0.0)
    return psi.astype(np.complex128), V


def gp3d_ring(g: Grid, omega=0.1, mu=1.0, ring_radius=6.0):
    """Thomas-Fermi cloud times the phase of a vortex ring of given radius in the z = 0 plane.

    Psi0 = sqrt(max(mu - V, 0)) exp(i atan2(z, rho - R)), rho = sqrt(x^2 + y^2).
    Boundary nodes are 0.  Returns (psi0 complex128, V float64)."""
    x, y, z = g.coords()
    V = harmonic_potential((x, y, z), omega)
    rho = np.sqrt(x * x + y * y)
    psi = np.sqrt(np.maximum(mu - V, 0.0)) * np.exp(1j * np.arctan2(z, rho - ring_radius))
    psi = np.where(g.boundary_mask(), 0.0, psi)
    return psi.astype(np.complex128), V


def dark_plane(dim, h, t=0.0, lo=-8.0, hi=8.0, width=2.0, x0=-6.5, a=0.5, s=-1.0, mu=1.0):
    """Stationary dark soliton plane of the defocusing NLSE (V = 0) in 1D, 2D or 3D.

    Psi = sqrt(mu/|s|) tanh(sqrt(mu/(2a)) (x - x0)) e^{-i mu t}, the same on every line along x
    (the c = 0 case of Eq. 1dmds with Omega = -mu).  x in [lo, hi], y and z in [0, width], step h.
    Its density never changes, so the modulus-squared Dirichlet (MSD) rule holds exactly on every
    face; with x0 near the x = lo face the density still varies steeply there.
    Returns (intervals per axis (nx[, ny[, nz]]), psi [z][y][x])."""
    nx, ny = int(round((hi - lo) / h)), int(round(width / h))
    x = lo + h * np.arange(nx + 1)
    prof = dark_soliton(x, t, a=a, s=s, omega=-mu, c=0.0, x0=x0)
    shape = (ny + 1,) * (dim - 1) + (nx + 1,)
    return (nx,) + (ny,) * (dim - 1), np.broadcast_to(prof, shape).astype(np.complex128)


def background_vortices(g: Grid, mu=1.0, s=-1.0, pairs=2, noise=1e-3, seed=0):
    """Vortex-antivortex pairs in a uniform background of density mu/|s| (V = 0), for the MSD rule.

    Psi0 = sqrt(mu/|s|) prod_k tanh(|r - r_k|) e^{+-i theta_k} + noise: `pairs` pairs with their
    centres at seeded positions within the inner 60 % of the box, one vortex of each charge 4 healing
    lengths apart; noise as in gp2d_vortex, on every node (the boundary evolves under MSD)."""
    rng = np.random.default_rng(seed)
    x, y = g.coords()
    psi = np.full(g.shape, math.sqrt(mu / abs(s)), dtype=np.complex128)
    half = 0.3 * (g.hi - g.lo)
    mid = 0.5 * (g.hi + g.lo)
    for _ in range(pairs):
        cx, cy = mid + rng.uniform(-half, half), mid + rng.uniform(-half, half)
        ang = rng.uniform(0, 2 * math.pi)
        for sgn in (1.0, -1.0):
            xk, yk = cx + sgn * 2.0 * math.cos(ang), cy + sgn * 2.0 * math.sin(ang)
            dx, dy = x - xk, y - yk
            psi = psi * np.tanh(np.sqrt(dx * dx + dy * dy)) * np.exp(1j * sgn * np.arctan2(dy, dx))
    if noise:
        psi = psi + _noise(rng, g.shape, noise, np.ones(g.shape))
    return psi.astype(np.complex128)


def background_ring(g: Grid, mu=1.0, s=-1.0, ring_radius=4.0):
    """Vortex ring of given radius in the z = 0 plane in a uniform background (V = 0), 3D.

    Psi0 = sqrt(mu/|s|) tanh(d) e^{i atan2(z, rho - R)}, d the distance to the ring's core line."""
    x, y, z = g.coords()
    rho = np.sqrt(x * x + y * y)
    d = np.sqrt((rho - ring_radius) ** 2 + z * z)
    psi = math.sqrt(mu / abs(s)) * np.tanh(d) * np.exp(1j * np.arctan2(z, rho - ring_radius))
    return psi.astype(np.complex128)


# ---------------------------------------------------------------------------
# Workload definitions
# ---------------------------------------------------------------------------

def smooth_random_3d(n, seed, boundary_amp=0.0):
    """A smooth complex test field on a 3D grid of n = (nx, ny, nz) intervals over the unit
    cube, stored [z][y][x]: four seeded plane-wave x standing-wave modes (wavenumbers 1-4 per
    axis, amplitudes 0.2-0.5), zero on the boundary, or, with boundary_amp, seeded Gaussian
    complex boundary values (fixed Dirichlet data).  Returns (psi, V) with the smooth
    potential V = 0.3 (x - 0.5)^2 + 0.2 (y - 0.4)^2 + 0.1 z."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*[np.linspace(0.0, 1.0, m + 1) for m in reversed(n)], indexing="ij")
    psi = np.zeros(x.shape, np.complex128)
    for _ in range(4):
        k = rng.uniform(1.0, 4.0, 3)
        ph = rng.uniform(0, 2 * np.pi, 3)
        psi += rng.uniform(0.2, 0.5) * np.exp(1j * (k[0] * 2 * np.pi * x + ph[0])) \
            * np.cos(k[1] * 2 * np.pi * y + ph[1]) * np.cos(k[2] * 2 * np.pi * z + ph[2])
    bnd = np.zeros(x.shape, bool)
    bnd[0, :, :] = bnd[-1, :, :] = bnd[:, 0, :] = bnd[:, -1, :] = bnd[:, :, 0] = bnd[:, :, -1] = True
    if boundary_amp:
        psi[bnd] = boundary_amp * (rng.standard_normal(bnd.sum()) + 1j * rng.standard_normal(bnd.sum()))
    else:
        psi[bnd] = 0.0
    V = 0.3 * (x - 0.5) ** 2 + 0.2 * (y - 0.4) ** 2 + 0.1 * z
    return psi, V


@dataclasses.dataclass
class ProblemSpec:
    """One NLSE problem: grid, coefficients, potential, initial field, boundary rule."""
    name: str
    grid: Grid
    a: float
    s: float
    V: np.ndarray | None
    psi0: np.ndarray
    bc: str = "dirichlet"          # or "msd"
    t_end: float | None = None
    steps: int | None = None

    @property
    def dim(self):
        return self.grid.dim

    @property
    def interior_points(self) -> int:
        return (self.grid.n - 1) ** self.grid.dim


def config_soliton_1d(n=1024):
    """1D bright soliton: a = s = 1, V = 0, x in [-50, 50], n intervals, Dirichlet 0, t_end = 10,
    Psi0 = sqrt(2) sech(x) exp(0.25 i x) (eta = 1, c = 0.5)."""
    g = grid(1, n, -50.0, 50.0)
    (x,) = g.coords()
    psi = bright_soliton(x, 0.0, a=1.0, s=1.0, eta=1.0, c=0.5)
    psi[0] = 0.0
    psi[-1] = 0.0
    return ProblemSpec("soliton1d", g, 1.0, 1.0, None, psi.astype(np.complex128), "dirichlet", 10.0)


def config_gp2d(n=2048, seed=2):
    """2D Gross-Pitaevskii: a = 0.5, s = -1, V = 0.5 (0.05)^2 r^2 on [-40, 40]^2, Dirichlet 0,
    vortex in a Thomas-Fermi cloud (mu = 1) plus 1e-3 complex Gaussian noise; 2000 RK4 steps."""
    g = grid(2, n, -40.0, 40.0)
    psi, V = gp2d_vortex(g, omega=0.05, mu=1.0, noise=1e-3, seed=seed)
    return ProblemSpec("gp2d", g, 0.5, -1.0, V, psi, "dirichlet", None, 2000)


def config_gp3d(n=512):
    """3D Gross-Pitaevskii: a = 0.5, s = -1, V = 0.5 (0.1)^2 r^2 on [-24, 24]^3, Dirichlet 0,
    Thomas-Fermi cloud (mu = 1) with the phase of a vortex ring of radius 6 at z = 0; 500 steps."""
    g = grid(3, n, -24.0, 24.0)
    psi, V = gp3d_ring(g, omega=0.1, mu=1.0, ring_radius=6.0)
    return ProblemSpec("gp3d", g, 0.5, -1.0, V, psi, "dirichlet", None, 500)


def paper_fig1(h, lo=-28.25, hi=28.25):
    """1D dark-soliton test (Sec. 4.1): s = -1, a = 1, c = 0.5, Omega = -1, MSD boundary,
    k = 0.0005 to t = 10.  The paper does not state the domain; a symmetric one is assumed."""
    n = int(round((hi - lo) / h))
    g = grid(1, n, lo, lo + n * h)
    (x,) = g.coords()
    psi = dark_soliton(x, 0.0, a=1.0, s=-1.0, omega=-1.0, c=0.5)
    return ProblemSpec("fig1", g, 1.0, -1.0, None, psi.astype(np.complex128), "msd", 10.0, 20000)


def paper_fig2(h, half=6.0):
    """2D linear Gaussian test (Sec. 4.2): a = 1, s = 0, V = (x^2+y^2)/a, Dirichlet, k = 0.001, t = 10."""
    n = int(round(2 * half / h))
    g = grid(2, n, -half, half)
    c = g.coords()
    psi = gaussian_ho(c, 0.0, a=1.0)
    return ProblemSpec("fig2", g, 1.0, 0.0, gaussian_ho_potential(c, 1.0), psi.astype(np.complex128),
                       "dirichlet", 10.0, 10000)


def paper_fig3(h, half=6.0):
    """3D linear Gaussian test (Sec. 4.3): a = 1, s = 0, V = r^2/a, Dirichlet, k = 0.0005, t = 10."""
    n = int(round(2 * half / h))
    g = grid(3, n, -half, half)
    c = g.coords()
    psi = gaussian_ho(c, 0.0, a=1.0)
    return ProblemSpec("fig3", g, 1.0, 0.0, gaussian_ho_potential(c, 1.0), psi.astype(np.complex128),
                       "dirichlet", 10.0, 20000)


def batch_instances(n1d=4096, n2d=256, seed=4, n_lo=256, n_hi=8192, n2d_grid=256):
    """Parameters of the batched workload: n1d independent 1D instances and n2d 2D instances.

    1D: n ~ U{n_lo..n_hi} intervals, s = +-1 (bright sech where s = +1, dark tanh where s = -1),
    eta ~ U[0.5, 2], c ~ U[-1, 1], a = 1, h = 0.125/eta, x in [-n h/2, n h/2]; bright instances
    use Dirichlet 0, dark instances the MSD boundary.
    2D: a = 0.5, s = -1, mu = 1, omega ~ U[0.02, 0.1], half-width 2 sqrt(mu)/omega, n2d_grid
    intervals, the vortex-plus-noise recipe.  Returns a list of ProblemSpec."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n1d):
        n = int(rng.integers(n_lo, n_hi + 1))
        s = 1.0 if rng.uniform() < 0.5 else -1.0
        eta = float(rng.uniform(0.5, 2.0))
        c = float(rng.uniform(-1.0, 1.0))
        h = 0.125 / eta
        g = grid(1, n, -0.5 * n * h, 0.5 * n * h)
        (x,) = g.coords()
        if s > 0:
            psi = bright_soliton(x, 0.0, a=1.0, s=1.0, eta=eta, c=c)
            psi[0] = 0.0
            psi[-1] = 0.0
            out.append(ProblemSpec(f"b1d_{i}", g, 1.0, 1.0, None, psi.astype(np.complex128), "dirichlet"))
        else:
            # dark soliton with width parameter eta: Omega = -2 a eta^2
            psi = dark_soliton(x, 0.0, a=1.0, s=-1.0, omega=-2.0 * eta * eta, c=c)
            out.append(ProblemSpec(f"d1d_{i}", g, 1.0, -1.0, None, psi.astype(np.complex128), "msd"))
    for j in range(n2d):
        om = float(rng.uniform(0.02, 0.1))
        half = 2.0 / om
        g = grid(2, n2d_grid, -half, half)
        psi, V = gp2d_vortex(g, omega=om, mu=1.0, noise=1e-3, seed=seed * 100003 + j)
        out.append(ProblemSpec(f"gp2d_{j}", g, 0.5, -1.0, V, psi, "dirichlet"))
    return out
