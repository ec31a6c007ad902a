"""Seeded synthetic inputs for the D3Q19 moving-particle sweep.

This module only *generates inputs*: sphere positions and radii (random
sequential addition), prescribed particle velocities, wall flags and the
charge density rho_e of the electric double layer around each sphere.  It
holds none of the lattice Boltzmann arithmetic, so both the CPU oracle and
the GPU library consume exactly the same arrays.

The workloads follow the shape of the paper's performance runs (Sec.
"Parallel Performance and Scaling": a block of cells with equally sized
spheres, about 2 % solid volume, a few hundred time steps) scaled to one
GPU.  The paper has no dataset; everything here is synthetic.

Charge density ("Gaussian shell"): the paper gets rho_e from the
Debye-Hueckel solution (Sec. "Electrophoresis"); the LBM sweep only needs
the resulting body force f_b = rho_e * E as an input.  As a stand-in with
the same support and decay length we use

    rho_e(x) = A * sum_p exp(-(d_p - R_p)^2 / (2 lambda_D^2)),

for d_p = |x - X_p| (minimum image) with 0 <= d_p - R_p <= 6 lambda_D,
zero inside spheres and beyond the cutoff.
"""
from __future__ import annotations

import dataclasses
import numpy as np

# user flag values (the C-ABI's LBMEP_FLUID / LBMEP_WALL)
FLUID = 0
WALL = 1


@dataclasses.dataclass
class Workload:
    """One complete synthetic problem: grid, walls, particles, force."""
    name: str
    shape: tuple            # (nx, ny, nz)
    periodic: tuple         # (px, py, pz) booleans
    nu: float
    magic: float
    flags: np.ndarray       # uint8 (nz, ny, nx), x fastest; 0 fluid / 1 wall
    X: np.ndarray           # (n, 3) float64 initial centres
    R: np.ndarray           # (n,) float64 radii
    U: np.ndarray           # (n, 3) float64 translational velocities
    W: np.ndarray           # (n, 3) float64 angular velocities
    moving: bool
    rho_e: np.ndarray | None  # (nz, ny, nx) float64 charge density, or None
    E: tuple                # uniform applied field
    fb: np.ndarray | None   # (3, nz, ny, nx) float64 dense force, or None
    steps: int
    precision: str          # "fp64" | "fp32dev" | "fp16dev"

    @property
    def ncells(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    def dense_force(self):
        """The per-cell body force as a dense SoA (3, nz, ny, nx) array."""
        if self.fb is not None:
            return self.fb
        nx, ny, nz = self.shape
        out = np.zeros((3, nz, ny, nx))
        if self.rho_e is not None:
            for a in range(3):
                out[a] = self.rho_e * self.E[a]
        return out


def _min_image(d, L, periodic):
    if periodic:
        d = d - L * np.round(d / L)
    return d


def rsa_spheres(rng, n, radius, shape, periodic, gap, lo=None, hi=None,
                max_tries=1000, strict=True):
    """Random sequential addition of n spheres.

    radius: scalar or callable(rng) -> radius.  gap: minimum surface gap
    (centre distance >= R_a + R_b + gap, minimum image on periodic axes).
    lo/hi: per-axis bounds for centres (defaults [0, L)).  Returns (X, R);
    if strict is False, spheres that cannot be placed in max_tries are
    dropped (their count is len(requested) - len(returned)).
    """
    L = np.asarray(shape, dtype=np.float64)
    lo = np.zeros(3) if lo is None else np.asarray(lo, dtype=np.float64)
    hi = L.copy() if hi is None else np.asarray(hi, dtype=np.float64)
    Xs, Rs = [], []
    for _ in range(n):
        r = float(radius(rng)) if callable(radius) else float(radius)
        placed = False
        for _ in range(max_tries):
            c = lo + (hi - lo) * rng.random(3)
            ok = True
            for Xo, Ro in zip(Xs, Rs):
                d = np.array([_min_image(c[a] - Xo[a], L[a], periodic[a]) for a in range(3)])
                if np.sqrt((d * d).sum()) < r + Ro + gap:
                    ok = False
                    break
            if ok:
                Xs.append(c)
                Rs.append(r)
                placed = True
                break
        if not placed and strict:
            raise RuntimeError("random sequential addition failed to place a sphere")
    X = np.array(Xs, dtype=np.float64).reshape(-1, 3)
    return X, np.array(Rs, dtype=np.float64)


def rsa_spheres_grid(rng, n, radius, shape, gap, max_tries=1000):
    """Fast RSA for many equal spheres in a fully periodic box (cell lists)."""
    L = np.asarray(shape, dtype=np.float64)
    cell = 2.0 * radius + gap
    nb = np.maximum(1, np.floor(L / cell).astype(int))
    bins = {}
    Xs = []
    for _ in range(n):
        for _ in range(max_tries):
            c = L * rng.random(3)
            b = tuple((c / L * nb).astype(int) % nb)
            ok = True
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        key = ((b[0] + dx) % nb[0], (b[1] + dy) % nb[1], (b[2] + dz) % nb[2])
                        for j in bins.get(key, ()):
                            d = c - Xs[j]
                            d = d - L * np.round(d / L)
                            if (d * d).sum() < cell * cell:
                                ok = False
                                break
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                bins.setdefault(b, []).append(len(Xs))
                Xs.append(c)
                break
        else:
            raise RuntimeError("random sequential addition failed to place a sphere")
    return np.array(Xs, dtype=np.float64), np.full(n, float(radius))


def gaussian_shell_rho_e(shape, periodic, X, R, lambda_d=2.0, amp=1e-5, cutoff=6.0):
    """Charge density of a Gaussian shell around every sphere (see module doc).

    Returned as float64 (nz, ny, nx).  Cell centres sit at i + 1/2.
    """
    nx, ny, nz = shape
    L = (nx, ny, nz)
    rho = np.zeros((nz, ny, nx), dtype=np.float64)
    for p in range(len(R)):
        reach = R[p] + cutoff * lambda_d
        idx = []
        for a in range(3):
            lo = int(np.floor(X[p, a] - reach)) - 1
            hi = int(np.floor(X[p, a] + reach)) + 1
            ii = np.arange(lo, hi + 1)
            if periodic[a]:
                if len(ii) >= L[a]:
                    ii = np.arange(L[a])
                else:
                    ii = ii % L[a]
            else:
                ii = ii[(ii >= 0) & (ii < L[a])]
            idx.append(ii)
        d = []
        for a in range(3):
            da = idx[a] + 0.5 - X[p, a]
            d.append(_min_image(da, L[a], periodic[a]))
        dz2 = d[2][:, None, None] ** 2
        dy2 = d[1][None, :, None] ** 2
        dx2 = d[0][None, None, :] ** 2
        dist = np.sqrt(dx2 + dy2 + dz2)
        s = dist - R[p]
        val = np.where((s >= 0.0) & (s <= cutoff * lambda_d),
                       amp * np.exp(-(s * s) / (2.0 * lambda_d * lambda_d)), 0.0)
        rho[np.ix_(idx[2], idx[1], idx[0])] += val
    return rho


def debye_huckel_psi(shape, periodic, X, R, zeta, kappa=0.5, cutoff=12.0):
    """EDL potential around every sphere: the Debye-Hueckel solution for a
    sphere of surface potential zeta_p (Sec. "Electrophoresis"),

        psi(x) = sum_p zeta_p (R_p / d_p) exp(-kappa (d_p - R_p)),

    for d_p = |x - X_p| (minimum image) with R_p <= d_p <= R_p + cutoff / kappa;
    zeta_p inside sphere p; zero beyond the cutoff.  Returned as float64
    (nz, ny, nx), cell centres at i + 1/2.  The same field is the input of
    both the CPU oracle and the library.
    """
    nx, ny, nz = shape
    L = (nx, ny, nz)
    psi = np.zeros((nz, ny, nx), dtype=np.float64)
    for p in range(len(R)):
        reach = R[p] + cutoff / kappa
        idx = []
        for a in range(3):
            lo = int(np.floor(X[p, a] - reach)) - 1
            hi = int(np.floor(X[p, a] + reach)) + 1
            ii = np.arange(lo, hi + 1)
            if periodic[a]:
                ii = np.arange(L[a]) if len(ii) >= L[a] else ii % L[a]
            else:
                ii = ii[(ii >= 0) & (ii < L[a])]
            idx.append(ii)
        d = [_min_image(idx[a] + 0.5 - X[p, a], L[a], periodic[a]) for a in range(3)]
        dist = np.sqrt(d[2][:, None, None] ** 2 + d[1][None, :, None] ** 2
                       + d[0][None, None, :] ** 2)
        val = np.where(dist < R[p], zeta[p],
                       np.where(dist <= reach,
                                zeta[p] * (R[p] / np.maximum(dist, R[p]))
                                * np.exp(-kappa * (np.maximum(dist, R[p]) - R[p])), 0.0))
        psi[np.ix_(idx[2], idx[1], idx[0])] += val
    return psi


def channel_flags(shape, wall_axis=1):
    """WALL cells on the first and last layer along wall_axis (0=x,1=y,2=z)."""
    nx, ny, nz = shape
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    if wall_axis == 1:
        f[:, 0, :] = WALL
        f[:, ny - 1, :] = WALL
    elif wall_axis == 0:
        f[:, :, 0] = WALL
        f[:, :, nx - 1] = WALL
    else:
        f[0] = WALL
        f[nz - 1] = WALL
    return f


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def sphere_at_centre(n=32, R=4.0, fb=1e-6, steps=200, nu=1.0 / 6.0):
    """Periodic n^3 box, one fixed sphere at the box centre (a cell corner),
    uniform force along x on fluid cells, FP64."""
    shape = (n, n, n)
    fbx = np.zeros((3, n, n, n))
    fbx[0] = fb
    return Workload(
        name=f"sphere{n}", shape=shape, periodic=(True, True, True),
        nu=nu, magic=3.0 / 16.0,
        flags=np.zeros((n, n, n), dtype=np.uint8),
        X=np.array([[n / 2, n / 2, n / 2]], dtype=np.float64),
        R=np.array([R]), U=np.zeros((1, 3)), W=np.zeros((1, 3)),
        moving=False, rho_e=None, E=(0.0, 0.0, 0.0), fb=fbx,
        steps=steps, precision="fp64")


def channel_spheres(n=128, count=64, R=6.0, seed=2, steps=1000, umax=1e-3,
                    precision="fp64"):
    """n^3 channel with no-slip walls at y=0 and y=n-1, periodic x and z,
    `count` moving spheres with a Gaussian-shell charge and E=(1e-3,0,0)."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    periodic = (True, False, True)
    lo = [0.0, 1.0 + R + 2.0, 0.0]
    hi = [float(n), n - 1.0 - R - 2.0, float(n)]
    X, Rs = rsa_spheres(rng, count, R, shape, periodic, gap=6.0, lo=lo, hi=hi)
    U = rng.uniform(-umax, umax, size=(count, 3))
    rho_e = gaussian_shell_rho_e(shape, periodic, X, Rs)
    return Workload(
        name=f"channel{n}", shape=shape, periodic=periodic,
        nu=1.0 / 6.0, magic=3.0 / 16.0, flags=channel_flags(shape),
        X=X, R=Rs, U=U, W=np.zeros((count, 3)), moving=True,
        rho_e=rho_e, E=(1e-3, 0.0, 0.0), fb=None, steps=steps,
        precision=precision)


def periodic_suspension(n=512, count=4096, R=4.0, seed=3, steps=500,
                        umax=5e-4, precision="fp32dev", with_rho_e=True):
    """Fully periodic n^3 box with `count` moving spheres of radius R placed
    with a surface gap of at least 3 cells; Gaussian-shell charge and
    E=(1e-3,0,0)."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    periodic = (True, True, True)
    X, Rs = rsa_spheres_grid(rng, count, R, shape, gap=3.0)
    U = rng.uniform(-umax, umax, size=(count, 3))
    rho_e = gaussian_shell_rho_e(shape, periodic, X, Rs) if with_rho_e else None
    return Workload(
        name=f"suspension{n}", shape=shape, periodic=periodic,
        nu=1.0 / 6.0, magic=3.0 / 16.0,
        flags=np.zeros((n, n, n), dtype=np.uint8),
        X=X, R=Rs, U=U, W=np.zeros((count, 3)), moving=True,
        rho_e=rho_e, E=(1e-3, 0.0, 0.0), fb=None, steps=steps,
        precision=precision)


def suspension_subrun(precision="fp32dev", steps=500):
    """The 128^3 sub-run of the 512^3 suspension: 64 spheres, seed 33."""
    return periodic_suspension(n=128, count=64, R=4.0, seed=33, steps=steps,
                               precision=precision)


SERVE_EDGES = (64, 96, 128, 192, 256)


def serving_request(r, base_seed=5_000_000):
    """Request r of the serving mix: random box edges, sphere count, radii
    and step count; fully periodic, FP32 deviation storage."""
    rng = np.random.default_rng(base_seed + r)
    shape = tuple(int(rng.choice(SERVE_EDGES)) for _ in range(3))
    steps = int(rng.integers(500, 5001))
    count = int(rng.integers(1, 201))
    periodic = (True, True, True)
    X, Rs = rsa_spheres(rng, count, lambda g: g.uniform(3.0, 8.0), shape,
                        periodic, gap=2.0, max_tries=1000, strict=False)
    k = len(Rs)
    U = rng.uniform(-5e-4, 5e-4, size=(k, 3))
    return dict(shape=shape, steps=steps, requested=count, X=X, R=Rs, U=U,
                W=np.zeros((k, 3)), periodic=periodic, E=(1e-3, 0.0, 0.0))


def random_state(rng, shape, base, amp=1e-2):
    """Random (non-physical) populations for brute-force comparisons:
    f_q = base_q * (1 + amp * U[-1, 1]) per cell, with base (19,) given by
    the caller.  Returned as float64 (19, nz, ny, nx)."""
    base = np.asarray(base, dtype=np.float64)
    nx, ny, nz = shape
    return base[:, None, None, None] * (1.0 + amp * rng.uniform(-1, 1, size=(19, nz, ny, nx)))
