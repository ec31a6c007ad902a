"""GPU parity: the gfx950 library (through its C ABI) against the FP64 CPU
oracle on the same seeded inputs.

Bars: particle maps (flags, owners) bit-exact; FP64 populations, velocity,
density within 1e-12 relative (the FP64 sweep evaluates the oracle's
operation sequence, so the observed difference is normally 0); forces and
torques within 1e-12 relative (the library sums the deviation part of the
link terms in FP64 in a fixed order and the rest-weight part exactly as
integers; the oracle sums the plain link terms in long double with
compensated summation).
"""
import os

import numpy as np
import pytest

from paper_1708_08741_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available()
    from paper_1708_08741_amd import lbmep
    lbmep.lib()
    return lbmep


def _pair(lbm, oracle_mod, shape, periodic=(True, True, True), nu=1.0 / 6.0, magic=3.0 / 16.0,
          moving=False, precision=0):
    o = oracle_mod.Oracle(shape, periodic, nu, magic)
    g = lbm.Lattice(shape, periodic, nu, magic, precision, moving)
    return o, g


def _rel(a, b):
    s = np.abs(b).max()
    return np.abs(a - b).max() / (s if s > 0 else 1.0)


def _compare_fields(o, g, tol=TOL):
    rho_o, u_o = o.macro()
    rho_g, u_g = g.macro()
    assert np.abs(rho_g - rho_o).max() <= tol, np.abs(rho_g - rho_o).max()
    assert _rel(u_g, u_o) <= tol, _rel(u_g, u_o)


# ---------------------------------------------------------------------------
# brute force: random populations, forces and walls on tiny grids
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,periodic,walls,seed", [
    ((5, 4, 3), (True, True, True), False, 0),
    ((7, 6, 5), (True, True, True), True, 1),
    ((8, 5, 6), (False, True, True), False, 2),
    ((6, 7, 5), (True, False, False), True, 3),
    ((1, 1, 1), (True, True, True), False, 4),
    ((3, 1, 2), (True, True, False), False, 5),
    ((130, 5, 4), (True, True, True), True, 6),
    ((1100, 3, 2), (True, False, True), True, 7),
])
def test_brute_force_random_state(lb, oracle_mod, shape, periodic, walls, seed):
    """P11: random (non-physical) populations, random dense force and random
    walls; 1-3 steps; FP64 populations equal to the oracle within 1e-15."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    o, g = _pair(lb, oracle_mod, shape, periodic)
    f = W.random_state(rng, shape, oracle_mod.W, amp=0.05)
    fb = 1e-3 * rng.standard_normal((3, nz, ny, nx))
    fl = (rng.random((nz, ny, nx)) < (0.15 if walls else 0.0)).astype(np.uint8)
    for L in (o, g):
        L.set_flags(fl)
        L.set_force(fb)
        L.set_pdfs(f)
    for k in range(1, 4):
        o.step(1)
        g.step(1)
        fo, fg = o.get_pdfs(), g.get_pdfs()
        fluid = fl == 0
        d = np.abs(fg - fo)[:, fluid]
        assert d.max() <= 1e-15, (k, d.max())
    _compare_fields(o, g)
    fl_o, _ = o.map()
    fl_g, _ = g.map()
    assert (fl_o == fl_g).all()


# ---------------------------------------------------------------------------
# particle mapping: bit-exact flags and owners
# ---------------------------------------------------------------------------

def test_map_sphere_counts_and_wrap(lb, oracle_mod):
    """P12 on the GPU: R = 4, 6, 8 at cell corners and spheres across the
    periodic boundary; flags and owners bit-identical to the oracle."""
    L = 24
    X = np.array([[12.0, 12.0, 12.0], [0.3, 5.0, 23.9], [20.5, 0.2, 3.0]])
    R = np.array([4.0, 3.3, 2.7])
    U = np.zeros((3, 3))
    o, g = _pair(lb, oracle_mod, (L, L, L))
    o.set_particles(X, R, U)
    g.set_particles(X, R, U)
    fo, oo = o.map()
    fg, og = g.map()
    assert (fo == fg).all() and (oo == og).all()
    assert (fg == lb.OBST).sum() > 280


def test_map_overlap_and_walls(lb, oracle_mod):
    """Overlapping spheres (lowest index owns) and spheres cut by walls and
    non-periodic edges map identically."""
    shape = (20, 18, 16)
    flags = np.zeros((16, 18, 20), dtype=np.uint8)
    flags[:, 0, :] = 1
    flags[3:5, :, 7] = 1
    X = np.array([[5.0, 2.0, 3.0], [7.5, 3.0, 4.0], [19.7, 9.0, 15.2], [10.0, 17.4, 8.0]])
    R = np.array([3.0, 2.5, 2.2, 1.6])
    for per in [(True, False, True), (False, False, False)]:
        o, g = _pair(lb, oracle_mod, shape, per)
        for Lt in (o, g):
            Lt.set_flags(flags)
            Lt.set_particles(X, R, np.zeros((4, 3)))
        fo, oo = o.map()
        fg, og = g.map()
        assert (fo == fg).all() and (oo == og).all()


def test_map_moving_many_steps(lb, oracle_mod):
    """Maps after every step of fast-moving spheres (re-mapping, uncover /
    cover) stay bit-identical, including across the periodic boundary."""
    shape = (24, 20, 16)
    X = np.array([[2.0, 10.0, 8.0], [14.0, 4.0, 3.0], [20.0, 15.0, 12.5]])
    R = np.array([3.1, 2.4, 2.8])
    U = np.array([[-0.07, 0.01, 0.0], [0.05, 0.03, -0.04], [0.0, -0.06, 0.09]])
    Wv = np.array([[0.0, 0.0, 0.01], [0.02, 0.0, 0.0], [0.0, 0.0, 0.0]])
    o, g = _pair(lb, oracle_mod, shape, moving=True)
    rng = np.random.default_rng(9)
    fb = 1e-4 * rng.standard_normal((3, 16, 20, 24))
    for Lt in (o, g):
        Lt.set_force(fb)
        Lt.init_equilibrium()
    o.set_particles(X, R, U, Wv, moving=True)
    g.set_particles(X, R, U, Wv)
    for k in range(60):
        o.step(1)
        g.step(1)
        fo, oo = o.map()
        fg, og = g.map()
        assert (fo == fg).all(), k
        assert (oo == og).all(), k
    _compare_fields(o, g)
    Fo, Mo = o.ft()
    Fg, Mg = g.ft()
    assert _rel(Fg, Fo) <= TOL and _rel(Mg, Mo) <= TOL


@pytest.mark.parametrize("shape,periodic", [
    ((12, 10, 14), (True, True, True)),
    ((13, 12, 9), (True, False, True)),
])
def test_map_large_spheres_moving(lb, oracle_mod, shape, periodic):
    """Spheres as wide as the grid or reaching well past a face (boxes that
    span a whole periodic axis, boxes that wrap, a box cut by non-periodic
    edges), moving: flags and owners bit-identical to the oracle after every
    step, and the fields within the FP64 tolerance."""
    nx, ny, nz = shape
    X = np.array([[0.4, 0.6, 0.3], [nx - 0.7, ny / 2.0, nz - 0.2], [nx / 2.0, ny - 0.5, 1.1]])
    R = np.array([5.6, 3.2, 2.1])
    U = np.array([[-0.08, 0.05, 0.06], [0.07, -0.04, 0.09], [0.05, 0.08, -0.07]])
    Wv = np.array([[0.0, 0.01, 0.0], [0.0, 0.0, 0.02], [0.01, 0.0, 0.0]])
    o, g = _pair(lb, oracle_mod, shape, periodic, moving=True)
    for Lt in (o, g):
        Lt.init_equilibrium()
    o.set_particles(X, R, U, Wv, moving=True)
    g.set_particles(X, R, U, Wv)
    for k in range(25):
        o.step(1)
        g.step(1)
        fo, oo = o.map()
        fg, og = g.map()
        assert (fo == fg).all(), k
        assert (oo == og).all(), k
    _compare_fields(o, g)


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def test_sphere32_fixed_200_steps(lb, oracle_mod):
    """32^3 periodic box, one fixed R=4 sphere at the centre, f_b = 1e-6 x,
    nu = 1/6, Lambda = 3/16, 200 steps: u, rho and the drag match the
    oracle within 1e-12."""
    wl = W.sphere_at_centre()
    o = oracle_mod.from_workload(wl)
    from paper_1708_08741_amd import lbmep
    g = lbmep.from_workload(wl)
    o.step(wl.steps)
    g.step(wl.steps)
    _compare_fields(o, g)
    Fo, Mo = o.ft()
    Fg, Mg = g.ft()
    assert abs(Fg[0, 0] - Fo[0, 0]) <= TOL * abs(Fo[0, 0])
    assert np.abs(Fg - Fo).max() <= TOL * abs(Fo[0, 0])
    assert np.abs(Mg - Mo).max() <= TOL * abs(Fo[0, 0]) * 4.0
    fo, _ = o.map()
    fg, _ = g.map()
    assert (fo == fg).all()
    assert (fg == lb.OBST).sum() == 280 and (fg == lb.NEAR).sum() == 344


def test_channel128_moving_spheres(lb, oracle_mod):
    """128^3 channel (walls y=0,127), 64 moving R=6 spheres with the Gaussian
    shell charge and E=(1e-3,0,0), the configuration's 1000 steps against
    the oracle (fields, per-particle force/torque, maps, FP64 global sums),
    also checked after the first 100 steps."""
    wl = W.channel_spheres()
    steps = int(os.environ.get("LBMEP_CHANNEL_STEPS", str(wl.steps)))
    o = oracle_mod.from_workload(wl)
    from paper_1708_08741_amd import lbmep
    g = lbmep.from_workload(wl)
    done = 0
    for n in sorted({min(100, steps), steps}):
        o.step(n - done)
        g.step(n - done)
        done = n
        fo, oo = o.map()
        fg, og = g.map()
        assert (fo == fg).all() and (oo == og).all(), n
        _compare_fields(o, g)
        Fo, Mo = o.ft()
        Fg, Mg = g.ft()
        sF = np.abs(Fo).max()
        assert np.abs(Fg - Fo).max() <= TOL * sF, n
        assert np.abs(Mg - Mo).max() <= TOL * sF * 6.0, n
        # FP64 sums of mass and momentum over the fluid cells
        io, ig = o.invariants(), g.invariants()
        _, u = o.macro()
        fluid = (fo == lb.FLUID) | (fo == lb.NEAR)
        scale = fluid.sum() * np.abs(u[:, fluid]).max()
        assert abs(ig[0] - io[0]) <= TOL * io[0] and abs(ig[0] - io[0]) < 1e-9, n
        assert np.abs(ig[1:] - io[1:]).max() <= TOL * scale, n
    print("channel128 steps", done)
    g.close()


def test_channel128_full_run_conservation(lb):
    """The full 1000-step channel run on the GPU (beyond what the oracle
    finishes in seconds): the FP64 global sums stay finite, the mean fluid
    density stays rho0 (mass only moves through covered / uncovered cells,
    each carrying ~rho0), and the walls stay walls."""
    wl = W.channel_spheres()
    from paper_1708_08741_amd import lbmep
    g = lbmep.from_workload(wl)
    g.step(wl.steps)
    i1 = g.invariants()
    assert np.isfinite(i1).all()
    fl, _ = g.map()
    nfluid = ((fl == lb.FLUID) | (fl == lb.NEAR)).sum()
    assert abs(i1[0] / nfluid - 1.0) < 1e-6
    rho, u = g.macro()
    assert np.abs(u).max() < 5e-3
    assert ((fl == lb.WALL)[:, [0, 127], :]).all()
