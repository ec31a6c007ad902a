"""GPU parity of the electrostatic body force computed inside the sweep from
the EDL potential psi (Sec. "Computing Electrostatic Forces on Fluid and
Particles"): f_b = rho_e(psi) (E - grad psi) with rho_e = -kappa^2 eps psi
(Eq. ChrgDensDHA) and grad psi from Eq. ElPotGradComp away from boundaries,
the D3Q7 difference with boundary values next to them.

The oracle evaluates the same formula on the CPU in FP64.  Bars: FP64 fields,
forces and torques within 1e-12 relative; FP32 / FP16 deviation storage
(psi kept in FP32) within the tolerances of the charge-force runs of the same
storage (the potential adds an FP32 difference of neighbouring psi values,
a relative error of a few 1e-7 on the gradient).
"""
import numpy as np
import pytest

from paper_1708_08741_amd import workloads as W

pytestmark = pytest.mark.gpu

TOLS = {  # rho: absolute, or relative to max |u| where that is larger
    "fp64": dict(u=1e-12, rho=1e-12, rho_u=0.0, F=1e-12, M=1e-12),
    "fp32dev": dict(u=5e-6, rho=1e-8, rho_u=0.0, F=1e-5, M=1e-6),
    # FP16 rounds the stored deviations (which grow with |u|, here up to
    # 0.03) to 2^-11 relative, so the density bound scales with max |u|
    "fp16dev": dict(u=3e-3, rho=5e-6, rho_u=1e-3, F=5e-3, M=1e-3),
}
KEPS = 1e-3       # kappa^2 eps_e in lattice units
KAPPA = 0.5       # inverse Debye length (cells^-1)


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available()
    from paper_1708_08741_amd import lbmep
    lbmep.lib()
    return lbmep


def _fluid(o):
    from oracle import oracle as O
    fl, _ = o.map()
    return (fl == O.FLUID) | (fl == O.NEAR)


@pytest.mark.parametrize("shape,periodic,walls,with_zeta,seed", [
    ((13, 11, 9), (True, True, True), False, True, 0),
    ((12, 10, 14), (False, True, False), True, True, 1),
    ((131, 7, 6), (True, False, True), True, False, 2),
    ((9, 8, 7), (False, False, False), False, False, 3),
    ((1, 1, 1), (True, True, True), False, False, 4),
    # even nx (colour-split psi) with odd periodic extents: across the wrap a
    # neighbour has the cell's own colour
    ((12, 9, 7), (True, True, True), True, True, 5),
    ((20, 7, 10), (True, True, False), False, True, 6),
])
def test_force_at_rest(lb, oracle_mod, shape, periodic, walls, with_zeta, seed):
    """At rest (rho = 1, u = 0) the read-out velocity is f_b / 2 at fluid
    cells: a direct comparison of the force stencil on random potentials,
    random walls, spheres (with and without a surface potential) and
    non-periodic edges; FP64 within 1e-12, FP32 within 1e-6 of max |f_b|."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    psi = 0.05 * rng.standard_normal((nz, ny, nx))
    fl = (rng.random((nz, ny, nx)) < (0.12 if walls else 0.0)).astype(np.uint8)
    n = 2 if min(shape) >= 6 else 0
    X = np.column_stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(0, nz, n)])
    R = rng.uniform(1.2, 2.5, n)
    zeta = rng.uniform(-0.1, 0.1, n) if with_zeta and n else None
    E = (1e-2, -2e-2, 5e-3)
    o = oracle_mod.Oracle(shape, periodic)
    o.set_flags(fl)
    o.set_particles(X, R, np.zeros((n, 3)), moving=False)
    o.set_potential_force(psi, KEPS, E, zeta)
    o.init_equilibrium()
    fb = o.force()
    rho_o, u_o = o.macro()
    fluid = _fluid(o)
    assert np.abs(fb[:, fluid]).max() > 0
    for prec, tol in ((lb.FP64, 1e-12), (lb.FP32DEV, 1e-6)):
        g = lb.Lattice(shape, periodic, precision=prec)
        g.set_flags(fl)
        g.set_particles(X, R, np.zeros((n, 3)))
        g.set_potential_force(psi, KEPS, E, zeta)
        g.init_equilibrium()
        rho_g, u_g = g.macro()
        fo, oo = o.map()
        fg, og = g.map()
        assert (fg == fo).all() and (og == oo).all()
        s = np.abs(u_o[:, fluid]).max()
        assert np.abs(u_g - u_o)[:, fluid].max() <= tol * s, prec
        assert np.abs(2.0 * u_o[:, fluid] - fb[:, fluid]).max() <= 1e-15 * s
        g.close()


@pytest.mark.parametrize("shape,periodic,seed", [
    ((16, 10, 8), (True, True, True), 21),    # even periodic extents: the sweep's fast stencil
    ((12, 9, 7), (True, True, True), 22),     # odd periodic ny, nz: across a wrap a neighbour
    ((20, 7, 10), (True, True, False), 23),   # keeps the cell's colour
])
def test_force_in_the_sweep(lb, oracle_mod, shape, periodic, seed):
    """A few collisions with the force from a random potential (random walls,
    spheres with a surface potential): the sweep's force agrees with the
    oracle, on even nx with even and with odd periodic extents (the
    precisions' tolerances of u relative to max |u| and of rho)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    psi = 0.05 * rng.standard_normal((nz, ny, nx))
    fl = (rng.random((nz, ny, nx)) < 0.05).astype(np.uint8)
    X = np.column_stack([rng.uniform(0, nx, 2), rng.uniform(0, ny, 2), rng.uniform(0, nz, 2)])
    R = rng.uniform(1.2, 2.0, 2)
    zeta = rng.uniform(-0.1, 0.1, 2)
    E = (1e-2, -2e-2, 5e-3)
    steps = 4
    o = oracle_mod.Oracle(shape, periodic)
    o.set_flags(fl)
    o.set_particles(X, R, np.zeros((2, 3)), moving=False)
    o.set_potential_force(psi, KEPS, E, zeta)
    o.init_equilibrium()
    o.step(steps)
    rho_o, u_o = o.macro()
    fluid = _fluid(o)
    s = np.abs(u_o[:, fluid]).max()
    assert s > 0
    for prec, name in ((lb.FP64, "fp64"), (lb.FP32DEV, "fp32dev")):
        g = lb.Lattice(shape, periodic, precision=prec)
        g.set_flags(fl)
        g.set_particles(X, R, np.zeros((2, 3)))
        g.set_potential_force(psi.astype(np.float64 if prec == lb.FP64 else np.float32), KEPS, E, zeta)
        g.init_equilibrium()
        g.step(steps)
        rho_g, u_g = g.macro()
        g.close()
        assert np.abs(u_g - u_o)[:, fluid].max() <= TOLS[name]["u"] * s, name
        assert np.abs(rho_g - rho_o)[fluid].max() <= TOLS[name]["rho"], name


SHAPE, PER = (70, 44, 38), (True, False, True)


def _edl_inputs():
    """Channel (walls at y = 0, ny-1; periodic x, z) with moving charged
    spheres, their Debye-Hueckel potential held fixed as the input."""
    rng = np.random.default_rng(11)
    R0 = 4.0
    X, R = W.rsa_spheres(rng, 5, R0, SHAPE, PER, gap=3.0, lo=[0.0, 1.0 + R0 + 2.0, 0.0],
                         hi=[70.0, 44 - 2.0 - R0 - 2.0, 38.0])
    U = rng.uniform(-0.02, 0.02, size=(len(R), 3))
    Wv = rng.uniform(-2e-3, 2e-3, size=(len(R), 3))
    zeta = rng.uniform(-0.08, 0.08, len(R))
    psi = W.debye_huckel_psi(SHAPE, PER, X, R, zeta, kappa=KAPPA)
    return dict(X=X, R=R, U=U, W=Wv, zeta=zeta, psi=psi, E=(5e-3, 0.0, -2e-3),
                flags=W.channel_flags(SHAPE), R0=R0)


def _edl_lattice(lbm, precision, q):
    g = lbm.Lattice(SHAPE, PER, precision=precision, move_particles=True)
    g.set_flags(q["flags"])
    g.set_particles(q["X"], q["R"], q["U"], q["W"])
    g.set_potential_force(q["psi"].astype(np.float64 if precision == lbm.FP64 else np.float32),
                          KEPS, q["E"], q["zeta"])
    g.init_equilibrium()
    return g


def _edl_case(precision, lbm, oracle_mod, steps):
    q = _edl_inputs()
    o = oracle_mod.Oracle(SHAPE, PER)
    o.set_flags(q["flags"])
    o.set_particles(q["X"], q["R"], q["U"], q["W"], moving=True)
    o.set_potential_force(q["psi"], KEPS, q["E"], q["zeta"])
    o.init_equilibrium()
    o.step(steps)
    g = _edl_lattice(lbm, precision, q)
    g.step(steps)
    return o, g, q["R0"]


@pytest.mark.parametrize("precision", ["fp64", "fp32dev", "fp16dev"])
def test_moving_charged_spheres(lb, oracle_mod, precision):
    """30 steps of moving spheres in a walled channel driven by the EDL
    force: maps bit-exact, fields / forces / torques within the precision's
    tolerance of the FP64 oracle."""
    prec = {"fp64": lb.FP64, "fp32dev": lb.FP32DEV, "fp16dev": lb.FP16DEV}[precision]
    o, g, R0 = _edl_case(prec, lb, oracle_mod, 30)
    fo, oo = o.map()
    fg, og = g.map()
    assert (fg == fo).all() and (og == oo).all()
    fluid = _fluid(o)
    rho_o, u_o = o.macro()
    rho_g, u_g = g.macro()
    F_o, M_o = o.ft()
    F_g, M_g = g.ft()
    g.close()
    tol = TOLS[precision]
    umax = np.abs(u_o[:, fluid]).max()
    sF = np.linalg.norm(F_o, axis=1).max()
    err = dict(u=np.abs(u_g - u_o)[:, fluid].max() / umax,
               rho=np.abs(rho_g - rho_o)[fluid].max(),
               F=np.linalg.norm(F_g - F_o, axis=1).max() / sF,
               M=np.linalg.norm(M_g - M_o, axis=1).max() / (sF * R0))
    print(precision, "umax", umax, err)
    assert err["u"] <= tol["u"]
    assert err["rho"] <= max(tol["rho"], tol["rho_u"] * umax)
    assert err["F"] <= tol["F"]
    assert err["M"] <= tol["M"]


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_sweep_variants_identical(lb, monkeypatch, precision):
    """Launch-shape variants of the sweep in the potential mode (streaming
    hints, one or two cells per thread, block order) give bitwise the same
    run."""
    q = _edl_inputs()
    ref = None
    for env in [dict(), dict(LBMEP_SWEEP_NT="0"), dict(LBMEP_SWEEP_NT="1", LBMEP_CPT="2"),
                dict(LBMEP_SWEEP_NT="2", LBMEP_CPT="2"),
                dict(LBMEP_XCD_SWIZZLE="0", LBMEP_BLOCK_X="256")]:
        for k in ("LBMEP_SWEEP_NT", "LBMEP_CPT", "LBMEP_XCD_SWIZZLE", "LBMEP_BLOCK_X"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        g = _edl_lattice(lb, precision, q)
        g.step(13)
        out = (g.get_pdfs(), g.ft())
        g.close()
        if ref is None:
            ref = out
        else:
            assert (out[0] == ref[0]).all(), env
            assert (out[1][0] == ref[1][0]).all() and (out[1][1] == ref[1][1]).all(), env


def test_checkpoint_keeps_the_potential(lb, tmp_path):
    """save / load in the potential mode (psi, kappa^2 eps, E, zeta) and
    continue: bitwise the uninterrupted run."""
    g = _edl_lattice(lb, lb.FP32DEV, _edl_inputs())
    g.step(7)
    path = str(tmp_path / "pot.ck")
    g.save(path)
    g.step(9)
    ref = (g.get_pdfs(), g.ft())
    g.close()
    h = lb.Lattice(SHAPE, PER, precision=lb.FP32DEV, move_particles=True)
    h.load(path)
    h.step(9)
    out = (h.get_pdfs(), h.ft())
    h.close()
    assert (out[0] == ref[0]).all()
    assert (out[1][0] == ref[1][0]).all() and (out[1][1] == ref[1][1]).all()


@pytest.mark.parametrize("prec", ["fp32dev", "fp64"])
def test_checkpoint_restores_all_of_psi_into_a_used_lattice(lb, tmp_path, prec):
    """Loading into a lattice that already holds another potential: every
    value of psi comes from the file (even nx, so psi is colour-split, and
    N = 117040 is not a multiple of 128, so a colour's slots run past N):
    potential() and the continued run are bitwise the uninterrupted run."""
    P = {"fp32dev": lb.FP32DEV, "fp64": lb.FP64}[prec]
    q = _edl_inputs()
    nx, ny, nz = SHAPE
    assert nx % 2 == 0 and (nx * ny * nz) % 128 != 0
    g = _edl_lattice(lb, P, q)
    g.step(5)
    path = str(tmp_path / "pot2.ck")
    g.save(path)
    psi_saved = g.potential()
    g.step(6)
    ref = (g.get_pdfs(), g.potential(), g.ft())
    g.close()
    # a lattice with another potential and another state, then load
    rng = np.random.default_rng(99)
    other = dict(q)
    other["psi"] = 0.3 * rng.standard_normal(SHAPE[::-1])
    h = _edl_lattice(lb, P, other)
    h.step(3)
    h.load(path)
    assert (h.potential() == psi_saved).all()
    h.step(6)
    out = (h.get_pdfs(), h.potential(), h.ft())
    h.close()
    assert (out[0] == ref[0]).all() and (out[1] == ref[1]).all()
    assert (out[2][0] == ref[2][0]).all() and (out[2][1] == ref[2][1]).all()


@pytest.mark.parametrize("shape", [(8, 6, 4), (7, 6, 4), (130, 3, 5), (2, 1, 1), (1, 1, 1)])
def test_potential_storage_round_trip(lb, shape):
    """psi goes into its storage order on upload (colour-split for even nx,
    cell order for odd nx) and comes back in cell order: FP64 bitwise, FP32
    equal to the float32 rounding of the input."""
    rng = np.random.default_rng(3)
    psi = rng.standard_normal(shape[::-1])
    for prec in (lb.FP64, lb.FP32DEV):
        g = lb.Lattice(shape, precision=prec)
        g.set_potential_force(psi, KEPS, (0.0, 0.0, 0.0))
        out = g.potential()
        g.close()
        want = psi if prec == lb.FP64 else psi.astype(np.float32).astype(np.float64)
        assert np.array_equal(out.reshape(psi.shape), want), prec


def test_set_particles_drops_zeta(lb):
    """The surface potentials belong to the particle table they came with:
    after set_particles the obstacle cells give psi's own value."""
    shape = (20, 18, 16)
    rng = np.random.default_rng(5)
    psi = 0.05 * rng.standard_normal(shape[::-1])
    X = np.array([[10.0, 9.0, 8.0]])
    R = np.array([3.0])
    out = []
    for zeta in ([0.3], None):
        g = lb.Lattice(shape, precision=lb.FP64)
        g.set_particles(X, R, np.zeros((1, 3)))
        g.set_potential_force(psi, KEPS, (0.0, 0.0, 0.0), zeta)
        if zeta is not None:
            g.set_particles(X, R, np.zeros((1, 3)))
        g.init_equilibrium()
        out.append(g.macro()[1])
        g.close()
    assert (out[0] == out[1]).all()


def test_bad_arguments(lb):
    g = lb.Lattice((8, 8, 8), precision=lb.FP64)
    g.set_particles([[4.0, 4.0, 4.0]], [2.0], [[0.0, 0.0, 0.0]])
    psi = np.zeros((8, 8, 8))
    for kw in (dict(kappa2_eps=float("nan")), dict(E=(0.0, float("inf"), 0.0)),
               dict(zeta=[float("nan")])):
        args = dict(psi=psi, kappa2_eps=1e-3, E=(0.0, 0.0, 0.0), zeta=None)
        args.update(kw)
        with pytest.raises(lb.LbmepError) as e:
            g.set_potential_force(**args)
        assert e.value.code == lb.EINVAL
    bad = psi.copy()
    bad[1, 2, 3] = np.nan
    with pytest.raises(lb.LbmepError):
        g.set_potential_force(bad, 1e-3, (0.0, 0.0, 0.0))
    g.close()


# ---------------------------------------------------------------------------
# red-black SOR for the Debye-Hueckel equation of psi
# ---------------------------------------------------------------------------

def _sor_case(shape, periodic, walls, n, with_zeta, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    psi = 0.05 * rng.standard_normal((nz, ny, nx))
    fl = (rng.random((nz, ny, nx)) < (0.08 if walls else 0.0)).astype(np.uint8)
    X = np.column_stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(0, nz, n)])
    R = rng.uniform(1.5, 3.0, n)
    zeta = rng.uniform(-0.1, 0.1, n) if with_zeta and n else None
    return psi, fl, X, R, zeta


@pytest.mark.parametrize("shape,periodic,walls,n,with_zeta,rf,seed", [
    ((16, 12, 10), (True, True, True), False, 3, True, 0.0, 0),
    ((13, 12, 9), (False, True, False), True, 2, True, 0.0, 1),
    ((131, 6, 8), (False, True, True), True, 2, False, 0.0, 2),
    ((20, 18, 16), (True, False, True), False, 4, True, 1e-6, 3),
    ((9, 7, 5), (False, False, False), True, 1, True, 1e-9, 4),
    ((2, 2, 2), (True, True, True), False, 0, False, 0.0, 5),
    ((1030, 6, 4), (True, True, True), True, 3, True, 0.0, 6),
    ((516, 6, 5), (False, True, False), False, 2, False, 1e-5, 7),
    ((130, 37, 19), (True, False, False), True, 5, True, 0.0, 8),
    ((258, 34, 12), (True, True, True), False, 6, True, 1e-6, 9),
])
def test_sor_solve_matches_oracle(lb, oracle_mod, shape, periodic, walls, n, with_zeta, rf,
                                  seed):
    """One solve (fixed count, or to a residual reduction checked every 3
    iterations): FP64 psi, iteration count and residual norms equal to the
    oracle's (1e-12); FP32 psi within 1e-5 of max |psi|.  Ragged x extents
    (odd: the scalar rows in cell order; even: the z-marching tiles on the
    colour-split psi, several tiles per row), walls, particles with and
    without surface potentials, Neumann edges."""
    psi, fl, X, R, zeta = _sor_case(shape, periodic, walls, n, with_zeta, seed)
    kappa2, omega, iters = 0.3, 1.7, 40
    o = oracle_mod.Oracle(shape, periodic)
    o.set_flags(fl)
    o.set_particles(X, R, np.zeros((n, 3)), moving=False)
    o.set_potential_force(psi, KEPS, (0.0, 0.0, 0.0), zeta)
    o.set_potential_solver(kappa2, omega, iters, rf, 3)
    it_o, r0_o, r_o = o.solve_potential()
    psi_o = o.potential()
    s = np.abs(psi_o).max()
    for prec, tol in ((lb.FP64, 1e-12), (lb.FP32DEV, 1e-5)):
        g = lb.Lattice(shape, periodic, precision=prec)
        g.set_flags(fl)
        g.set_particles(X, R, np.zeros((n, 3)))
        g.set_potential_force(psi, KEPS, (0.0, 0.0, 0.0), zeta)
        g.set_potential_solver(kappa2, omega, iters, rf, 3)
        it_g, r0_g, r_g = g.solve_potential()
        psi_g = g.potential()
        g.close()
        err = np.abs(psi_g - psi_o).max()
        print(prec, it_g, it_o, r0_g, r0_o, r_g, r_o, err / s)
        assert err <= tol * s, (prec, err / s)
        if prec == lb.FP64:
            assert it_g == it_o
            if rf > 0:
                assert abs(r0_g - r0_o) <= 1e-12 * r0_o and abs(r_g - r_o) <= 1e-12 * r0_o
            else:
                assert r0_g == -1.0 and r_g == -1.0


@pytest.mark.parametrize("shape,periodic,n,rf,mzc,mrw", [
    ((130, 34, 70), (False, True, True), 6, 0.0, "16", "8"),
    ((64, 16, 32), (True, True, True), 3, 0.0, "5", "8"),
    ((66, 18, 34), (True, True, True), 4, 1e-3, "16", "8"),   # ny = 18: 2 rows per thread
    ((256, 12, 10), (True, True, False), 5, 0.0, "3", "8"),   # ny = 12: 4 rows per thread
    ((2048, 4, 6), (True, True, True), 3, 0.0, "4", "4"),     # 16 wavefronts per row
    ((128, 24, 22), (False, True, True), 5, 1e-3, "7", "4"),  # walls in every row
    ((384, 8, 12), (True, True, True), 4, 0.0, "5", "4"),     # 3 wavefronts per row
    ((2050, 4, 6), (True, True, True), 3, 0.0, "16", "8"),    # rows too long: two launches
    ((18, 6, 20), (False, False, False), 2, 0.0, "1", "2"),
    ((130, 35, 9), (True, False, False), 4, 0.0, "16", "8"),  # odd ny: one row per thread
    ((7, 5, 3), (False, False, False), 1, 0.0, "16", "8"),    # odd nx: cell order
    ((2, 2, 2), (True, True, True), 0, 0.0, "16", "8"),
    ((1, 1, 1), (False, False, False), 0, 0.0, "16", "8"),
])
@pytest.mark.parametrize("precision", [0, 1])
def test_sor_one_pass_equals_two_pass(lb, monkeypatch, shape, periodic, n, rf, mzc, mrw, precision):
    """The one-pass iteration (a z-march from psi into a second buffer
    between the red and black boundary lists) gives bitwise the psi and the
    iteration count of the in-place one-launch-per-colour form: chunks of 1,
    3, 4, 5 and 16 planes with ragged tails, 1, 2, 4 and 8 rows per thread,
    1 to 16 wavefronts per row, periodic wrap of every halo, walls,
    particles with and without surface potentials, non-periodic edges, tiny
    grids; odd and even iteration counts, with and without a residual stop."""
    psi, fl, X, R, zeta = _sor_case(shape, periodic, True, n, True, 9)
    out = {}
    monkeypatch.setenv("LBMEP_SOR_MZC", mzc)
    monkeypatch.setenv("LBMEP_SOR_MRW", mrw)
    for fused in ("1", "0"):
        monkeypatch.setenv("LBMEP_SOR_FUSED", fused)
        res = []
        for iters in (7, 8):
            g = lb.Lattice(shape, periodic, precision=precision)
            g.set_flags(fl)
            g.set_particles(X, R, np.zeros((n, 3)))
            g.set_potential_force(psi, KEPS, (0.0, 0.0, 0.0), zeta if iters == 7 else None)
            g.set_potential_solver(0.3, 1.7, iters, rf, 2)
            st = g.solve_potential()
            res.append((st, g.potential()))
            g.close()
        out[fused] = res
    for (st_f, p_f), (st_t, p_t) in zip(out["1"], out["0"]):
        assert st_f[0] == st_t[0]
        assert (p_f == p_t).all(), np.abs(p_f - p_t).max()


@pytest.mark.parametrize("shape,periodic,n", [
    ((130, 37, 19), (True, False, False), 5),
    ((64, 16, 32), (True, True, True), 3),
    ((258, 18, 9), (True, True, False), 4),
    ((1030, 12, 6), (True, True, True), 5),
    ((2, 2, 2), (True, True, True), 0),
    ((4, 40, 3), (False, False, False), 1),
])
@pytest.mark.parametrize("precision", [0, 1])
def test_sor_plane_chunks_identical(lb, monkeypatch, shape, periodic, n, precision):
    """The interior half-sweep marches each workgroup through a chunk of z
    planes (LBMEP_SOR_ZC planes, the window of three planes in registers):
    every chunk size, workgroup tile (LBMEP_SOR_WX waves along x,
    LBMEP_SOR_ROWS rows per thread), block order (LBMEP_SOR_XCD) and
    workgroup count of the boundary list part (LBMEP_SOR_NEARBLK) gives
    bitwise the same psi -- one plane per
    workgroup, chunks with ragged tails, one chunk over the whole grid --
    with several row segments and tiles with ragged ends, periodic wrap in
    z and y, walls and particles."""
    psi, fl, X, R, zeta = _sor_case(shape, periodic, True, n, True, 11)
    monkeypatch.setenv("LBMEP_SOR_FUSED", "0")  # the in-place half-sweeps
    ref = None
    for zc, wx, xcd, rows, nblk in (("1", "1", "0", "4", "8"), ("3", "1", "1", "4", "1024"),
                                    ("8", "2", "0", "4", "256"), ("1024", "4", "1", "4", "64"),
                                    ("5", "4", "0", "4", "2048"), ("8", "1", "1", "4", "256"),
                                    ("4", "4", "1", "8", "8"), ("3", "1", "0", "8", "512"),
                                    ("16", "2", "1", "8", "256")):
        monkeypatch.setenv("LBMEP_SOR_ZC", zc)
        monkeypatch.setenv("LBMEP_SOR_WX", wx)
        monkeypatch.setenv("LBMEP_SOR_XCD", xcd)
        monkeypatch.setenv("LBMEP_SOR_ROWS", rows)
        monkeypatch.setenv("LBMEP_SOR_NEARBLK", nblk)
        g = lb.Lattice(shape, periodic, precision=precision)
        g.set_flags(fl)
        g.set_particles(X, R, np.zeros((n, 3)))
        g.set_potential_force(psi, KEPS, (0.0, 0.0, 0.0), zeta)
        g.set_potential_solver(0.3, 1.7, 9, 0.0, 1)
        st = g.solve_potential()
        out = (st[0], g.potential())
        g.close()
        if ref is None:
            ref = out
        else:
            assert out[0] == ref[0]
            assert (out[1] == ref[1]).all(), (zc, np.abs(out[1] - ref[1]).max())


def _coupled_inputs():
    shape = (48, 36, 32)
    per = (True, False, True)
    rng = np.random.default_rng(21)
    R0 = 4.0
    X, R = W.rsa_spheres(rng, 4, R0, shape, per, gap=3.0, lo=[0.0, 1.0 + R0 + 2.0, 0.0],
                         hi=[48.0, 36 - 2.0 - R0 - 2.0, 32.0])
    U = rng.uniform(-0.03, 0.03, size=(len(R), 3))
    Wv = rng.uniform(-2e-3, 2e-3, size=(len(R), 3))
    zeta = rng.uniform(-0.08, 0.08, len(R))
    return dict(shape=shape, per=per, X=X, R=R, U=U, W=Wv, zeta=zeta, R0=R0,
                flags=W.channel_flags(shape), E=(5e-3, 0.0, -2e-3))


@pytest.mark.parametrize("precision,rf", [("fp64", 0.0), ("fp64", 1e-4), ("fp32dev", 0.0)])
def test_coupled_steps_with_per_step_solve(lb, oracle_mod, precision, rf):
    """Electrophoresis loop (Alg. 'Electrophoresis Algorithm'): before every
    collision the Debye-Hueckel equation is solved on the current map of
    the moving spheres (starting from the previous solution), and the
    collision uses the force of that potential.  25 steps from psi = 0:
    maps bit-exact; FP64 fields, forces, torques and potential within 1e-12
    of the oracle, FP32 within the charge-force tolerances."""
    q = _coupled_inputs()
    shape, per = q["shape"], q["per"]
    psi0 = np.zeros(shape[::-1])
    kappa2, iters, steps = 0.05, 12, 25
    o = oracle_mod.Oracle(shape, per)
    o.set_flags(q["flags"])
    o.set_particles(q["X"], q["R"], q["U"], q["W"], moving=True)
    o.set_potential_force(psi0, KEPS, q["E"], q["zeta"])
    o.set_potential_solver(kappa2, 1.7, iters, rf, 2)
    o.init_equilibrium()
    o.step(steps)
    prec = {"fp64": lb.FP64, "fp32dev": lb.FP32DEV}[precision]
    g = lb.Lattice(shape, per, precision=prec, move_particles=True)
    g.set_flags(q["flags"])
    g.set_particles(q["X"], q["R"], q["U"], q["W"])
    g.set_potential_force(psi0.astype(np.float64 if prec == lb.FP64 else np.float32), KEPS,
                          q["E"], q["zeta"])
    g.set_potential_solver(kappa2, 1.7, iters, rf, 2)
    g.init_equilibrium()
    g.step(steps)
    fo, oo = o.map()
    fg, og = g.map()
    assert (fg == fo).all() and (og == oo).all()
    fluid = _fluid(o)
    rho_o, u_o = o.macro()
    rho_g, u_g = g.macro()
    F_o, M_o = o.ft()
    F_g, M_g = g.ft()
    psi_o, psi_g = o.potential(), g.potential()
    st_o, st_g = o.solver_stats(), g.solver_stats()
    g.close()
    tol = TOLS[precision]
    umax = np.abs(u_o[:, fluid]).max()
    sF = np.linalg.norm(F_o, axis=1).max()
    err = dict(u=np.abs(u_g - u_o)[:, fluid].max() / umax,
               rho=np.abs(rho_g - rho_o)[fluid].max(),
               F=np.linalg.norm(F_g - F_o, axis=1).max() / sF,
               M=np.linalg.norm(M_g - M_o, axis=1).max() / (sF * q["R0"]),
               psi=np.abs(psi_g - psi_o).max() / np.abs(psi_o).max())
    print(precision, rf, st_g, st_o, err)
    assert err["u"] <= tol["u"]
    assert err["rho"] <= max(tol["rho"], tol["rho_u"] * umax)
    assert err["F"] <= tol["F"]
    assert err["M"] <= tol["M"]
    assert err["psi"] <= (1e-12 if precision == "fp64" else 1e-5)
    if precision == "fp64":
        assert st_g[0] == st_o[0]


def test_sor_bad_arguments(lb):
    g = lb.Lattice((6, 4, 4), precision=lb.FP64)
    with pytest.raises(lb.LbmepError) as e:
        g.set_potential_solver(0.2, 1.7, 3)  # no potential yet
    assert e.value.code == lb.EINVAL
    g.set_potential_force(np.zeros((4, 4, 6)), 1e-3, (0.0, 0.0, 0.0))
    for args in ((0.0, 1.7, 3), (0.2, 2.0, 3), (0.2, 1.7, -1), (float("nan"), 1.7, 3)):
        with pytest.raises(lb.LbmepError) as e:
            g.set_potential_solver(*args)
        assert e.value.code == lb.EINVAL
    with pytest.raises(lb.LbmepError):
        g.set_potential_solver(0.2, 1.7, 3, 0.0, 0)
    g.close()
    h = lb.Lattice((5, 4, 4), precision=lb.FP64)  # odd periodic extent
    h.set_potential_force(np.zeros((4, 4, 5)), 1e-3, (0.0, 0.0, 0.0))
    with pytest.raises(lb.LbmepError) as e:
        h.set_potential_solver(0.2, 1.7, 3)
    assert e.value.code == lb.EINVAL
    h.close()
    k = lb.Lattice((5, 4, 4), (False, True, True), precision=lb.FP64)
    k.set_potential_force(np.zeros((4, 4, 5)), 1e-3, (0.0, 0.0, 0.0))
    k.set_potential_solver(0.2, 1.7, 3)
    assert k.solve_potential()[0] == 3
    k.close()


def test_checkpoint_keeps_the_solver(lb, tmp_path):
    """save / load with a configured per-step solve: bitwise continuation."""
    q = _coupled_inputs()
    def make():
        g = lb.Lattice(q["shape"], q["per"], precision=lb.FP32DEV, move_particles=True)
        g.set_flags(q["flags"])
        g.set_particles(q["X"], q["R"], q["U"], q["W"])
        g.set_potential_force(np.zeros(q["shape"][::-1], np.float32), KEPS, q["E"], q["zeta"])
        g.set_potential_solver(0.05, 1.7, 6)
        g.init_equilibrium()
        return g
    g = make()
    g.step(5)
    path = str(tmp_path / "sor.ck")
    g.save(path)
    g.step(6)
    ref = (g.get_pdfs(), g.potential(), g.ft())
    g.close()
    h = lb.Lattice(q["shape"], q["per"], precision=lb.FP32DEV, move_particles=True)
    h.load(path)
    h.step(6)
    out = (h.get_pdfs(), h.potential(), h.ft())
    h.close()
    assert (out[0] == ref[0]).all() and (out[1] == ref[1]).all()
    assert (out[2][0] == ref[2][0]).all() and (out[2][1] == ref[2][1]).all()
