"""C-ABI behaviour on the GPU: checkpoint / resume, argument errors leave
the lattice unchanged, FP64 global sums (mass and momentum bookkeeping),
read-outs of solid cells, per-launch timing."""
import os

import numpy as np
import pytest

from paper_1708_08741_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available()
    from paper_1708_08741_amd import lbmep
    lbmep.lib()
    return lbmep


def _moving_case(lb, precision):
    shape = (40, 36, 32)
    rng = np.random.default_rng(21)
    X, R = W.rsa_spheres(rng, 5, 3.5, shape, (True, True, True), gap=3.0)
    U = rng.uniform(-0.02, 0.02, size=(5, 3))
    Wv = rng.uniform(-0.002, 0.002, size=(5, 3))
    rho_e = W.gaussian_shell_rho_e(shape, (True, True, True), X, R)
    g = lb.Lattice(shape, precision=precision, move_particles=True)
    g.set_charge_force(rho_e.astype(np.float64 if precision == lb.FP64 else np.float32),
                       (1e-2, 0.0, 0.0))
    g.init_equilibrium()
    g.set_particles(X, R, U, Wv)
    return g, (shape, X, R, U, Wv, rho_e)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_save_load_bitwise_continuation(lb, tmp_path, precision):
    """P14: N steps == k steps + save + load into a fresh lattice + N-k steps,
    bitwise in the populations, maps and read-outs."""
    a, _ = _moving_case(lb, precision)
    a.step(30)
    path = tmp_path / "ck.bin"
    a.save(str(path))
    a.step(25)
    b, _ = _moving_case(lb, precision)
    b.load(str(path))
    assert b.time == 30
    b.step(25)
    assert (a.get_pdfs() == b.get_pdfs()).all()
    fa, oa = a.map()
    fb, ob = b.map()
    assert (fa == fb).all() and (oa == ob).all()
    ra, ua = a.macro()
    rb, ub = b.macro()
    assert (ra == rb).all() and (ua == ub).all()
    Fa, Ma = a.ft()
    Fb, Mb = b.ft()
    assert np.allclose(Fa, Fb, rtol=0, atol=1e-15 * max(1e-30, np.abs(Fa).max()) + 1e-20)


def test_readouts_do_not_change_the_run(lb):
    """Reading the state between steps (which gathers the post-stream state)
    does not change the trajectory."""
    a, _ = _moving_case(lb, lb.FP32DEV)
    b, _ = _moving_case(lb, lb.FP32DEV)
    for _ in range(5):
        a.step(7)
        a.macro()
        a.invariants()
        a.get_pdfs()
    b.step(35)
    assert (a.get_pdfs() == b.get_pdfs()).all()


def test_argument_errors_leave_state_unchanged(lb):
    g, (shape, X, R, U, Wv, rho_e) = _moving_case(lb, lb.FP64)
    g.step(3)
    f0 = g.get_pdfs()
    m0 = g.map()
    bad = [
        lambda: g.set_particles(X, -R, U, Wv),
        lambda: g.set_particles(X * np.nan, R, U, Wv),
        lambda: g.set_particles(X, R, U + 2.0, Wv),  # moves >= 1 cell per step
        lambda: g.set_flags(np.full(shape[::-1], 7, dtype=np.uint8)),
        lambda: g.step(-1),
        lambda: g.init_equilibrium(1.0, (np.inf, 0, 0)),
        lambda: g.set_force(np.full((3,) + shape[::-1], np.nan)),
    ]
    for fn in bad:
        with pytest.raises(lb.LbmepError) as e:
            fn()
        assert e.value.code == lb.EINVAL
    assert (g.get_pdfs() == f0).all()
    m1 = g.map()
    assert (m0[0] == m1[0]).all() and (m0[1] == m1[1]).all()
    assert g.time == 3


def test_bad_config_rejected(lb):
    with pytest.raises(lb.LbmepError) as e:
        lb.Lattice((8, 8, 8), nu=-1.0)
    assert e.value.code == lb.EINVAL
    with pytest.raises(lb.LbmepError):
        lb.Lattice((8, 8, 8), device=99, stream=0)


def test_gpu_invariants_momentum_bookkeeping(lb):
    """T4: with a resting sphere the GPU's FP64 sums show exact mass
    conservation and dP = sum_fluid f_b - F per step (Eq. LBMhydrodynForce),
    the force summed by the momentum-exchange kernel."""
    n = 24
    rng = np.random.default_rng(4)
    fb = np.zeros((3, n, n, n))
    fb[0] = 2e-5
    fb[1] = 1e-5 * rng.standard_normal((n, n, n))
    g = lb.Lattice((n, n, n), precision=lb.FP64)
    g.set_force(fb)
    g.init_equilibrium()
    g.set_particles([[12.3, 11.7, 12.1]], [4.2], [[0, 0, 0]])
    fl, _ = g.map()
    fluid = (fl == lb.FLUID) | (fl == lb.NEAR)
    sfb = fb[:, fluid].sum(axis=1)
    for _ in range(4):
        i0 = g.invariants()
        g.step(1)
        i1 = g.invariants()
        F, _ = g.ft()
        assert abs(i1[0] - i0[0]) < 1e-13 * i0[0]
        assert np.allclose(i1[1:] - i0[1:], sfb - F[0], rtol=0, atol=1e-16 * n ** 3)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_nonfinite_populations_reported(lb, precision):
    """lbmep_get_invariants returns LBMEP_ENONFINITE when a population is
    NaN or infinite (a NaN planted through a device buffer, which
    lbmep_set_pdfs does not scan), and the library stays usable."""
    import torch
    shape = (12, 10, 8)
    g = lb.Lattice(shape, precision=precision)
    g.init_equilibrium()
    f = torch.from_numpy(g.get_pdfs()).cuda()
    f[7, 3, 4, 5] = float("nan")
    g.set_pdfs(f.reshape(-1))
    with pytest.raises(lb.LbmepError) as ei:
        g.invariants()
    assert ei.value.code == lb.ENONFINITE
    g.init_equilibrium()
    assert np.isfinite(g.invariants()).all()
    g.close()


def test_copy_reference(lb):
    """The achievable-bandwidth reference copy moves the bytes exactly and
    rejects sizes and pointers that are not multiples of 16 bytes."""
    import torch
    src = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    lb.copy_reference(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    assert lb.lib().lbmep_copy_reference(None, None, 16, None) == lb.EINVAL
    assert lb.lib().lbmep_copy_reference(dst.data_ptr(), src.data_ptr() + 4, 64, None) == lb.EINVAL
    assert lb.lib().lbmep_copy_reference(dst.data_ptr(), src.data_ptr(), 24, None) == lb.EINVAL


def test_solver_shape(lb):
    """The solver reports the one-pass iteration where it applies (even nx,
    rows of at most 2048 cells) and the in-place half-sweeps otherwise."""
    for shape, one in (((64, 12, 8), 1), ((63, 12, 8), 0), ((2050, 4, 4), 0)):
        g = lb.Lattice(shape, (True, True, True) if shape[0] % 2 == 0 else (False, True, True))
        g.set_potential_force(np.zeros(shape[::-1]), 1e-3, (0.0, 0.0, 0.0))
        g.set_potential_solver(0.2, 1.7, 2)
        sh = g.solver_shape()
        assert sh[0] == one, (shape, sh)
        if one:
            assert shape[1] % sh[1] == 0 and sh[3] == (shape[0] // 2 + 63) // 64
        g.close()


def test_macro_of_solid_cells(lb):
    """Obstacle cells report rho0 and their rigid-body surface velocity, wall
    cells rho0 and zero velocity."""
    shape = (16, 16, 16)
    flags = np.zeros((16, 16, 16), dtype=np.uint8)
    flags[:, 0, :] = 1
    g = lb.Lattice(shape, periodic=(True, False, True))
    g.set_flags(flags)
    g.init_equilibrium()
    X = np.array([[8.0, 8.0, 8.0]])
    U = np.array([[1e-3, -2e-3, 5e-4]])
    Wv = np.array([[0.0, 0.0, 1e-3]])
    g.set_particles(X, [3.0], U, Wv)
    rho, u = g.macro()
    fl, ow = g.map()
    obst = fl == lb.OBST
    assert obst.sum() > 0
    z, y, x = np.nonzero(obst)
    r = np.stack([x + 0.5, y + 0.5, z + 0.5], axis=1) - X
    us = U + np.cross(np.broadcast_to(Wv, r.shape), r)
    assert np.abs(u[:, obst].T - us).max() < 1e-18
    assert (rho[obst] == 1.0).all()
    assert (u[:, fl == lb.WALL] == 0).all() and (rho[fl == lb.WALL] == 1.0).all()


def test_timing_counts_launches(lb):
    g = lb.Lattice((64, 8, 8), precision=lb.FP32DEV)
    g.set_timing(True)
    g.step(12)
    ms, n = g.get_timing()
    assert n == 12 and ms > 0
    g.set_timing(False)
    g.step(3)
    ms, n = g.get_timing()
    assert n == 0


def test_empty_particle_table_and_zero_steps(lb):
    g = lb.Lattice((8, 8, 8), move_particles=True)
    g.init_equilibrium()
    g.set_particles(np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3)))
    f0 = g.get_pdfs()
    g.step(0)
    assert (g.get_pdfs() == f0).all()
    g.step(5)
    F, M = g.ft()
    assert F.shape == (0, 3)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_sweep_variants_identical(lb, monkeypatch, precision):
    """Launch-shape variants of the sweep (streaming hints on / off, one or
    two cells per thread, XCD block order, workgroups per CU capped) and the
    step with the next level's mapping on a second stream or in one stream
    compute bitwise the same run."""
    ref = None
    for env in [dict(), dict(LBMEP_STEP_OVERLAP="0"), dict(LBMEP_SWEEP_WGCU="0"),
                dict(LBMEP_SWEEP_WGCU="5"),
                dict(LBMEP_SWEEP_NT="0"), dict(LBMEP_SWEEP_NT="1"),
                dict(LBMEP_SWEEP_NT="2"), dict(LBMEP_SWEEP_NT="0", LBMEP_CPT="2"),
                dict(LBMEP_SWEEP_NT="1", LBMEP_CPT="2"), dict(LBMEP_SWEEP_NT="2", LBMEP_CPT="2"),
                dict(LBMEP_XCD_SWIZZLE="0", LBMEP_BLOCK_X="256"),
                dict(LBMEP_XCD_SWIZZLE="1", LBMEP_BLOCK_X="512")]:
        for k in ("LBMEP_SWEEP_NT", "LBMEP_CPT", "LBMEP_XCD_SWIZZLE", "LBMEP_BLOCK_X",
                  "LBMEP_SWEEP_WGCU", "LBMEP_STEP_OVERLAP"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        g, _ = _moving_case(lb, precision)
        g.step(17)
        out = (g.get_pdfs(), g.ft())
        g.close()
        if ref is None:
            ref = out
        else:
            assert (out[0] == ref[0]).all(), env
            assert (out[1][0] == ref[1][0]).all() and (out[1][1] == ref[1][1]).all(), env
