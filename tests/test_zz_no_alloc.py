"""The allocation-free entry point lbmep_get_invariants_noalloc against
lbmep_get_invariants on the same lattice: bitwise the same FP64 sums (same
kernels, same reduction order), on two calls in a row, the second on a
smaller grid (fewer partial blocks than the first left in the static
scratch array)."""
import numpy as np
import pytest

from paper_1708_08741_amd import workloads as W

pytestmark = pytest.mark.gpu


def _lattice(lb, shape, precision, seed):
    rng = np.random.default_rng(seed)
    X, R = W.rsa_spheres(rng, 4, 3.0, shape, (True, True, True), gap=2.0)
    U = rng.uniform(-0.02, 0.02, size=(len(R), 3))
    rho_e = W.gaussian_shell_rho_e(shape, (True, True, True), X, R)
    g = lb.Lattice(shape, precision=precision, move_particles=True)
    g.set_charge_force(rho_e.astype(np.float64 if precision == lb.FP64 else np.float32),
                       (1e-2, 0.0, 0.0))
    g.init_equilibrium()
    g.set_particles(X, R, U)
    g.step(7)
    return g


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_invariants_noalloc_equals_invariants(precision):
    import torch

    from paper_1708_08741_amd import lbmep as lb
    # 256 x 200 x 168 cells fill all 4096 partial blocks; 24 x 20 x 18 use 5
    for shape, seed in (((256, 200, 168), 1), ((24, 20, 18), 2)):
        g = _lattice(lb, shape, precision, seed)
        out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        g.invariants_noalloc(out)
        g.sync()
        got = out.cpu().numpy()
        ref = g.invariants()
        assert np.isfinite(ref).all()
        assert (got == ref).all(), (shape, got, ref)
        g.close()
