"""The request server (lbmep_server_*): continuous batching with packed
launches.

* A mix of requests of uneven grid sizes, particle counts, precisions and
  step counts, served with fewer slots than requests (so that requests are
  admitted while others run) and a chunk length that does not divide the step
  counts, gives every request the result it has alone on a plain lattice:
  fields, FP64 invariants, forces and torques bitwise (the per-particle sums
  are formed in one workgroup in a fixed order).
* An FP64 request served in the mix matches the FP64 CPU oracle (1e-12).
* Admission respects the HBM budget: with a budget for two requests at a
  time, never more than two are resident.
"""
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


def _requests(lb):
    """Uneven small simulations (ragged x extents, walls on some)."""
    specs = [
        ((40, 36, 32), 3, 3.5, 37, lb.FP32DEV, True),
        ((130, 20, 24), 2, 4.0, 23, lb.FP32DEV, False),
        ((48, 32, 40), 4, 3.0, 51, lb.FP64, True),
        ((32, 32, 32), 1, 5.0, 16, lb.FP16DEV, True),
        ((56, 40, 24), 5, 3.2, 44, lb.FP32DEV, True),
        ((24, 64, 28), 0, 3.0, 12, lb.FP32DEV, True),
        ((72, 30, 30), 3, 3.6, 29, lb.FP64, True),
        ((36, 44, 36), 2, 4.4, 33, lb.FP32DEV, True),
    ]
    out = []
    for i, (shape, n, R, steps, prec, moving) in enumerate(specs):
        rng = np.random.default_rng(100 + i)
        per = (True, True, True)
        flags = None
        if i % 3 == 1:
            per = (True, False, True)
            flags = W.channel_flags(shape)
        lo = hi = None
        if flags is not None:
            lo = [0.0, 1.0 + R + 1.0, 0.0]
            hi = [shape[0], shape[1] - 2.0 - R - 1.0, shape[2]]
        X, Rs = W.rsa_spheres(rng, n, R, shape, per, gap=2.0, lo=lo, hi=hi)
        U = rng.uniform(-0.01, 0.01, size=(len(Rs), 3))
        Wv = rng.uniform(-1e-3, 1e-3, size=(len(Rs), 3))
        rho_e = W.gaussian_shell_rho_e(shape, per, X, Rs) if len(Rs) else np.full(
            shape[::-1], 1e-5)
        dt = np.float64 if prec == lb.FP64 else np.float32
        out.append(dict(shape=shape, X=X, R=Rs, U=U, W=Wv, steps=steps, flags=flags,
                        periodic=per, rho_e=rho_e.astype(dt), E=(2e-2, -1e-2, 0.0),
                        precision=prec, moving=moving))
    return out


def _alone(lb, q):
    g = lb.Lattice(q["shape"], q["periodic"], precision=q["precision"],
                   move_particles=q["moving"])
    if q["flags"] is not None:
        g.set_flags(q["flags"])
    g.set_charge_force(q["rho_e"], q["E"])
    g.init_equilibrium()
    g.set_particles(q["X"], q["R"], q["U"], q["W"])
    g.step(q["steps"])
    rho, u = g.macro()
    inv = g.invariants()
    F, M = g.ft()
    g.close()
    return rho, u, inv, F, M


def test_mix_equals_alone(lb):
    reqs = _requests(lb)
    srv = lb.Server(hbm_budget=2 << 30, max_slots=3, chunk_steps=7)
    ids = [srv.submit(q["shape"], X=q["X"], R=q["R"], U=q["U"], W=q["W"], steps=q["steps"],
                      rho_e=q["rho_e"], E=q["E"], flags=q["flags"], periodic=q["periodic"],
                      precision=q["precision"], moving=q["moving"], keep_fields=True)
           for q in reqs]
    order = srv.wait_all(ids, timeout=300)
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["resident"] == 0 and st["bytes_in_use"] == 0
    assert len(order) == len(ids)
    for q, rid in zip(reqs, ids):
        F, M, inv, t = srv.result(rid)
        rho, u = srv.fields(rid)
        rho_a, u_a, inv_a, F_a, M_a = _alone(lb, q)
        assert (rho == rho_a).all() and (u == u_a).all(), q["shape"]
        assert (inv == inv_a).all(), (inv, inv_a)
        assert (F == F_a).all() and (M == M_a).all()
        assert t[0] <= t[1] <= t[2]
        srv.release(rid)
    srv.close()


def test_served_fp64_request_matches_oracle(lb, oracle_mod):
    shape = (40, 34, 30)
    rng = np.random.default_rng(7)
    X, R = W.rsa_spheres(rng, 3, 3.4, shape, (True, True, True), gap=2.0)
    U = rng.uniform(-0.03, 0.03, size=(3, 3))
    Wv = rng.uniform(-3e-3, 3e-3, size=(3, 3))
    rho_e = W.gaussian_shell_rho_e(shape, (True, True, True), X, R)
    E = (1e-2, 0.0, 5e-3)
    steps = 41
    srv = lb.Server(hbm_budget=1 << 30, max_slots=4, chunk_steps=5)
    # two FP32 neighbours in the mix
    other = [srv.submit((33, 29, 31), X=[[10.0, 10.0, 10.0]], R=[3.0], U=[[0.01, 0, 0]],
                        steps=s, rho_e=np.full(33 * 29 * 31, 1e-5, np.float32),
                        E=(1e-2, 0, 0)) for s in (13, 60)]
    rid = srv.submit(shape, X=X, R=R, U=U, W=Wv, steps=steps, rho_e=rho_e, E=E,
                     precision=lb.FP64, keep_fields=True)
    srv.wait_all(other + [rid], timeout=300)
    F, M, inv, _ = srv.result(rid)
    rho, u = srv.fields(rid)
    o = oracle_mod.Oracle(shape)
    o.set_force(np.stack([rho_e * E[0], rho_e * E[1], rho_e * E[2]]))
    o.init_equilibrium()
    o.set_particles(X, R, U, Wv, moving=True)
    o.step(steps)
    rho_o, u_o = o.macro()
    F_o, M_o = o.ft()
    assert np.abs(rho - rho_o).max() <= 1e-12
    assert np.abs(u - u_o).max() <= 1e-12 * np.abs(u_o).max()
    sF = np.abs(F_o).max()
    assert np.abs(F - F_o).max() <= 1e-12 * sF
    assert np.abs(M - M_o).max() <= 1e-12 * sF * R.max()
    srv.close()


def test_admission_respects_the_budget(lb):
    shape = (48, 40, 36)
    kw = dict(X=[[20.0, 20.0, 18.0]], R=[4.0], U=[[0.01, 0.0, 0.0]], steps=40,
              rho_e=np.full(48 * 40 * 36, 1e-5, np.float32), E=(1e-2, 0, 0))
    fp = lb.Server.request_footprint(shape, **kw)
    srv = lb.Server(hbm_budget=2 * fp + fp // 2, max_slots=8, chunk_steps=4)
    ids = [srv.submit(shape, **kw) for _ in range(6)]
    done = []
    max_res = 0
    import time
    t0 = time.monotonic()
    while len(done) < len(ids):
        done += srv.poll()
        st = srv.stats()
        max_res = max(max_res, st["resident"])
        assert st["bytes_reserved"] <= st["budget"]
        assert time.monotonic() - t0 < 300
        time.sleep(2e-4)
    assert max_res == 2
    invs = [srv.result(i)[2] for i in ids]
    for v in invs[1:]:
        assert (v == invs[0]).all()  # identical requests, identical results
    # a request that can never fit is refused at submit
    with pytest.raises(lb.LbmepError) as e:
        srv.submit((96, 96, 96), steps=1)
    assert e.value.code == lb.EINVAL
    srv.close()


def test_queue_limit_and_bad_requests(lb):
    srv = lb.Server(hbm_budget=256 << 20, max_slots=1, chunk_steps=3, max_queue=2)
    kw = dict(steps=5)
    a = srv.submit((16, 16, 16), **kw)
    b = srv.submit((16, 16, 16), **kw)
    with pytest.raises(lb.LbmepError) as e:
        srv.submit((16, 16, 16), **kw)
    assert e.value.code == lb.EBUSY
    with pytest.raises(lb.LbmepError) as e:
        srv.submit((16, 16, 16), steps=0)
    assert e.value.code == lb.EINVAL
    with pytest.raises(lb.LbmepError) as e:
        srv.submit((16, 16, 16), steps=3, X=[[1, 1, 1]], R=[-1.0], U=[[0, 0, 0]])
    assert e.value.code == lb.EBUSY  # queue still full
    srv.wait_all([a, b], timeout=120)
    # set-up errors surface as a failed request, not as a server error
    c = srv.submit((16, 16, 16), steps=3, X=[[1, 1, 1]], R=[-1.0], U=[[0, 0, 0]])
    srv.wait_all([c], timeout=120)
    with pytest.raises(lb.LbmepError) as e:
        srv.result(c)
    assert e.value.code == lb.EINVAL
    st = srv.stats()
    assert st["completed"] == 2 and st["failed"] == 1
    # packed launches: a fixed-size mix of one lattice still uses the packed path
    assert st["packed_launches"] > 0
    srv.close()
