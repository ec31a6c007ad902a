"""Benchmark of the moving-particle D3Q19 TRT sweep on one MI355X.

A step is one full time step of the method on the GPU: the fused
collide/stream sweep with the charge body force, wall and velocity
bounce-back and the per-particle momentum exchange, followed by the
prescribed kinematics, re-mapping and refill for the next time level.

Workload: 512^3 fully periodic box, 4096 moving spheres of radius 4
(random sequential addition, surface gap >= 3, velocities uniform in
[-5e-4, 5e-4]), body force rho_e * E with a Gaussian-shell charge density
(Debye length 2, amplitude 1e-5) and E = (1e-3, 0, 0), nu = 1/6,
Lambda = 3/16, populations stored as FP32 deviations from the rest weights.

Prints ONE JSON line.  `value` is MLUPS (all cells); `roofline` prices the
fused sweep kernel against the 8 TB/s HBM peak with 152 algorithmic bytes
per cell update (19 FP32 loads + 19 FP32 stores); `cpu_baseline` times the
FP64 CPU oracle on a bounded sample of the same workload shape.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline, 512^3 FP32/FP16 vs FP64; serve p50/p99 latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = {"fp64": 304, "fp32dev": 152, "fp16dev": 76}
DTYPE = {"fp64": "f64", "fp32dev": "f32", "fp16dev": "f32"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_stream_collide_512.json")
# the gather / collide sweep instantiation timed per precision (storage type,
# charge force, 32-bit offsets, streaming-hint mode, one cell per thread)
SWEEP_KERNEL = {"fp32dev": "k_sweep<float, 2, unsigned int, 4, 1>",
                "fp64": "k_sweep<double, 2, unsigned int, 4, 1>",
                "fp16dev": "k_sweep<__half, 2, unsigned int, 4, 1>"}
KERNEL_SRC = os.path.join(ROOT, "paper_1708_08741_amd", "csrc", "sweep_impl.h")
# the sweep's launch shape (segment width, block order, population stride) is
# set in the API source: counters taken on other settings do not apply
LAUNCH_SRC = os.path.join(ROOT, "paper_1708_08741_amd", "csrc", "lbmep_api.hip")
SERVE_FULL = os.path.join(ROOT, "profiles", "serving_2000_requests_fp32.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in (KERNEL_SRC, LAUNCH_SRC):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


SOR_SRC = os.path.join(ROOT, "paper_1708_08741_amd", "csrc", "k_potential.hip")


def sor_traffic():
    """HBM bytes of one FP32 one-pass SOR iteration (k_sor_march) from the
    committed counter summary, if it was taken on the current SOR source;
    else None."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    sha = hashlib.sha256(open(SOR_SRC, "rb").read()).hexdigest()[:16]
    if d.get("sor_kernel_sha") != sha:
        return None
    for k, e in d.get("other_kernels", {}).items():
        if k.startswith("k_sor_march<float"):
            return e.get("hbm_bytes_per_launch")
    return None


def traffic_for(precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current sweep source; else None."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_hash():
        return None
    e = d.get("per_precision", {}).get(precision)
    if not e:
        return None
    return e.get("hbm_bytes_per_launch")


def run_gpu(wl, precision, steps, warmup, potential=None):
    import torch

    from paper_1708_08741_amd import lbmep as lb

    stream = torch.cuda.current_stream()
    L = lb.from_workload(wl, precision=precision, stream=stream.cuda_stream)
    if potential is not None:
        # the body force computed in the sweep from the EDL potential
        psi, keps, zeta = potential
        L.set_potential_force(psi.astype(np.float64 if precision == "fp64" else np.float32),
                              keps, wl.E, zeta)
    fl, _ = L.map()
    nfluid = int(((fl == lb.FLUID) | (fl == lb.NEAR)).sum())
    del fl
    L.step(warmup)
    L.sync()
    L.get_timing()  # reset
    L.set_timing(True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    kern_ms, launches = L.get_timing()
    L.set_timing(False)
    inv = L.invariants()
    L.close()
    torch.cuda.empty_cache()
    return dict(total_ms=total_ms, kernel_ms=kern_ms / max(launches, 1), launches=launches,
                nfluid=nfluid, invariants=inv.tolist())


def run_coupled(wl, precision, steps, warmup, sor_iters, kappa=0.5):
    """The electrophoresis step (Alg. "Electrophoresis Algorithm"): a fixed
    number of red-black SOR iterations of the Debye-Hueckel equation on the
    current map, the stream-collide step with the force from the potential,
    the momentum exchange, and the Newton-Euler update of the charged
    particles.  The spheres' Debye-Hueckel fields (surface potentials in
    [-0.05, 0.05]) are the initial potential.  Also times one standalone
    solve of sor_iters iterations (HIP events on the lattice's stream)."""
    import torch

    from paper_1708_08741_amd import lbmep as lb
    from paper_1708_08741_amd import workloads as W

    zeta = np.random.default_rng(4).uniform(-0.05, 0.05, len(wl.R))
    psi = W.debye_huckel_psi(wl.shape, wl.periodic, wl.X, wl.R, zeta, kappa=kappa, cutoff=6.0)
    stream = torch.cuda.current_stream()
    L = lb.from_workload(wl, precision=precision, stream=stream.cuda_stream)
    L.set_potential_force(psi.astype(np.float64 if precision == "fp64" else np.float32),
                          1e-3, wl.E, zeta)
    del psi
    L.set_potential_solver(kappa * kappa, 1.7, sor_iters, 0.0)
    # the particles move under their forces: density ratio of the paper's
    # particles (1195 / 1000), charges q ~ U[-0.1, 0.1] in the applied field
    qp = np.random.default_rng(5).uniform(-0.1, 0.1, len(wl.R))
    L.set_dynamics(1.195, qp, wl.E)
    L.step(warmup)
    L.sync()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    L.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / steps
    # one standalone solve: 2 sor_iters half-sweep launches back to back
    solves = 3
    e0.record(stream)
    for _ in range(solves):
        L.solve_potential()
    e1.record(stream)
    torch.cuda.synchronize()
    solve_ms = e0.elapsed_time(e1) / solves
    shape = L.solver_shape()
    L.close()
    torch.cuda.empty_cache()
    return dict(step_ms=step_ms, solve_ms=solve_ms, shape=shape)


def _time_oracle(wl, steps, repeats, threads):
    """Median wall time per step of the oracle on workload wl (after a
    5-step warm-up), with the given OpenMP thread count."""
    from oracle import oracle as O
    O.set_num_threads(threads)
    o = O.from_workload(wl)
    o.step(5)
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        o.step(steps)
        ts.append((time.perf_counter() - t0) / steps)
    fl, _ = o.map()
    nfluid = int(((fl == O.FLUID) | (fl == O.NEAR)).sum())
    o.close()
    return float(np.median(ts)), nfluid


def cpu_baseline():
    """The FP64 oracle on bounded samples of the two 128^3 configurations:
    the sub-run of the 512^3 suspension (64 moving R=4 spheres, charge force)
    and the channel (walls y=0,127, 64 moving R=6 spheres), each on every
    host core and on one core; median of 3 timed repeats after a 5-step
    warm-up.  `value` is the all-core rate on the sub-run (the headline
    workload's shape)."""
    from oracle import oracle as O
    from paper_1708_08741_amd import workloads as W

    cores = O.num_threads()
    out = {}
    for name, wl in (("subrun128", W.suspension_subrun(precision="fp64")),
                     ("channel128", W.channel_spheres())):
        for label, threads, steps in (("all_cores", cores, 10), ("one_core", 1, 2)):
            per, nfluid = _time_oracle(wl, steps, 3, threads)
            out[f"{name}_{label}"] = {"MLUPS": round(wl.ncells / per / 1e6, 3),
                                      "MFLUPS": round(nfluid / per / 1e6, 3),
                                      "threads": threads, "steps_timed": steps}
            log(f"[bench] oracle {name} {label}: {out[f'{name}_{label}']}")
    O.set_num_threads(cores)
    rec = {"value": out["subrun128_all_cores"]["MLUPS"], "unit": "MLUPS", "cores": cores,
           "kind": "oracle",
           "sample": "128^3 periodic sub-run (64 moving R=4 spheres, charge force), FP64, median "
                     "of 3 x 10 steps after 5 warm-up steps, all host cores; also 1 core and the "
                     "128^3 channel (64 moving R=6 spheres), see 'samples'",
           "samples": out,
           "paper_context_MFLUPS_per_16_core_node": 61.2}
    return rec


def precision_errors(steps=500):
    """Errors of the GPU FP64 / FP32-dev / FP16-dev runs of the 128^3
    sub-run against the FP64 oracle after the configuration's 500 steps
    (relative to max |u| over fluid cells and max |F_p|; |drho| absolute;
    torque relative to max |F| R; FP64 mass and momentum sums: mass relative,
    momentum relative to N_fluid max |u|)."""
    from oracle import oracle as O
    from paper_1708_08741_amd import lbmep as lb
    from paper_1708_08741_amd import workloads as W

    wl = W.suspension_subrun(precision="fp64", steps=steps)
    o = O.from_workload(wl)
    t0 = time.perf_counter()
    o.step(steps)
    log(f"[bench] oracle sub-run, {steps} steps: {time.perf_counter() - t0:.1f} s")
    rho_o, u_o = o.macro()
    F_o, M_o = o.ft()
    fl, _ = o.map()
    inv_o = o.invariants()
    o.close()
    fluid = (fl == O.FLUID) | (fl == O.NEAR)
    umax = np.abs(u_o[:, fluid]).max()
    sF = np.linalg.norm(F_o, axis=1).max()
    scale_P = fluid.sum() * umax
    out = {"steps": steps, "workload": "128^3 sub-run (64 moving R=4 spheres)"}
    for p in ("fp64", "fp32dev", "fp16dev"):
        g = lb.from_workload(wl, precision=p)
        g.step(steps)
        rho_g, u_g = g.macro()
        F_g, M_g = g.ft()
        inv_g = g.invariants()
        out[p] = {
            "u_rel": float(np.abs(u_g - u_o)[:, fluid].max() / umax),
            "rho_abs": float(np.abs(rho_g - rho_o)[fluid].max()),
            "F_rel": float(np.linalg.norm(F_g - F_o, axis=1).max() / sF),
            "M_rel": float(np.linalg.norm(M_g - M_o, axis=1).max() / (sF * 4.0)),
            "mass_drift_rel": float(abs(inv_g[0] - inv_o[0]) / inv_o[0]),
            "momentum_drift_rel": float(np.abs(inv_g[1:] - inv_o[1:]).max() / scale_P),
        }
        g.close()
    return out


def fullsize_vs_fp64(wl, steps=500):
    """FP32-dev and FP16-dev against GPU-FP64 on the full 512^3 suspension
    after `steps` steps: u (relative to max |u| of the FP64 run over fluid
    cells), rho (absolute), F (relative to max |F_p|), M (relative to max
    |F| R) and the FP64 mass / momentum sums; compared on the device."""
    import torch

    from paper_1708_08741_amd import lbmep as lb

    dev = torch.device("cuda")
    n = wl.ncells
    res = {}
    ref = None
    for p in ("fp64", "fp32dev", "fp16dev"):
        L = lb.from_workload(wl, precision=p)
        L.step(steps)
        rho = torch.empty(n, dtype=torch.float64, device=dev)
        u = torch.empty(3 * n, dtype=torch.float64, device=dev)
        L.macro_device(rho, u)
        F, M = L.ft()
        inv = L.invariants()
        if ref is None:
            fl, _ = L.map()
            fluid = torch.from_numpy(((fl == lb.FLUID) | (fl == lb.NEAR)).reshape(-1)).to(dev)
            del fl
            umax = u.view(3, n)[:, fluid].abs().max().item()
            ref = dict(rho=rho, u=u, F=F, M=M, inv=inv, fluid=fluid, umax=umax,
                       nfluid=int(fluid.sum().item()))
        else:
            fluid = ref["fluid"]
            sF = np.linalg.norm(ref["F"], axis=1).max()
            res[p] = {
                "u_rel": (u - ref["u"]).view(3, n)[:, fluid].abs().max().item() / ref["umax"],
                "rho_abs": (rho - ref["rho"])[fluid].abs().max().item(),
                "F_rel": float(np.linalg.norm(F - ref["F"], axis=1).max() / sF),
                "M_rel": float(np.linalg.norm(M - ref["M"], axis=1).max() / (sF * 4.0)),
                "mass_drift_rel": float(abs(inv[0] - ref["inv"][0]) / ref["inv"][0]),
                "momentum_drift_rel": float(np.abs(inv[1:] - ref["inv"][1:]).max() /
                                            (ref["nfluid"] * ref["umax"])),
            }
            del rho, u
        L.close()
        torch.cuda.empty_cache()
        log(f"[bench] {p} {steps} steps at full size done")
    res["steps"] = steps
    res["workload"] = "512^3 suspension (4096 moving R=4 spheres), against the GPU FP64 run"
    del ref
    torch.cuda.empty_cache()
    return res


def copy_reference_gbps(gib=4.0, iters=10):
    """Achievable HBM bandwidth: the library's reference copy (16-byte lanes,
    streaming stores) of `gib` GiB, bytes read + written per second."""
    import torch

    from paper_1708_08741_amd import lbmep as lb

    nbytes = int(gib * 2 ** 30) // 16 * 16
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        lb.copy_reference(dst, src, stream.cuda_stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(iters):
        lb.copy_reference(dst, src, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    assert torch.equal(dst[:1024], src[:1024])
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms / 1e3) / 1e9


def _serving_inputs(r):
    """Request r of the serving mix with its charge density (FP32)."""
    from paper_1708_08741_amd import workloads as W
    q = W.serving_request(r)
    q["rho_e"] = W.gaussian_shell_rho_e(q["shape"], q["periodic"], q["X"], q["R"]).astype(
        np.float32)
    return q


class _RequestStream:
    """Requests of the serving mix generated by a pool of host processes, at
    most `ahead` of them in flight or buffered (bounded host memory)."""

    def __init__(self, first, count, ahead=32):
        import multiprocessing as mp
        self.pool = mp.get_context("fork").Pool(min(16, os.cpu_count() or 1))
        self.next_submit = first
        self.end = first + count
        self.pending = {}
        self.ahead = ahead
        self.next_take = first
        self._fill()

    def _fill(self):
        while self.next_submit < self.end and len(self.pending) < self.ahead:
            r = self.next_submit
            self.pending[r] = self.pool.apply_async(_serving_inputs, (r,))
            self.next_submit += 1

    def take(self):
        r = self.next_take
        q = self.pending.pop(r).get()
        self.next_take += 1
        self._fill()
        return q

    def close(self):
        self.pool.terminate()
        self.pool.join()


def serving_bench(n_load, n_sat, load, budget_gib, slots, chunk):
    """Continuous batching of the serving mix (FP32-dev, moving spheres,
    charge force).  Saturated throughput: n_sat requests queued at once (more
    than the slots), cell updates completed per second while the queue is not
    empty.  Then n_load requests arriving as a Poisson process (seed 5) at
    `load` times that throughput; latency = completion - arrival (server
    clock)."""
    from paper_1708_08741_amd import lbmep as lb

    def work(q):
        nx, ny, nz = q["shape"]
        return nx * ny * nz * q["steps"]

    def submit(srv, q):
        return srv.submit(q["shape"], X=q["X"], R=q["R"], U=q["U"], W=q["W"], steps=q["steps"],
                          rho_e=q["rho_e"], E=q["E"], periodic=q["periodic"],
                          precision=lb.FP32DEV, moving=True)

    srv = lb.Server(hbm_budget=int(budget_gib * 2 ** 30), max_slots=slots, chunk_steps=chunk)
    t0 = time.perf_counter()
    stream = _RequestStream(0, n_sat, ahead=n_sat)
    sat = [stream.take() for _ in range(n_sat)]
    stream.close()
    log(f"[serve] {n_sat} saturation requests generated in {time.perf_counter() - t0:.1f} s")
    dropped = sum(q["requested"] - len(q["R"]) for q in sat)
    ids = [submit(srv, q) for q in sat]
    del sat
    # rate over the window in which requests wait (every slot or the budget busy)
    w0 = w1 = None
    done = set()
    while len(done) < len(ids):
        done.update(srv.poll())
        st = srv.stats()
        now = srv.now()
        if st["cell_updates_done"] > 0 and w0 is None:
            w0 = (now, st["cell_updates_done"])
        if w0 is not None and (st["queued"] > 0 or w1 is None):
            w1 = (now, st["cell_updates_done"])
        time.sleep(2e-4)
    for i in ids:
        srv.release(i)
    sat_rate = (w1[1] - w0[1]) / max(w1[0] - w0[0], 1e-9)
    log(f"[serve] saturated: {sat_rate / 1e6:.0f} MLUPS over {w1[0] - w0[0]:.2f} s "
        f"with a full queue")

    # Poisson arrivals at `load` of the saturated rate; inputs generated ahead
    stream = _RequestStream(n_sat, n_load)
    mean_work = 147.2 ** 3 * 2750.0   # expected cell updates per request of the mix
    lam = load * sat_rate / mean_work
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n_load))
    start = srv.now()
    ids, works = [], []
    done = set()
    max_res = 0
    nxt = stream.take()
    last_log = time.perf_counter()
    while len(done) < n_load:
        now = srv.now() - start
        while nxt is not None and arrivals[len(ids)] <= now:
            ids.append(submit(srv, nxt))
            works.append(work(nxt))
            dropped += nxt["requested"] - len(nxt["R"])
            nxt = stream.take() if len(ids) < n_load else None
        done.update(srv.poll())
        max_res = max(max_res, srv.stats()["resident"])
        if time.perf_counter() - last_log > 30:
            log(f"[serve] t={now:.0f} s: {len(ids)} arrived, {len(done)} done")
            last_log = time.perf_counter()
        if now > 36000:
            raise TimeoutError("serving run did not finish")
        time.sleep(2e-4)
    stream.close()
    lat, t_end = [], 0.0
    for i in ids:
        _, _, _, t = srv.result(i)
        lat.append(t[2] - t[0])
        t_end = max(t_end, t[2])
    span = t_end - start
    st = srv.stats()
    srv.close()
    lat = np.array(lat)
    return {
        "requests": n_load, "saturation_requests": n_sat,
        "throughput_req_per_s": round(float(n_load / span), 3),
        "aggregate_MLUPS": round(float(sum(works) / span / 1e6), 1),
        "saturated_MLUPS": round(float(sat_rate / 1e6), 1),
        "offered_load": load, "arrival_rate_per_s": round(float(lam), 4),
        "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
        "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
        "latency_max_s": round(float(lat.max()), 3),
        "max_resident": max_res, "slots": slots, "chunk_steps": chunk,
        "hbm_budget_GiB": budget_gib, "packed_launches": int(st["packed_launches"]),
        "spheres_dropped_by_rsa": int(dropped),
        "mix": "edges {64,96,128,192,256}^3, 1-200 spheres R 3-8, 500-5000 steps, FP32-dev",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=512, help="box edge (cells)")
    ap.add_argument("--precision", default="fp32dev", choices=list(BYTES_PER_CELL))
    ap.add_argument("--variants", default="fp64,fp16dev,fp32dev_pot",
                    help="other storage precisions timed on the same workload ('' = none; "
                         "a _pot suffix: force from the EDL potential)")
    ap.add_argument("--variant-steps", type=int, default=100)
    ap.add_argument("--sor-iters", type=int, default=29,
                    help="SOR iterations per step of the coupled electrophoresis leg (0 = none)")
    ap.add_argument("--coupled-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the Poisson-arrival serving run (0 = no serving leg)")
    ap.add_argument("--serve-sat-requests", type=int, default=48,
                    help="requests of the saturated-throughput serving run (more than the "
                         "slots: the rate is taken while requests wait)")
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-chunk", type=int, default=20)
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="also run a plain device copy of this many GiB (the reference "
                         "kernel that scales HBM byte counters)")
    ap.add_argument("--copy-gib", type=float, default=4.0,
                    help="size of the reference copy that measures the achievable bandwidth "
                         "(0 = skip)")
    ap.add_argument("--fullsize-steps", type=int, default=500,
                    help="steps of the full-size FP32-dev / FP16-dev against FP64 comparison "
                         "(0 = skip)")
    ap.add_argument("--error-steps", type=int, default=500,
                    help="steps of the sub-run compared with the FP64 oracle")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path has no multi-GPU decomposition in this "
              "build (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_1708_08741_amd import workloads as W

    n = args.n
    count = 4096 * (n // 512) ** 3 if n >= 512 else max(1, int(4096 * (n / 512) ** 3))
    log(f"[bench] generating the {n}^3 workload ({count} spheres)")
    t0 = time.perf_counter()
    wl = W.periodic_suspension(n=n, count=count, R=4.0, seed=3, steps=args.steps,
                               precision=args.precision)
    log(f"[bench] inputs ready in {time.perf_counter() - t0:.1f} s")

    if args.copy_calibration > 0:
        # the reference copy of args.copy_calibration GiB: that many bytes
        # read and written per launch (scales the HBM byte counters)
        from paper_1708_08741_amd import lbmep as lbc
        nbytes = int(args.copy_calibration * 2 ** 30) // 16 * 16
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            lbc.copy_reference(dst, src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nbytes} bytes read and written per launch")
        del src, dst
        torch.cuda.empty_cache()
    copy_gbps = None
    if args.copy_gib > 0:
        copy_gbps = copy_reference_gbps(args.copy_gib)
        log(f"[bench] reference copy ({args.copy_gib} GiB, 16-byte lanes): {copy_gbps:.0f} GB/s")

    res = run_gpu(wl, args.precision, args.steps, args.warmup)
    cells = wl.ncells
    t_s = res["total_ms"] / 1e3
    mlups = cells * args.steps / t_s / 1e6
    mflups = res["nfluid"] * args.steps / t_s / 1e6
    k_s = res["kernel_ms"] / 1e3
    bpc = BYTES_PER_CELL[args.precision]
    achieved = bpc * cells / k_s / 1e9
    log(f"[bench] {args.precision}: {mlups:.0f} MLUPS, sweep kernel {res['kernel_ms']:.3f} ms "
        f"= {achieved:.0f} GB/s")

    variants = {}
    for v in [s for s in args.variants.split(",") if s]:
        if v == args.precision:
            continue
        pot = None
        base = v
        if v.endswith("_pot"):
            # the same suspension with the force from the spheres' Debye-Hueckel
            # potential (surface potentials in [-0.05, 0.05], kappa = 0.5)
            base = v[:-4]
            zeta = np.random.default_rng(4).uniform(-0.05, 0.05, len(wl.R))
            psi = W.debye_huckel_psi(wl.shape, wl.periodic, wl.X, wl.R, zeta, kappa=0.5,
                                     cutoff=6.0)
            pot = (psi, 1e-3, zeta)
        r = run_gpu(wl, base, args.variant_steps, 5, pot)
        pot = psi = None
        tv = r["total_ms"] / 1e3
        kv = r["kernel_ms"] / 1e3
        v_bpc = BYTES_PER_CELL[base]
        variants[v] = {
            "MLUPS": round(cells * args.variant_steps / tv / 1e6, 1),
            "steps": args.variant_steps,
            "sweep_kernel_ms": round(r["kernel_ms"], 4),
            "sweep_GBps": round(v_bpc * cells / kv / 1e9, 1),
            "roofline_frac": round(v_bpc * cells / kv / 1e9 / HBM_PEAK_GBS, 4),
        }
        log(f"[bench] {v}: {variants[v]}")

    coupled = None
    if args.sor_iters > 0:
        # the electrophoresis step: SOR iterations + stream-collide with the
        # force from the potential (the paper's scaling runs use 29 per step)
        r = run_coupled(wl, args.precision, args.coupled_steps, 3, args.sor_iters)
        es = 4 if args.precision != "fp64" else 8
        sor_bytes = (2 * es + 1) * cells  # psi read and written once, one flag byte
        it_ms = r["solve_ms"] / args.sor_iters
        one, rows, planes, waves = r["shape"]
        if one:
            label = (f"k_sor_march: one pass per iteration on colour-split psi, from one buffer "
                     f"into the other; workgroups of {waves} wavefronts hold whole rows, "
                     f"{rows} rows per thread, marching through chunks of {planes} z planes")
        else:
            label = (f"k_sor_half_vec: one colour per launch, two per iteration, {rows} rows "
                     f"per thread, chunks of {planes} z planes")
        coupled = {
            "MLUPS": round(cells / (r["step_ms"] / 1e3) / 1e6, 1),
            "ms_per_step": round(r["step_ms"], 4),
            "sor_iterations_per_step": args.sor_iters,
            "sor_ms_per_iteration": round(it_ms, 4),
            "sor_GBps": round(sor_bytes / (it_ms / 1e3) / 1e9, 1),
            "sor_roofline_frac": round(sor_bytes / (it_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "sor_bytes_per_cell_iteration": 2 * es + 1,
            "sor_byte_model": "ideal: psi read once and written once plus one flag byte per cell; "
                              "the one-pass kernel reads psi once (plus halo rows), writes it "
                              "once, and reads 2 bits per cell plus the codes of non-interior "
                              "cells instead of the flag byte",
            "sor_kernel": label,
            "sor_traffic_per_iteration": sor_traffic() if es == 4 and one else None,
            "steps": args.coupled_steps,
        }
        log(f"[bench] coupled step: {coupled}")

    fullsize = None
    if args.fullsize_steps > 0:
        log(f"[bench] FP32-dev / FP16-dev against FP64 at full size, {args.fullsize_steps} steps")
        fullsize = fullsize_vs_fp64(wl, args.fullsize_steps)
        log(f"[bench] full-size errors: {fullsize}")

    cpu = None
    errors = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle samples")
        cpu = cpu_baseline()
        log(f"[bench] GPU precisions against the oracle sub-run ({args.error_steps} steps)")
        errors = precision_errors(args.error_steps)
        log(f"[bench] errors: {errors}")

    serving = None
    if args.serve_requests > 0:
        log("[bench] serving leg")
        serving = serving_bench(args.serve_requests, args.serve_sat_requests, args.serve_load,
                                args.serve_budget_gib, args.serve_slots, args.serve_chunk)
        serving["note"] = (f"a bounded sample of {args.serve_requests} Poisson arrivals; the full "
                           f"configuration (2000 requests) is run with --serve-requests 2000, its "
                           f"record in 'full_configuration_run'")
        try:
            serving["full_configuration_run"] = json.load(open(SERVE_FULL))
            serving["full_configuration_run"]["file"] = os.path.relpath(SERVE_FULL, ROOT)
        except (OSError, ValueError):
            serving["full_configuration_run"] = None
        log(f"[bench] serving: {serving}")

    traffic = traffic_for(args.precision)
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["total_ms"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"{n}^3 periodic box, {count} moving spheres R=4, Gaussian-shell "
                        f"charge force E=(1e-3,0,0), D3Q19 TRT nu=1/6 Lambda=3/16, "
                        f"{args.precision} storage",
            "cells": cells, "fluid_cells": res["nfluid"], "particles": count,
            "precision": args.precision, "MFLUPS": round(mflups, 1),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_note": "HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / "
                            "WRITE_SIZE summary (profiles/), used only when it was taken on the "
                            "current sweep and launch sources; not measured in this run",
            "kernel": SWEEP_KERNEL.get(args.precision, "k_sweep"),
            "kernel_ms": round(res["kernel_ms"], 4),
            "bytes_per_cell": bpc,
            "achievable_copy_GBps": round(copy_gbps, 1) if copy_gbps else None,
            "frac_of_copy": round(achieved / copy_gbps, 4) if copy_gbps else None,
        },
        "cpu_baseline": cpu,
        "variants": variants,
        "coupled_electrophoresis_step": coupled,
        "errors_vs_fp64_oracle": errors,
        "fullsize_vs_gpu_fp64": fullsize,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
