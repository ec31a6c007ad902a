"""Stokes wall effect of a sphere driven through a free-slip duct.

The validation setup of Sec. "Validation of Electrophoretic Motion of a
Sphere" (Tab. ElectrophoresisValidSpheres_DomainSizes, R_L = 4): a sphere of
radius 4 on the axis of a 864 x 1248 x 864 box whose six faces are free-slip
(Sec. "Simulation Setups": the sphere starts at y_0 = 98 R_L and is pushed
along y), tau = 6 (Eq. kinVisc: nu = (tau - 1/2) / 3), the TRT rates of
Sec. 3.1 with Lambda = 3/16.  The sphere moves under a constant force F along
y by the Newton-Euler update of the particle dynamics (particle density
1195 / 1000 of the fluid's, Tab. Electrolyte_Sphere_Parameters); F is chosen
for the paper's particle Reynolds number Re = U d / nu = 0.018 at the Stokes
velocity U_St = F / (6 pi rho_0 nu R) (Eq. StokesVelSphere, rho_0 = 1).

As in the paper, the velocity is sampled every 20 steps and the terminal
velocity U* is the mean over the last half of the samples; reported are
Delta_r U_Stokes = (U* - U_St) / U_St, the fluctuation (max - min) / U* over
that half, and the drift of U over it (a straight-line fit).

    python -m paper_1708_08741_amd.wall_effect --steps 40000 --max-seconds 1000 \
        --precision fp32dev --out result.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

SHAPE = (864, 1248, 864)
RADIUS = 4.0
TAU = 6.0
Y0 = 98.0 * RADIUS
RE_P = 0.018
RHO_P = 1.195
SAMPLE_EVERY = 20


def stokes_force(nu, radius, u):
    """Stokes drag 6 pi rho_0 nu R U (rho_0 = 1) at velocity u."""
    return 6.0 * math.pi * nu * radius * u


def terminal_stats(t, u, u_st):
    """U* (mean of the last half of the samples), Delta_r U_Stokes,
    fluctuation and drift (relative change of a straight-line fit over the
    last half, per 10,000 steps)."""
    t = np.asarray(t, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    h = len(u) // 2
    tt, uu = t[h:], u[h:]
    ustar = float(uu.mean())
    slope = float(np.polyfit(tt, uu, 1)[0]) if len(uu) > 2 else float("nan")
    return {
        "U_star": ustar,
        "delta_r_U_stokes_pct": 100.0 * (ustar - u_st) / u_st,
        "fluctuation_pct": 100.0 * float(uu.max() - uu.min()) / ustar,
        "drift_pct_per_10k_steps": 100.0 * slope * 1e4 / ustar,
        "samples_averaged": int(len(uu)),
        "from_step": int(tt[0]) if len(tt) else None,
    }


def run(steps, precision, max_seconds, shape=SHAPE, radius=RADIUS, progress=True):
    import torch
    from paper_1708_08741_amd import lbmep as lb

    torch.cuda.set_device(0)
    prec = {"fp64": lb.FP64, "fp32dev": lb.FP32DEV, "fp16dev": lb.FP16DEV}[precision]
    nu = (TAU - 0.5) / 3.0
    u_st = RE_P * nu / (2.0 * radius)
    force = stokes_force(nu, radius, u_st)
    t0 = time.perf_counter()
    g = lb.Lattice(shape, (False, False, False), nu=nu, magic=3.0 / 16.0, precision=prec,
                   move_particles=True)
    g.set_free_slip((1, 1, 1, 1, 1, 1))
    g.init_equilibrium()
    X = np.array([[shape[0] / 2.0, Y0 if shape == SHAPE else shape[1] / 3.0, shape[2] / 2.0]])
    g.set_particles(X, [radius], np.zeros((1, 3)))
    # the constant force acts as q E with q = 1, E = (0, F, 0)
    g.set_dynamics(RHO_P, q=[1.0], E=(0.0, force, 0.0))
    g.sync()
    setup_s = time.perf_counter() - t0
    if progress:
        print(f"[wall_effect] {shape} {precision}: nu {nu:.6f}, F {force:.6f}, U_Stokes {u_st:.6e}, "
              f"set-up {setup_s:.1f} s", flush=True)
    ts, us, ys = [], [], []
    t1 = time.perf_counter()
    done = 0
    last_print = t1
    while done < steps:
        g.step(SAMPLE_EVERY)
        done += SAMPLE_EVERY
        Xp, Up, _ = g.particles()
        ts.append(done)
        us.append(float(Up[0, 1]))
        ys.append(float(Xp[0, 1]))
        now = time.perf_counter()
        if progress and now - last_print > 30.0:
            print(f"[wall_effect] step {done}: U_y {us[-1]:.6e} ({100 * (us[-1] - u_st) / u_st:+.3f} % "
                  f"of Stokes), y {ys[-1]:.2f}, {1e3 * (now - t1) / done:.2f} ms/step", flush=True)
            last_print = now
        if now - t1 > max_seconds:
            break
    elapsed = time.perf_counter() - t1
    F, M = g.ft()
    g.close()
    res = {
        "setup": {
            "shape": list(shape), "faces": "free-slip on all six", "radius": radius, "tau": TAU,
            "nu": nu, "Lambda": 3.0 / 16.0, "x0": X[0].tolist(), "rho_p": RHO_P,
            "force_y": force, "Re_p_at_stokes": RE_P, "U_stokes": u_st, "precision": precision,
            "sample_every": SAMPLE_EVERY,
        },
        "steps": done,
        "ms_per_step": 1e3 * elapsed / max(done, 1),
        "hydrodynamic_force_last_step": F[0].tolist(),
        "final_position": [float(v) for v in Xp[0]],
        "paper_delta_r_U_stokes_pct": -3.04,
    }
    res.update(terminal_stats(ts, us, u_st))
    # a coarse history (every 500 steps) for the record
    res["history"] = [[t, u] for t, u in zip(ts, us) if t % 500 == 0]
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=40000)
    ap.add_argument("--max-seconds", type=float, default=1000.0,
                    help="stop stepping after this much wall time (the result states the steps done)")
    ap.add_argument("--precision", default="fp32dev", choices=["fp64", "fp32dev", "fp16dev"])
    ap.add_argument("--shape", default=None, help="nx,ny,nz (default: the paper's 864,1248,864)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else SHAPE
    res = run(args.steps, args.precision, args.max_seconds, shape=shape)
    line = json.dumps(res)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
