"""Accuracy of the GPU forms against the FP64 oracle on the seeded workloads,
one JSON line per workload (needs the HIP device; test infrastructure, like
the rest of this directory):

    python tests/accuracy_report.py [--quick] > accuracy.jsonl

Velocity error of one evaluation: ||u_gpu(X_n) - u_oracle(X_n)|| /
||u_oracle(X_n)|| over one system's 3N components, both at the GPU's own
FP64 state X_n with the spring (and steric) forces at t_n, i.e. the first
RK4 stage of step n. Reported as max and median over the checkpoints (for an
ensemble, the worst system at each checkpoint).

Centre drift: ||dR_gpu - dR_oracle|| / ||dR_oracle||, dR the displacement of
every dumbbell centre (X_2s + X_2s+1)/2 from the start, over all dumbbells of
a system (worst system for an ensemble), at every checkpoint; the value at the
last one is reported. The oracle integrates the same initial state with the
same integrator in FP64.

The 65536-sphere workload is too large for an oracle trajectory (about 5 s per
step on 16 cores), so it gets spot checks only: the velocity error of 64
random spheres (index generator seeded with 7 + step) at the GPU state,
every 50 steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import paper_1004_1932_amd as P  # noqa: E402
from oracle import adref  # noqa: E402
from workload import make_preset  # noqa: E402

sys.path.insert(0, os.path.join(ROOT, "tests"))
from parity_metrics import sphere_err  # noqa: E402


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def centres(X):
    return 0.5 * (X[0::2] + X[1::2])


def systems(w):
    if hasattr(w, "S_per_sys"):
        off = w.sphere_offsets
        return [int(s) for s in w.S_per_sys], [slice(int(off[b]), int(off[b + 1])) for b in range(w.nsys)]
    return [w.S], [slice(0, w.N)]


def velocity_errors(w, sim, X, t):
    """per-system (norm, per-sphere) velocity errors at state X (host array),
    time t"""
    S, sl = systems(w)
    F = np.concatenate([adref.forces(w.params, X[s], w.phi[s.start // 2:s.stop // 2], t) for s in sl])
    u = sim.mobility(X, F).cpu().numpy()
    out = []
    for s in sl:
        uo = adref.mobility(w.params, X[s], F[s])
        out.append((relerr(u[s], uo), sphere_err(u[s], uo)))
    return out


def trajectory_report(name, precision, nsteps, chunk, launch="tuned"):
    w = make_preset(name)
    p = w.params
    S, sl = systems(w)
    sim = P.Simulator(p, S, precision=precision, launch=launch if precision == "fp32c" else None, graph=True)
    sim.set_state(w.X, w.phi)
    Xo = w.X.copy()
    c0 = centres(w.X)
    verr, serr, drift, bitwise = [], [], [], True
    t_gpu = t_orc = 0.0
    for n0 in range(0, nsteps, chunk):
        k = min(chunk, nsteps - n0)
        t = time.perf_counter()
        _, _, code = sim.run(k, 0)
        assert code == 0, f"{name}: status {code}"
        Xg = sim.get_state()[0].cpu().numpy()
        t_gpu += time.perf_counter() - t
        t = time.perf_counter()
        Xo, _, _, _ = adref.run(p, Xo, w.phi, k, t0=0.0, step0=n0, S_per_sys=S)
        t_orc += time.perf_counter() - t
        n = n0 + k
        bitwise = bitwise and bool(np.array_equal(Xg, Xo))
        dg, do = centres(Xg) - c0, centres(Xo) - c0
        d = [relerr(dg[s.start // 2:s.stop // 2], do[s.start // 2:s.stop // 2]) for s in sl]
        drift.append(max(d))
        if precision == "fp32c":
            ve = velocity_errors(w, sim, Xg, n * p.dt)
            verr.append(max(e for e, _ in ve))
            serr.append(max(x for _, x in ve))
        log(f"  {name} {precision} step {n}: drift {drift[-1]:.3e}"
            + (f", velocity error {verr[-1]:.3e}" if verr else "") + f" (gpu {t_gpu:.1f} s, oracle {t_orc:.1f} s)")
    out = {"workload": name, "form": precision, "steps": nsteps, "checkpoints": len(drift),
           "centre_drift_end": drift[-1], "centre_drift_max": max(drift), "bitwise_equal_to_oracle": bitwise}
    if verr:
        out.update({"velocity_error_max": max(verr), "velocity_error_median": float(np.median(verr)),
                    "per_sphere_error_max": max(serr)})
    if precision == "fp32c":
        out["launch"] = sim.launch
    sim.close()
    return out


def spot_report(name, nsteps, every):
    w = make_preset(name)
    p = w.params
    sim = P.Simulator(p, [w.S], precision="fp32c", launch="tuned", graph=True)
    sim.set_state(w.X, w.phi)
    errs, serrs = [], []
    for n0 in range(0, nsteps, every):
        _, _, code = sim.run(every, 0)
        assert code == 0, f"{name}: status {code}"
        n = n0 + every
        X, _, _ = sim.get_state()
        F = sim.forces(X, n * p.dt)  # bitwise equal to the oracle's forces (tested)
        u = sim.mobility(X, F).cpu().numpy()
        Xh, Fh = X.cpu().numpy(), F.cpu().numpy()
        rows = np.random.default_rng(7 + n).choice(w.N, 64, replace=False)
        uo = adref.mobility_rows(p, Xh, Fh, rows)
        errs.append(relerr(u[rows], uo))
        serrs.append(sphere_err(u[rows], uo))
        log(f"  {name} step {n}: sampled velocity error {errs[-1]:.3e}, per-sphere {serrs[-1]:.3e}")
    out = {"workload": name, "form": "fp32c", "steps": nsteps, "checkpoints": len(errs),
           "sampled_velocity_error_max": max(errs), "sampled_velocity_error_median": float(np.median(errs)),
           "sampled_per_sphere_error_max": max(serrs), "launch": sim.launch}
    sim.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="a tenth of the steps")
    ap.add_argument("--only", action="append", help="workload names to run")
    args = ap.parse_args()
    q = 10 if args.quick else 1
    adref.build(force=False)
    plan = [
        ("n16", "fp64", 10_000, 1_000),
        ("n512", "fp64", 100_000, 10_000),
        ("n512", "fp32c", 100_000, 10_000),
        ("n4096", "fp32c", 10_000, 1_000),
        ("ens512", "fp32c", 2_000, 250),
    ]
    for name, prec, nsteps, chunk in plan:
        if args.only and name not in args.only:
            continue
        log(f"{name} {prec} {nsteps // q} steps")
        print(json.dumps(trajectory_report(name, prec, nsteps // q, max(1, chunk // q))), flush=True)
    if not args.only or "n65536" in args.only:
        log(f"n65536 fp32c {1000 // q} steps, spot checks")
        print(json.dumps(spot_report("n65536", 1000 // q, 50 if not args.quick else 10)), flush=True)


if __name__ == "__main__":
    main()
