"""Autotuner for the pair-kernel launch shape.

For a given set of system sizes it tries launch shapes (targets per lane,
j-chunk, work-group size, waves per j-tile, position split), rejects every
shape whose FP32C velocities differ from the library's own FP64 path by more
than an error gate, and keeps the one with the shortest graph-replayed RK4
step. Results are stored per size bucket in a JSON table that
`Simulator(..., launch="tuned")` reads.
"""
from __future__ import annotations

import json
import math
from pathlib import Path

import numpy as np

from . import binding as B

TABLE = Path(__file__).resolve().parent / "tuning_gfx950.json"


# an ensemble of fewer systems than this is tuned apart: its wide work list
# (64 targets per work-group) can hold fewer work-groups than there are CUs
FEW_SYSTEMS = 32


def bucket_key(S_per_sys) -> str:
    """Size bucket of a workload: one system by N rounded to a power of two,
    an ensemble by the power-of-two bucket of its largest system, with
    ":few" appended for fewer than FEW_SYSTEMS systems."""
    S = np.asarray(S_per_sys).reshape(-1)
    n = int(2 * S.max())
    p2 = 1 << max(0, math.ceil(math.log2(max(n, 1))))
    if len(S) == 1:
        return f"single:N<={p2}"
    return f"ensemble:N<={p2}" + (":few" if len(S) < FEW_SYSTEMS else "")


def load_table(path: Path = TABLE) -> dict:
    if path.exists():
        return json.loads(path.read_text())
    return {}


def tuned_launch(S_per_sys, path: Path = TABLE):
    """The table's launch for the workload's size bucket. A few-system
    ensemble whose ":few" bucket is not tuned takes its size bucket's entry.
    A workload smaller than the smallest tuned bucket of its kind (single or
    ensemble) takes that bucket's launch, which holds for any smaller size;
    any other bucket the table lacks gets None (the library default, two
    kernels per stage)."""
    table = load_table(path)
    key = bucket_key(S_per_sys)
    plain = key.removesuffix(":few")
    for k in (key, plain):
        if k in table:
            return table[k].get("launch")
    kind, n = plain.split(":N<=")
    tuned = sorted(int(k.split(":N<=")[1]) for k in table if k.startswith(kind + ":N<=") and not k.endswith(":few"))
    if tuned and int(n) < tuned[0]:
        return table[f"{kind}:N<={tuned[0]}"].get("launch")
    return None


# the plain FP64 forms take the resident form (one work-group per system, every
# stage of a run of steps in one launch; bitwise the same sums as the
# two-kernel form) up to this many spheres per system: 16 spheres 4.4 us per
# step against 34 for two kernels per stage, 64 lattices of 27 dumbbells 24
# against 70. Past about 64 spheres its term chunks become long sequential
# loops per thread and the two-kernel form wins.
RESIDENT_FP64_MAX = 64
RESIDENT_FP64 = {"ipl": 1, "jchunk": 128, "wg": 64, "wj": 1, "posmode": 0, "fused": 4}


def tuned_launch_fp64(S_per_sys, steric: bool = False):
    """Launch of the plain FP64 forms (AD_FP64, AD_FP64_TILED) under
    launch="tuned": the resident form for systems of up to RESIDENT_FP64_MAX
    spheres without steric forces, else None (the library default)."""
    S = np.asarray(S_per_sys).reshape(-1)
    if steric or len(S) == 0 or 2 * int(S.max()) > RESIDENT_FP64_MAX:
        return None
    return dict(RESIDENT_FP64)


def candidates(N: int, ensemble: bool):
    out = []
    for posmode in (B.AD_POS_HILO, B.AD_POS_SINGLE):
        if ensemble or N < 1024:
            for ipl in (1, 2):
                for jc in (128, 256, 512):
                    out.append(dict(wg=64, wj=1, ipl=ipl, jchunk=jc, posmode=posmode))
            for jc in (256, 512):
                out.append(dict(wg=256, wj=4, ipl=1, jchunk=jc, posmode=posmode))
            continue
        # j-chunks from 256 up to a size that leaves about 256 work-groups
        top = max(256, min(N, 256 * (1 << max(0, math.ceil(math.log2(max(1.0, N * N / (64 * 256 * 256))))))))
        for ipl in (1, 2, 4):
            jc = 128
            while jc <= top:
                out.append(dict(wg=256, wj=4, ipl=ipl, jchunk=jc, posmode=posmode))
                jc *= 2
        for ipl in (1, 2):
            out.append(dict(wg=256, wj=1, ipl=ipl, jchunk=256, posmode=posmode))
            for jc in (128, 256):
                out.append(dict(wg=64, wj=1, ipl=ipl, jchunk=jc, posmode=posmode))
    # one kernel per stage with every source of a system in LDS (refused where
    # it does not apply); the other fields serve ad_mobility_apply
    for posmode in (B.AD_POS_HILO, B.AD_POS_SINGLE):
        if ensemble:
            out.append(dict(wg=64, wj=1, ipl=1, jchunk=128, posmode=posmode, fused=1))
            out.append(dict(wg=64, wj=1, ipl=1, jchunk=128, posmode=posmode, fused=2))
            if N >= 1024:
                out.append(dict(wg=64, wj=1, ipl=1, jchunk=128, posmode=posmode, fused=3))
        else:
            out.append(dict(wg=256, wj=4, ipl=1, jchunk=256, posmode=posmode, fused=1))
            if N >= 256:  # the streamed form pads every system to 1024 sources
                out.append(dict(wg=256, wj=4, ipl=1, jchunk=256, posmode=posmode, fused=3))
        if N <= 256:  # the resident form: one work-group per system for a run of steps
            out.append(dict(wg=64, wj=1, ipl=1, jchunk=128, posmode=posmode, fused=4))
    uniq = []
    for c in out:
        if c not in uniq:
            uniq.append(c)
    return uniq


def _relerr(u, ref, offsets):
    """The largest per-system relative error: the bar of the velocity and
    drift checks holds for every system, and a norm over the whole ensemble
    would dilute a small system's error by the large ones."""
    import torch
    worst = 0.0
    for b in range(len(offsets) - 1):
        sl = slice(int(offsets[b]), int(offsets[b + 1]))
        worst = max(worst, float(torch.linalg.norm(u[sl] - ref[sl]) / torch.linalg.norm(ref[sl])))
    return worst


def _step_time(sim, steps: int) -> float:
    import torch
    sim.step(max(2, steps // 10))
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    sim.step(steps)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def gate_states(params, X, seed: int = 12345):
    """The states a launch shape must pass: the given positions with forces
    at t = 0.37 T, and the positions displaced by N(0, (0.2 a)^2) per
    coordinate with forces at t = 0.03 T. The displaced state stretches every
    spring and, where steric forces are on, pushes spheres into overlap, so
    dumbbells carry net forces whose far fields decay like 1/r; single-float
    positions lose most there in large boxes."""
    Xp = X + np.random.default_rng(seed).normal(scale=0.2 * params.a, size=X.shape)
    return [(X, 0.37 * params.T), (Xp, 0.03 * params.T)]


def tune(params, S_per_sys, X, phi, gate: float = 5e-7, steps: int = 50, cands=None, verbose=False) -> dict:
    """Tune on the state (X, phi). Returns {"launch", "ms_per_step", "err",
    "tried"}. A shape's error is the largest, over the gate states and the
    systems, relative difference between its velocities and AD_FP64_TILED
    velocities at the same positions and forces (forces from ad_forces), and
    between its displacement over one step from that state and
    AD_FP64_TILED's."""
    import torch
    S_per_sys = np.asarray(S_per_sys, dtype=np.int32).reshape(-1)
    offsets = np.concatenate([[0], np.cumsum(2 * S_per_sys.astype(np.int64))])
    ref = B.Simulator(params, S_per_sys, precision="fp64_tiled")
    ref.set_state(X, phi)
    states = []
    for Xs, t in gate_states(params, X):
        Xd = torch.as_tensor(Xs, dtype=torch.float64, device=ref.device).contiguous()
        F = ref.forces(Xd, t)
        u = ref.mobility(Xd, F)
        ref.set_state(Xs, phi)
        ref.step(1)
        states.append((Xs, Xd, F, u, ref.get_state()[0] - Xd))
    ref.close()
    sim = B.Simulator(params, S_per_sys, precision="fp32c", graph=True)
    sim.set_state(X, phi)
    N = int(2 * S_per_sys.max())
    tried = []
    best = None
    for c in (cands or candidates(N, len(S_per_sys) > 1)):
        try:
            sim.set_launch(**c)
        except B.ADError as e:
            tried.append({"launch": c, "error": str(e)})
            continue
        err = 0.0
        for Xs, Xd, F, u_ref, dX_ref in states:
            err = max(err, _relerr(sim.mobility(Xd, F), u_ref, offsets))
            # one step from the same state: the step path (fused or not)
            sim.set_state(Xs, phi)
            sim.step(1)
            err = max(err, _relerr(sim.get_state()[0] - Xd, dX_ref, offsets))
        sim.set_state(X, phi)
        rec = {"launch": sim.launch, "err": err}
        if err <= gate:
            rec["ms_per_step"] = _step_time(sim, steps)
            if best is None or rec["ms_per_step"] < best["ms_per_step"]:
                best = rec
        tried.append(rec)
        if verbose:
            print(json.dumps(rec), flush=True)
    sim.close()
    if best is None:
        raise RuntimeError("no launch shape met the error gate")
    return {"launch": best["launch"], "ms_per_step": best["ms_per_step"], "err": best["err"],
            "gate": gate, "tried": tried}


def store(S_per_sys, result: dict, path: Path = TABLE) -> None:
    table = load_table(path)
    table[bucket_key(S_per_sys)] = {k: result[k] for k in ("launch", "ms_per_step", "err", "gate")}
    path.write_text(json.dumps(table, indent=1, sort_keys=True) + "\n")


def tuning_workload(name: str):
    """A named workload to tune on: a preset (n512, n4096, ens512, ...),
    "single:N" (one suspension of N spheres at the density of the 4096-sphere
    preset, side 240 (N/4096)^(1/3)), or "arrays:x:W" (W checkerboard x^3
    arrays at spacing 10 ell with the Fig. 1 parameters, one ensemble)."""
    from workload import array_runs, fig1_params, make_preset, make_single
    if name.startswith("single:"):
        N = int(name.split(":")[1])
        return make_single(N // 2, 240.0 * (N / 4096.0) ** (1.0 / 3.0), 0)
    if name.startswith("arrays:"):
        _, x, W = name.split(":")
        p = fig1_params()
        return array_runs(int(x), 10 * p.ell, int(W), "checkerboard", params=p)[0]
    return make_preset(name)


def main(argv=None):
    """Tune named synthetic workloads and write the table:
    python -m paper_1004_1932_amd.autotune --workload n4096 --out table.json"""
    import argparse
    import sys

    sys.path.insert(0, str(Path(__file__).resolve().parents[1]))

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", action="append", required=True)
    ap.add_argument("--out", default=str(TABLE))
    ap.add_argument("--gate", type=float, default=5e-7)
    ap.add_argument("--steps", type=int, default=50)
    args = ap.parse_args(argv)
    for name in args.workload:
        w = tuning_workload(name)
        sizes = getattr(w, "S_per_sys", None)
        sizes = [w.S] if sizes is None else sizes
        print(f"tuning {name}", flush=True)
        res = tune(w.params, sizes, w.X, w.phi, gate=args.gate, steps=args.steps, verbose=True)
        store(sizes, res, Path(args.out))
        print(json.dumps({"workload": name, "launch": res["launch"], "ms_per_step": res["ms_per_step"],
                          "err": res["err"]}), flush=True)


if __name__ == "__main__":
    main()
