"""Write the oracle trajectories that the full-length GPU parity tests compare
against (tests/test_gpu_configs.py). Test infrastructure: this script calls
only the FP64 CPU oracle (oracle/) and the seeded input generators
(workload/); no value in the files comes from the GPU library.

    python tests/golden/make_config_goldens.py [--only n512,n4096,ens512]

Files (numpy .npz, plain arrays, no pickles), one per workload, and a
manifest config_goldens.json with each file's sha256, the sha256 of the
oracle source and of the input generator it was made with, and the sizes:

  n512_rk4.npz    S = 256 (N = 512), cube side 120, seed 0, 1e5 RK4 steps:
                  dumbbell centres and the centre of mass every 1e4 steps
                  (10 records), and the final positions.
  n4096_rk4.npz   S = 2048 (N = 4096), cube side 240, seed 0, 1e4 RK4 steps:
                  centres and centre of mass every 1000 steps, final positions.
  ens512_rk4.npz  the 512-system ensemble (S_b uniform in [16, 400], density
                  0.02, system b seeded 1 + b), 2000 RK4 steps: 32 of the
                  systems (the largest, the smallest and 30 drawn with
                  default_rng(2024)), each integrated alone (the systems are
                  independent), centres every 500 steps.

Parameters of every run: a = eta = k = 1, ell = 4, lambda = 1, T = 100,
dt = 0.01, Oseen tensor, RK4, t0 = 0.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import sys
import time
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
ROOT = HERE.parents[1]
sys.path.insert(0, str(ROOT))

from oracle import adref  # noqa: E402
from workload import make_preset  # noqa: E402

MANIFEST = HERE / "config_goldens.json"

# workload -> (steps, record interval)
RUNS = {"n512": (100_000, 10_000), "n4096": (10_000, 1_000), "ens512": (2_000, 500)}
ENS_SAMPLE = 32
ENS_SAMPLE_SEED = 2024


def sha256(path: Path) -> str:
    return hashlib.sha256(path.read_bytes()).hexdigest()


def ens_sample(S_per_sys: np.ndarray) -> np.ndarray:
    """The sampled systems of the ensemble: largest, smallest, 30 random."""
    order = np.argsort(S_per_sys, kind="stable")
    pick = [int(order[-1]), int(order[0])]
    rest = np.setdiff1d(np.arange(len(S_per_sys)), pick)
    pick += [int(b) for b in np.random.default_rng(ENS_SAMPLE_SEED).choice(rest, ENS_SAMPLE - 2, replace=False)]
    return np.array(sorted(pick), dtype=np.int64)


def make_single_run(name: str) -> dict:
    steps, rec = RUNS[name]
    sus = make_preset(name)
    X, cen, com, _ = adref.run(sus.params, sus.X, sus.phi, steps, record_every=rec)
    return {"steps": np.int64(steps), "record_every": np.int64(rec), "centres": cen, "com": com, "X": X}


def make_ens_run() -> dict:
    steps, rec = RUNS["ens512"]
    ens = make_preset("ens512")
    pick = ens_sample(ens.S_per_sys)
    cens = []
    for b in pick:
        sysb = ens.system(int(b))
        _, cen, _, _ = adref.run(ens.params, sysb.X, sysb.phi, steps, record_every=rec)
        cens.append(cen)
    return {"steps": np.int64(steps), "record_every": np.int64(rec), "systems": pick,
            "S": ens.S_per_sys[pick].astype(np.int64), "centres": np.concatenate(cens, axis=1)}


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=",".join(RUNS))
    args = ap.parse_args()
    adref.build(force=False)
    manifest = json.loads(MANIFEST.read_text()) if MANIFEST.exists() else {}
    manifest["oracle_sha256"] = sha256(ROOT / "oracle" / "adref.c")
    manifest["workload_sha256"] = sha256(ROOT / "workload" / "suspensions.py")
    manifest.setdefault("files", {})
    for name in args.only.split(","):
        t = time.perf_counter()
        data = make_ens_run() if name == "ens512" else make_single_run(name)
        path = HERE / f"{name}_rk4.npz"
        np.savez_compressed(path, **data)
        manifest["files"][path.name] = {"sha256": sha256(path), "workload": name,
                                        "steps": int(data["steps"]), "record_every": int(data["record_every"])}
        print(f"{path.name}: {time.perf_counter() - t:.1f} s", flush=True)
    MANIFEST.write_text(json.dumps(manifest, indent=1, sort_keys=True) + "\n")


if __name__ == "__main__":
    main()
