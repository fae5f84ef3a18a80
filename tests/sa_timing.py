"""Time the stroke-averaged equations (Sec. III) on the GPU: one checkerboard
lattice of x^3 dumbbells at spacing 10 ell with the Fig. 1 parameters, RK4
steps of T/20, for x = 5, 7, 9 (the paper's arrays) and 16 (4096 dumbbells).
Prints one JSON line per size: microseconds per RK4 step and pair
evaluations per second (4 S (S - 1) per step).

    python tests/sa_timing.py
"""
import json
import sys
import time
from pathlib import Path

sys.path.insert(0, str(Path(__file__).resolve().parents[1]))


def main(steps: int = 2000):
    import torch

    import paper_1004_1932_amd as P
    from workload import fig1_params, lattice_array

    p = fig1_params(0.2, 5000)
    for x in (5, 7, 9, 16):
        R, N, phi = lattice_array(x, 10 * p.ell, 3, "checkerboard")
        sa = P.StrokeAveraged(p, R, N, phi)
        assert sa.run(p.T / 20, 20) == 0  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        assert sa.run(p.T / 20, steps) == 0
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        S = len(R)
        print(json.dumps({"dumbbells": S, "us_per_step": dt / steps * 1e6,
                          "pair_evaluations_per_s": 4 * S * (S - 1) * steps / dt}), flush=True)


if __name__ == "__main__":
    main()
