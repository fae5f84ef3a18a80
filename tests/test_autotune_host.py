"""Host logic of the autotuner: size buckets, candidate shapes, the tuning
workloads and the shipped table (no GPU needed)."""
import json

import numpy as np

from paper_1004_1932_amd import autotune as A


def test_bucket_keys():
    assert A.bucket_key([2048]) == "single:N<=4096"
    assert A.bucket_key([2049]) == "single:N<=8192"
    assert A.bucket_key([256]) == "single:N<=512"
    assert A.bucket_key([16, 400, 3]) == "ensemble:N<=1024:few"
    assert A.bucket_key(np.array([27] * 64)) == "ensemble:N<=64"
    assert A.bucket_key(np.array([343] * 10)) == "ensemble:N<=1024:few"
    assert A.bucket_key(np.array([343] * 32)) == "ensemble:N<=1024"


def test_tuned_launch_below_and_between_buckets(tmp_path):
    """A size below the smallest tuned bucket of its kind takes that bucket's
    launch; a missing bucket above it gets the library default (None)."""
    rec = lambda f: {"launch": {"fused": f}, "ms_per_step": 1.0, "err": 0.0, "gate": 5e-7}
    path = tmp_path / "t.json"
    path.write_text(json.dumps({"single:N<=512": rec(1), "single:N<=4096": rec(3), "ensemble:N<=64": rec(2),
                                "ensemble:N<=1024": rec(2), "ensemble:N<=1024:few": rec(1)}))
    assert A.tuned_launch([8], path) == {"fused": 1}          # N = 16
    assert A.tuned_launch([256], path) == {"fused": 1}        # its own bucket
    assert A.tuned_launch([700], path) is None                # N <= 2048 missing, above the smallest
    assert A.tuned_launch([2048], path) == {"fused": 3}
    assert A.tuned_launch([3, 5], path) == {"fused": 2}       # ensemble N <= 16
    assert A.tuned_launch([100, 5], path) is None             # ensemble N <= 256 missing
    assert A.tuned_launch([343] * 10, path) == {"fused": 1}   # the few-system bucket
    assert A.tuned_launch([343] * 40, path) == {"fused": 2}   # many systems
    assert A.tuned_launch([20] * 10, path) == {"fused": 2}    # no N <= 64 few bucket: its size bucket
    assert A.tuned_launch([8], tmp_path / "none.json") is None


def test_tuning_workloads_land_in_their_buckets():
    for name, key, nsys in (("single:1024", "single:N<=1024", 1), ("single:8192", "single:N<=8192", 1),
                            ("arrays:3:4", "ensemble:N<=64:few", 4), ("arrays:5:2", "ensemble:N<=256:few", 2),
                            ("ens512", "ensemble:N<=1024", 512)):
        w = A.tuning_workload(name)
        S = getattr(w, "S_per_sys", None)
        S = [w.S] if S is None else S
        assert A.bucket_key(S) == key and len(S) == nsys, name


def test_candidates_are_unique_and_include_the_fused_form():
    for N, ens in ((512, False), (4096, False), (65536, False), (800, True)):
        c = A.candidates(N, ens)
        assert len(c) == len({json.dumps(x, sort_keys=True) for x in c})
        assert any(x.get("fused") == 1 for x in c)


def test_shipped_table_is_gated():
    """Every stored shape passed the accuracy gate it was tuned under."""
    table = A.load_table()
    assert "single:N<=4096" in table
    for key, rec in table.items():
        assert rec["err"] <= rec["gate"] <= 5e-7, key
        assert rec["ms_per_step"] > 0 and isinstance(rec["launch"], dict), key


def test_fp64_tuned_launch_is_resident_for_small_systems():
    """launch="tuned" for the plain FP64 forms: the resident form for systems
    of up to 64 spheres without steric forces, else the library default."""
    assert A.tuned_launch_fp64([8]) == A.RESIDENT_FP64
    assert A.tuned_launch_fp64([27] * 64)["fused"] == 4
    assert A.tuned_launch_fp64([32, 5]) == A.RESIDENT_FP64
    assert A.tuned_launch_fp64([33]) is None
    assert A.tuned_launch_fp64([8], steric=True) is None
    assert A.tuned_launch_fp64([]) is None
