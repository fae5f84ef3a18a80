"""The stored oracle trajectories (tests/golden/*_rk4.npz) are what the
oracle computes today: the manifest's file hashes and source hashes match,
and the first records of the 512-sphere run and of two sampled ensemble
systems are recomputed here and compared bit for bit."""
import hashlib
import json

import numpy as np

from workload import make_preset


def _sha(path):
    return hashlib.sha256(path.read_bytes()).hexdigest()


def _manifest(golden_dir):
    return json.loads((golden_dir / "config_goldens.json").read_text())


def test_manifest_matches_files_and_sources(golden_dir):
    man = _manifest(golden_dir)
    root = golden_dir.parents[1]
    assert man["oracle_sha256"] == _sha(root / "oracle" / "adref.c")
    assert man["workload_sha256"] == _sha(root / "workload" / "suspensions.py")
    for name, entry in man["files"].items():
        assert _sha(golden_dir / name) == entry["sha256"], name


def test_n512_first_record_recomputes(oracle, golden_dir):
    with np.load(golden_dir / "n512_rk4.npz", allow_pickle=False) as z:
        rec = int(z["record_every"])
        cen0 = z["centres"][0]
        com0 = z["com"][0]
    sus = make_preset("n512")
    _, cen, com, _ = oracle.run(sus.params, sus.X, sus.phi, rec, record_every=rec)
    assert np.array_equal(cen[0], cen0) and np.array_equal(com[0], com0)


def test_ens512_sampled_systems_recompute(oracle, golden_dir):
    with np.load(golden_dir / "ens512_rk4.npz", allow_pickle=False) as z:
        rec = int(z["record_every"])
        systems, S, cen = z["systems"], z["S"], z["centres"]
    ens = make_preset("ens512")
    off = np.concatenate([[0], np.cumsum(S)])
    for k in (int(np.argmin(S)), 5):
        sysb = ens.system(int(systems[k]))
        _, c, _, _ = oracle.run(ens.params, sysb.X, sysb.phi, rec, record_every=rec)
        assert np.array_equal(c[0], cen[0, off[k]:off[k + 1]])
