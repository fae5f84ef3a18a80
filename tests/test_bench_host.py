"""bench.py names a kernel for every stage form the library accepts."""
import importlib.util
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_kernel_names_cover_every_stage_form():
    spec = importlib.util.spec_from_file_location("bench_module", ROOT / "bench.py")
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    assert sorted(bench.KERNEL_NAMES) == [0, 1, 2, 3, 4]
