"""The C-ABI library loads, exports what include/ad.h declares, and rejects
bad arguments before touching a device (no GPU needed)."""
import ctypes as C
import re
from dataclasses import replace
from pathlib import Path

import numpy as np
import pytest

import paper_1004_1932_amd as P
from paper_1004_1932_amd import binding as B
from workload import Params

ROOT = Path(__file__).resolve().parents[1]


def declared_symbols():
    text = (ROOT / "include" / "ad.h").read_text()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(ad_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("ad_create", "ad_set_state", "ad_forces", "ad_mobility_apply", "ad_step", "ad_run"):
        assert required in names
    assert sorted(B.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(str(P.LIB_PATH))
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    # 9 doubles, 4 int32, kT, seed
    assert C.sizeof(B.ad_params) == 9 * 8 + 4 * 4 + 8 + 8
    assert C.sizeof(B.ad_launch) == 24


@pytest.mark.parametrize("bad", [dict(a=0.0), dict(eta=-1.0), dict(T=0.0), dict(dt=float("nan")),
                                 dict(k=float("inf"))])
def test_create_rejects_bad_parameters(bad):
    p = replace(Params(), **bad)
    with pytest.raises(P.ADError) as e:
        P.ad_create(P.make_params(p), [4])
    assert e.value.code == B.AD_EINVAL
    assert P.ad_last_error(None)


def test_create_rejects_bad_sizes_and_enums():
    with pytest.raises(P.ADError):
        P.ad_create(P.make_params(Params()), [4, 0])
    with pytest.raises(P.ADError):
        P.ad_create(P.make_params(Params()), np.zeros(0, np.int32))
    bad = P.make_params(Params())
    bad.precision = 7
    with pytest.raises(P.ADError):
        P.ad_create(bad, [4])
    bad = P.make_params(Params())
    bad.integrator = 3
    with pytest.raises(P.ADError):
        P.ad_create(bad, [4])
    bad = P.make_params(Params())
    bad.tensor = 5
    with pytest.raises(P.ADError):
        P.ad_create(bad, [4])
    P.ad_destroy(P.ad_create(P.make_params(Params(), tensor="rpy"), [4]))
    with pytest.raises(P.ADError):  # noise needs Heun
        P.ad_create(P.make_params(Params(), integrator="rk4", kT=0.1), [4])
    with pytest.raises(P.ADError):
        P.ad_create(P.make_params(Params(), integrator="heun", kT=-1.0), [4])
    P.ad_destroy(P.ad_create(P.make_params(Params(), integrator="heun", kT=0.1, seed=3), [4]))


def test_calls_before_workspace_fail_cleanly():
    ctx = P.ad_create(P.make_params(Params()), [8])
    try:
        lib = P.lib()
        assert lib.ad_step(ctx, 1, None) == B.AD_ESTATE
        assert "workspace" in P.ad_last_error(ctx)
        assert lib.ad_check(ctx, None) == B.AD_ESTATE
        assert lib.ad_mobility_apply(ctx, None, None, None, None) == B.AD_ESTATE
        assert lib.ad_bind_workspace(ctx, None, 0) == B.AD_EINVAL
        assert lib.ad_bind_workspace(ctx, C.c_void_p(256), 16) == B.AD_ENOMEM
        assert lib.ad_bind_workspace(ctx, C.c_void_p(100), 1 << 30) == B.AD_EINVAL
    finally:
        P.ad_destroy(ctx)


def test_launch_shapes_and_workspace_size():
    ctx = P.ad_create(P.make_params(Params(), "fp32c"), [2048])
    try:
        L = P.ad_get_launch(ctx)
        assert L["wg"] in (64, 256) and L["ipl"] in (1, 2, 4) and L["jchunk"] >= 64
        P.ad_set_launch(ctx, ipl=4, jchunk=4096, wg=256)
        one_chunk = P.ad_workspace_size(ctx)
        P.ad_set_launch(ctx, ipl=4, jchunk=64, wg=256)
        assert P.ad_get_launch(ctx) == {"ipl": 4, "jchunk": 64, "wg": 256, "wj": 4, "posmode": 1, "fused": 0}
        # 64 j-chunks hold 64 partial sums per sphere instead of one
        assert P.ad_workspace_size(ctx) - one_chunk >= 63 * 3 * 4096 * 8
        P.ad_set_launch(ctx, ipl=2, jchunk=512, wg=256, wj=4, posmode=2)
        assert P.ad_get_launch(ctx)["posmode"] == 2
        for bad in (dict(ipl=3), dict(wg=128), dict(jchunk=32), dict(wg=256, wj=2), dict(wg=64, wj=4),
                    dict(posmode=3)):
            with pytest.raises(P.ADError):
                P.ad_set_launch(ctx, **bad)
    finally:
        P.ad_destroy(ctx)
    ctx = P.ad_create(P.make_params(Params(), "fp64"), [2048])
    try:
        with pytest.raises(P.ADError):
            P.ad_set_launch(ctx, ipl=4)
        with pytest.raises(P.ADError):
            P.ad_set_launch(ctx, wg=256, wj=4)
    finally:
        P.ad_destroy(ctx)


def test_dense_mode_launch_rules_and_workspace():
    """AD_FP64_DENSE keeps each system's 3Nb x 3Nb FP64 tensor in the
    workspace (72 Nb^2 bytes) and takes only its own launch shape."""
    S = [64, 40]
    sizes = {}
    for prec in ("fp64_tiled", "fp64_dense"):
        ctx = P.ad_create(P.make_params(Params(), prec), S)
        try:
            sizes[prec] = P.ad_workspace_size(ctx)
            if prec == "fp64_dense":
                L = P.ad_get_launch(ctx)
                assert L["wg"] == 256 and L["ipl"] == 1 and L["wj"] == 1 and 64 <= L["jchunk"] <= 1024
                P.ad_set_launch(ctx, jchunk=64)
                assert P.ad_get_launch(ctx)["jchunk"] == 64
                for bad in (dict(jchunk=2048), dict(jchunk=32), dict(wg=64), dict(ipl=2), dict(posmode=1)):
                    with pytest.raises(P.ADError):
                        P.ad_set_launch(ctx, **bad)
        finally:
            P.ad_destroy(ctx)
    tensor = sum(72 * (2 * s) ** 2 for s in S)
    assert sizes["fp64_dense"] - sizes["fp64_tiled"] >= tensor
    # 32 GiB of tensors at most: N = 2 * 12000 needs 41 GB
    with pytest.raises(P.ADError):
        P.ad_create(P.make_params(Params(), "fp64_dense"), [12000])
    P.ad_destroy(P.ad_create(P.make_params(Params(), "fp64_dense"), [8000]))


def test_fused_stage_launch_rules():
    """launch.fused: AD_FP32C, no steric forces, every source of a system in
    LDS (6784 spheres with single-float positions, 4544 with hi/lo; ensembles
    of systems up to those sizes)."""
    ctx = P.ad_create(P.make_params(Params(), "fp32c"), [2048])
    try:
        P.ad_set_launch(ctx, fused=1, posmode=2)
        assert P.ad_get_launch(ctx)["fused"] == 1
        P.ad_set_launch(ctx, fused=1, posmode=1)
        with pytest.raises(P.ADError):
            P.ad_set_launch(ctx, fused=4)
        with pytest.raises(P.ADError):
            P.ad_set_launch(ctx, fused=-1)
    finally:
        P.ad_destroy(ctx)
    ok = P.ad_create(P.make_params(Params(), "fp32c"), [3392])      # 6784 spheres
    try:
        P.ad_set_launch(ok, fused=1, posmode=2)
        with pytest.raises(P.ADError):
            P.ad_set_launch(ok, fused=1, posmode=1)                    # hi/lo: 4544 at most
    finally:
        P.ad_destroy(ok)
    ens = P.ad_create(P.make_params(Params(), "fp32c"), [64, 32, 5])
    try:
        P.ad_set_launch(ens, fused=1, posmode=1)
        assert P.ad_get_launch(ens)["fused"] == 1
    finally:
        P.ad_destroy(ens)
    for prec, sizes, params in (("fp64", [64], Params()), ("fp64_tiled", [64], Params()),
                                ("fp32c", [3400], Params()), ("fp32c", [10, 3500], Params()),
                                ("fp32c", [64], Params(steric_k=100.0, steric_r=2.0))):
        ctx = P.ad_create(P.make_params(params, prec), sizes)
        try:
            with pytest.raises(P.ADError):
                P.ad_set_launch(ctx, fused=1, posmode=2 if prec == "fp32c" else 0)
        finally:
            P.ad_destroy(ctx)


def test_wide_fused_stage_launch_rules():
    """launch.fused = 2 (64 targets per work-group): the same rules as the
    first form, with sources padded to 4 instead of 4 x waves, so systems of
    up to 6824 spheres single-float and 4548 hi/lo fit; one system or an
    ensemble; the work list holds one item per 64-target block."""
    for sizes in ([2048], [64, 32, 5], [16, 400, 3, 27]):
        ctx = P.ad_create(P.make_params(Params(), "fp32c"), sizes)
        try:
            for posmode in (1, 2):
                P.ad_set_launch(ctx, fused=2, posmode=posmode)
                assert P.ad_get_launch(ctx)["fused"] == 2
            P.ad_set_launch(ctx, fused=1, posmode=2)
            P.ad_set_launch(ctx, fused=2, posmode=2)
            P.ad_set_launch(ctx, fused=0)
        finally:
            P.ad_destroy(ctx)
    ok = P.ad_create(P.make_params(Params(), "fp32c"), [3412])      # 6824 spheres
    try:
        P.ad_set_launch(ok, fused=2, posmode=2)
        with pytest.raises(P.ADError):
            P.ad_set_launch(ok, fused=1, posmode=2)                    # 16-wave form: 6784 at most
        with pytest.raises(P.ADError):
            P.ad_set_launch(ok, fused=2, posmode=1)
    finally:
        P.ad_destroy(ok)
    hl = P.ad_create(P.make_params(Params(), "fp32c"), [2274])       # 4548 spheres
    try:
        P.ad_set_launch(hl, fused=2, posmode=1)
    finally:
        P.ad_destroy(hl)
    for prec, sizes, params in (("fp64", [64], Params()), ("fp64_dense", [64], Params()),
                                ("fp32c", [3414], Params()), ("fp32c", [10, 3414], Params()),
                                ("fp32c", [64, 8], Params(steric_k=100.0, steric_r=2.0))):
        ctx = P.ad_create(P.make_params(params, prec), sizes)
        try:
            with pytest.raises(P.ADError):
                P.ad_set_launch(ctx, fused=2, posmode=2 if prec == "fp32c" else 0)
        finally:
            P.ad_destroy(ctx)


def test_streamed_fused_stage_launch_rules():
    """launch.fused = 3 (sources streamed per wave): AD_FP32C or
    AD_FP64_TILED without steric forces, any system size (no LDS limit), one
    system or an ensemble; not the plain FP64 form (bitwise the sequential
    sum) nor the dense one."""
    for sizes in ([2048], [3414], [20000], [64, 32, 5]):
        ctx = P.ad_create(P.make_params(Params(), "fp32c"), sizes)
        try:
            for posmode in (1, 2):
                P.ad_set_launch(ctx, fused=3, posmode=posmode)
                assert P.ad_get_launch(ctx)["fused"] == 3
        finally:
            P.ad_destroy(ctx)
    for sizes in ([2048], [20000], [64, 32, 5]):
        ctx = P.ad_create(P.make_params(Params(), "fp64_tiled"), sizes)
        try:
            P.ad_set_launch(ctx, fused=3, posmode=0)
            assert P.ad_get_launch(ctx)["fused"] == 3
        finally:
            P.ad_destroy(ctx)
    for prec, sizes, params in (("fp64", [64], Params()), ("fp64_dense", [64], Params()),
                                ("fp64_tiled", [64], Params(steric_k=100.0, steric_r=2.0)),
                                ("fp32c", [64, 8], Params(steric_k=100.0, steric_r=2.0))):
        ctx = P.ad_create(P.make_params(params, prec), sizes)
        try:
            with pytest.raises(P.ADError):
                P.ad_set_launch(ctx, fused=3, posmode=2 if prec == "fp32c" else 0)
        finally:
            P.ad_destroy(ctx)


def test_destroy_null_is_noop():
    assert P.lib().ad_destroy(None) == 0


def test_stroke_averaged_entry_points_validate_on_the_host():
    lib = P.lib()
    prm = P.make_params(Params())
    n = C.c_uint64()
    assert lib.ad_sa_workspace_size(0, C.byref(n)) == B.AD_EINVAL
    assert lib.ad_sa_workspace_size(125, C.byref(n)) == 0 and n.value >= 6 * 125 * 24
    fake = C.c_void_p(4096)
    assert lib.ad_sa_run(C.byref(prm), 125, fake, fake, fake, 1.0, 1, fake, 16, None) == B.AD_ENOMEM
    assert lib.ad_sa_run(C.byref(prm), 125, fake, fake, fake, -1.0, 1, fake, n.value, None) == B.AD_EINVAL
    bad = P.make_params(Params(T=0.0))
    assert lib.ad_sa_rhs(C.byref(bad), 125, fake, fake, fake, fake, fake, None) == B.AD_EINVAL


def test_oracle_keeps_sin_and_cos_separate():
    """The oracle's library calls libm sin and cos, never a merged sincos
    (whose last bit differs for some arguments from the separate calls the
    library's host table makes)."""
    import shutil
    import subprocess
    from oracle import adref
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    adref.build(force=False)
    out = subprocess.run(["nm", "-D", str(adref.LIB)], capture_output=True, text=True, check=True).stdout
    undefined = {line.split()[-1].split("@")[0] for line in out.splitlines() if " U " in line}
    assert {"sin", "cos"} <= undefined and "sincos" not in undefined


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; --gpus N > 1 exits at once with a message."""
    import json
    import subprocess
    import sys
    from pathlib import Path
    root = Path(__file__).resolve().parents[1]
    res = subprocess.run([sys.executable, str(root / "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in json.loads(res.stdout.strip().splitlines()[-1])["error"]


def test_resident_launch_limits():
    """launch.fused = 4 (one work-group per system for a run of steps) takes
    systems of at most 256 spheres in AD_FP32C and 128 in the FP64 modes, and
    no steric forces; refused before any device work."""
    def try_launch(S, precision, steric=False):
        p = replace(Params(), steric_k=100.0) if steric else Params()
        ctx = P.ad_create(P.make_params(p, precision), S)
        try:
            P.ad_set_launch(ctx, ipl=1, jchunk=256, wg=64, wj=1, posmode=1 if precision == "fp32c" else 0,
                            fused=4)
            return B.AD_OK
        except P.ADError as e:
            return e.code
        finally:
            P.ad_destroy(ctx)
    assert try_launch([128, 3], "fp32c") == B.AD_OK
    assert try_launch([129], "fp32c") == B.AD_EINVAL
    assert try_launch([64, 10], "fp64") == B.AD_OK
    assert try_launch([65], "fp64") == B.AD_EINVAL
    assert try_launch([64], "fp64_tiled") == B.AD_OK
    assert try_launch([20], "fp32c", steric=True) == B.AD_EINVAL
    assert try_launch([20], "fp64_dense") == B.AD_EINVAL


def test_static_apply_refuses_before_any_device_work():
    """ad_mobility_apply_static (no context, no allocation) rejects null
    pointers, odd sizes and sizes beyond its fixed scratch with a message,
    before touching a device."""
    p = P.make_params(Params(), "fp32c")
    fake = C.c_void_p(256)  # never dereferenced: the checks come first
    lib = P.lib()
    assert lib.ad_mobility_apply_static(C.byref(p), 8, None, fake, fake, None) == B.AD_EINVAL
    assert lib.ad_mobility_apply_static(C.byref(p), 7, fake, fake, fake, None) == B.AD_EINVAL
    assert "even" in P.ad_last_error(None)
    assert lib.ad_mobility_apply_static(C.byref(p), 400000, fake, fake, fake, None) == B.AD_ENOMEM
    assert "scratch" in P.ad_last_error(None)
    bad = P.make_params(Params(), "fp64_dense")
    assert lib.ad_mobility_apply_static(C.byref(bad), 8, fake, fake, fake, None) == B.AD_EINVAL
