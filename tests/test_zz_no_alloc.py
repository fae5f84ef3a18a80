"""ad_mobility_apply_static (the entry point that allocates nothing) through
the C ABI against ad_mobility_apply on a context with the default launch:
two calls in a row, the second on a smaller system, in each precision and
tensor; the same bits (same launch shape, same kernels), and the oracle's
bars as a second check."""
import numpy as np
import pytest

import paper_1004_1932_amd as P
from paper_1004_1932_amd import binding as B
from parity_metrics import check_fp32c, relerr
from workload import make_single

pytestmark = pytest.mark.gpu


def _with_context(sus, precision, tensor, X, F):
    s = P.Simulator(sus.params, [sus.S], precision=precision, tensor=tensor)
    return s.mobility(X, F).cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32c", "fp64", "fp64_tiled"])
@pytest.mark.parametrize("tensor", ["oseen", "rpy"])
def test_static_equals_context_apply(oracle, precision, tensor):
    import torch
    assert torch.cuda.is_available()
    # ragged sizes: 4100 and 3000 span several 64- and 256-target blocks and
    # source chunks with a partial last one (and, in AD_FP64, 4- and 2-target
    # blocks); 150 is below the large-system shape
    for S, side, seed in ((2050, 240.0, 33), (1500, 200.0, 31), (75, 40.0, 32)):
        sus = make_single(S, side, seed)
        rng = np.random.default_rng(seed)
        X = sus.X + rng.normal(scale=0.1, size=sus.X.shape)
        F = rng.standard_normal(sus.X.shape)
        p = B.make_params(sus.params, precision, tensor=tensor)
        Xd = torch.as_tensor(X, device="cuda")
        Fd = torch.as_tensor(F, device="cuda")
        ud = torch.full_like(Xd, float("nan"))
        B.ad_mobility_apply_static(p, Xd, Fd, ud)
        torch.cuda.synchronize()
        u = ud.cpu().numpy()
        uc = _with_context(sus, precision, tensor, X, F)
        print(f"{precision} {tensor} N={2 * S}: equal {np.array_equal(u, uc)}", flush=True)
        assert np.array_equal(u, uc), (precision, tensor, 2 * S)
        uo = oracle.mobility(sus.params, X, F, tensor=1 if tensor == "rpy" else 0)
        if precision == "fp32c":
            check_fp32c(u, uo, f"N={2 * S} against the oracle")
        elif precision == "fp64":
            assert np.array_equal(u, uo)
        else:
            assert relerr(u, uo) <= 1e-13


def test_static_fp64_rpy_beyond_the_block_list():
    """AD_FP64 with RPY at 129,000 spheres: the target-block list no longer
    fits the scratch array beside the rest, so the call sums in the
    one-chunk pair kernel instead; the same bits as the context's call."""
    import torch
    assert torch.cuda.is_available()
    S = 64500
    sus = make_single(S, 1600.0, 34, exclusion=False)
    F = np.random.default_rng(35).standard_normal(sus.X.shape)
    p = B.make_params(sus.params, "fp64", tensor="rpy")
    Xd = torch.as_tensor(sus.X, device="cuda")
    Fd = torch.as_tensor(F, device="cuda")
    ud = torch.full_like(Xd, float("nan"))
    B.ad_mobility_apply_static(p, Xd, Fd, ud)
    torch.cuda.synchronize()
    u = ud.cpu().numpy()
    uc = _with_context(sus, "fp64", "rpy", sus.X, F)
    assert np.isfinite(u).all()
    assert np.array_equal(u, uc)


def test_static_refuses_sizes_and_arguments():
    """Odd N and sizes beyond the 16 MiB scratch are refused before any
    launch, with a message."""
    import torch
    assert torch.cuda.is_available()
    sus = make_single(4, 20.0, 1)
    p = B.make_params(sus.params, "fp32c")
    X = torch.as_tensor(sus.X, device="cuda")
    u = torch.empty_like(X)
    ptr = [B.C.c_void_p(t.data_ptr()) for t in (X, X, u)]
    assert B.lib().ad_mobility_apply_static(B.C.byref(p), 7, *ptr, None) == B.AD_EINVAL
    assert "even" in B.ad_last_error(None)
    assert B.lib().ad_mobility_apply_static(B.C.byref(p), 400000, *ptr, None) == B.AD_ENOMEM
    assert "scratch" in B.ad_last_error(None)
