"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Bars (written in each test):
  * AD_FP64 (sequential j, fixed operation order, no FMA): bitwise equal.
  * AD_FP64_TILED: relative velocity error <= 1e-13 (only the summation order
    differs).
  * AD_FP32C: relative velocity error <= 1e-6 per evaluation (the norm of the
    error over one system's 3N components divided by the norm of the oracle
    velocity), relative centre displacement drift <= 1e-4 over 1e4 steps.
"""
import math
import os

import numpy as np
import pytest

import paper_1004_1932_amd as P
from parity_metrics import check_fp32c
from workload import Params, make_ensemble, make_single, make_preset

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def say(msg):
    print(msg, flush=True)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def perturbed(sus, scale=0.05, seed=1):
    return sus.X + np.random.default_rng(seed).normal(scale=scale, size=sus.X.shape)


def sim(sus_or_S, params, precision, **kw):
    S = [sus_or_S.S] if hasattr(sus_or_S, "S") else sus_or_S
    return P.Simulator(params, S, precision=precision, **kw)


# ---------------------------------------------------------------- forces

def test_forces_bitwise(oracle):
    _torch()
    for name, sus in (("n16", make_preset("n16")), ("n512", make_preset("n512"))):
        say(f"forces {name}")
        s = sim(sus, sus.params, "fp64")
        s.set_state(sus.X, sus.phi)
        X = perturbed(sus, 0.1)
        for t in (0.0, 13.37, 2500.25):
            F = s.forces(X, t).cpu().numpy()
            assert np.array_equal(F, oracle.forces(sus.params, X, sus.phi, t))


def test_forces_bitwise_over_stage_times(oracle):
    """Spring forces at 2000 RK4 stage times spread over the first 60 000
    steps, t = 487.305 among them (the half-step time of step 48 730, where
    the oracle's sin and cos once came from a merged sincos call): the host
    (sin, cos)(omega t) of the library and of the oracle agree bitwise."""
    _torch()
    sus = make_preset("n512")
    s = sim(sus, sus.params, "fp64")
    s.set_state(sus.X, sus.phi)
    dt = sus.params.dt
    steps = np.random.default_rng(9).integers(0, 60_000, 1999)
    times = [48_730 * dt + 0.5 * dt] + [n * dt + 0.5 * dt for n in steps[:999]] + [n * dt + dt for n in steps[999:]]
    bad = []
    for t in times:
        F = s.forces(sus.X, t).cpu().numpy()
        if not np.array_equal(F, oracle.forces(sus.params, sus.X, sus.phi, t)):
            bad.append(t)
    assert not bad, bad[:5]


def test_forces_steric_bitwise(oracle):
    _torch()
    p = Params(steric_k=100.0, steric_r=2.0)
    sus = make_single(40, 14.0, 5, p, exclusion=False)
    s = sim(sus, p, "fp64")
    s.set_state(sus.X, sus.phi)
    F = s.forces(sus.X, 1.0).cpu().numpy()
    Fo = oracle.forces(p, sus.X, sus.phi, 1.0)
    assert np.abs(Fo).max() > 1.0  # overlaps present
    assert np.array_equal(F, Fo)


# ---------------------------------------------------------------- mobility

@pytest.mark.parametrize("S,side", [(1, 10.0), (3, 12.0), (8, 40.0), (37, 40.0), (256, 120.0)])
def test_mobility_fp64_bitwise(oracle, S, side):
    _torch()
    say(f"mobility fp64 S={S}")
    sus = make_single(S, side, 2)
    F = np.random.default_rng(3).standard_normal(sus.X.shape)
    s = sim(sus, sus.params, "fp64")
    u = s.mobility(sus.X, F).cpu().numpy()
    assert np.array_equal(u, oracle.mobility(sus.params, sus.X, F))


@pytest.mark.parametrize("launch", [None, dict(ipl=1, jchunk=64, wg=64), dict(ipl=2, jchunk=192, wg=256),
                                    dict(ipl=2, jchunk=100, wg=64)])
def test_mobility_fp64_tiled(oracle, launch):
    _torch()
    say(f"mobility fp64_tiled {launch}")
    sus = make_single(700, 150.0, 4)
    F = np.random.default_rng(5).standard_normal(sus.X.shape)
    s = sim(sus, sus.params, "fp64_tiled", launch=launch)
    u = s.mobility(sus.X, F).cpu().numpy()
    assert relerr(u, oracle.mobility(sus.params, sus.X, F)) <= 1e-13


FP32C_LAUNCHES = [None, dict(ipl=1, jchunk=64, wg=64), dict(ipl=2, jchunk=320, wg=256, wj=1),
                  dict(ipl=4, jchunk=256, wg=256, wj=4), dict(ipl=1, jchunk=1000, wg=256, wj=4),
                  dict(ipl=4, jchunk=1000, wg=64), dict(ipl=2, jchunk=512, wg=256, wj=4, posmode=2),
                  dict(ipl=1, jchunk=64, wg=64, posmode=2), dict(ipl=1, jchunk=128, wg=256, wj=4, posmode=2),
                  dict(ipl=2, jchunk=100, wg=256, wj=4)]


@pytest.mark.parametrize("launch", FP32C_LAUNCHES)
@pytest.mark.parametrize("S,side", [(1, 10.0), (5, 20.0), (300, 120.0), (2048, 240.0)])
def test_mobility_fp32c(oracle, S, side, launch):
    """Spring-like forces (equal and opposite per dumbbell) at a perturbed
    state, and arbitrary forces; relative velocity error <= 1e-6."""
    _torch()
    say(f"mobility fp32c S={S} {launch}")
    sus = make_single(S, side, 6)
    X = perturbed(sus, 0.2)
    s = sim(sus, sus.params, "fp32c", launch=launch)
    s.set_state(sus.X, sus.phi)
    F = oracle.forces(sus.params, X, sus.phi, 7.0)
    u = s.mobility(X, F).cpu().numpy()
    check_fp32c(u, oracle.mobility(sus.params, X, F), "spring forces")
    G = np.random.default_rng(7).standard_normal(X.shape)
    check_fp32c(s.mobility(X, G).cpu().numpy(), oracle.mobility(sus.params, X, G), "random forces")


@pytest.mark.parametrize("launch", [None, "tuned",
                                    {"ipl": 2, "jchunk": 4096, "wg": 256, "wj": 4, "posmode": 1},
                                    {"ipl": 4, "jchunk": 2048, "wg": 256, "wj": 1, "posmode": 1}])
def test_mobility_fp32c_full_size_sampled(oracle, launch):
    """65536 spheres, default, tuned and large-N launch shapes: 64 sampled
    target spheres against the oracle's rows, error relative to the sampled
    velocity norm."""
    torch = _torch()
    sus = make_preset("n65536")
    say(f"mobility fp32c n65536 sampled, launch {launch}")
    X = perturbed(sus, 0.2)
    F = oracle.forces(sus.params, X, sus.phi, 3.0)
    s = sim(sus, sus.params, "fp32c", launch=launch)
    say(f"  launch {s.launch}")
    u = s.mobility(X, F).cpu().numpy()
    rows = np.random.default_rng(7).choice(sus.N, 64, replace=False)
    uo = oracle.mobility_rows(sus.params, X, F, rows)
    check_fp32c(u[rows], uo, "64 sampled rows")
    del s
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- trajectories

def _run_both(oracle, sus, precision, nsteps, rec, integrator="rk4", launch=None, graph=False, S_per_sys=None):
    p = sus.params
    S = S_per_sys if S_per_sys is not None else [sus.S]
    s = P.Simulator(p, S, precision=precision, integrator=integrator, launch=launch, graph=graph)
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(nsteps, rec)
    assert code == 0
    Xg = s.get_state()[0].cpu().numpy()
    Xo, ceno, como, _ = oracle.run(p, sus.X, sus.phi, nsteps, record_every=rec,
                                   S_per_sys=S, integrator=1 if integrator == "heun" else 0)
    return Xg, cen.cpu().numpy(), com.cpu().numpy(), Xo, ceno, como


@pytest.mark.parametrize("integrator", ["rk4", "heun"])
@pytest.mark.parametrize("graph", [False, True])
def test_trajectory_fp64_bitwise_small(oracle, integrator, graph):
    """16 spheres, 2000 steps: state, centres and centre of mass bitwise."""
    _torch()
    say(f"trajectory fp64 n16 {integrator} graph={graph}")
    sus = make_preset("n16")
    Xg, cg, mg, Xo, co, mo = _run_both(oracle, sus, "fp64", 2000, 250, integrator, graph=graph)
    assert np.array_equal(Xg, Xo)
    assert np.array_equal(cg, co)
    assert np.array_equal(mg, mo)


def test_trajectory_fp64_bitwise_full_n16(oracle):
    """The plain FP64 workload in full: 16 spheres, 1e4 RK4 steps."""
    _torch()
    sus = make_preset("n16")
    Xg, cg, mg, Xo, co, mo = _run_both(oracle, sus, "fp64", 10_000, 1000, graph=True)
    assert np.array_equal(Xg, Xo) and np.array_equal(cg, co) and np.array_equal(mg, mo)


_ORACLE_RUNS = {}


def _oracle_run_cached(oracle, name, nsteps, rec):
    key = (name, nsteps, rec)
    if key not in _ORACLE_RUNS:
        sus = make_preset(name)
        _ORACLE_RUNS[key] = oracle.run(sus.params, sus.X, sus.phi, nsteps, record_every=rec)
    return _ORACLE_RUNS[key]


FUSED_SINGLE = {"ipl": 1, "jchunk": 256, "wg": 256, "wj": 4, "posmode": 2, "fused": 1}
FUSED_HILO = {"ipl": 1, "jchunk": 256, "wg": 256, "wj": 4, "posmode": 1, "fused": 1}


@pytest.mark.parametrize("name,nsteps,launch", [("n512", 10_000, None), ("n512", 10_000, "tuned"),
                                                ("n4096", 1_000, "tuned"), ("n512", 10_000, FUSED_HILO),
                                                ("n4096", 1_000, FUSED_SINGLE)])
def test_trajectory_fp32c_drift(oracle, name, nsteps, launch):
    """FP32C trajectories against the FP64 oracle: dumbbell-centre
    displacement relative drift <= 1e-4 at every record, and velocity error
    at the GPU's own final state <= 1e-6 (both sides on the same X)."""
    _torch()
    sus = make_preset(name)
    rec = nsteps // 10
    say(f"trajectory fp32c {name} {nsteps} steps launch={launch}")
    s = P.Simulator(sus.params, [sus.S], precision="fp32c", launch=launch, graph=True)
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(nsteps, rec)
    assert code == 0
    Xg = s.get_state()[0].cpu().numpy()
    Xo, co, mo, _ = _oracle_run_cached(oracle, name, nsteps, rec)
    R0 = 0.5 * (sus.X[0::2] + sus.X[1::2])
    dg, do = cen.cpu().numpy() - R0, co - R0
    drift = [relerr(dg[r], do[r]) for r in range(len(do))]
    say(f"  launch {s.launch} drift per record {['%.2e' % x for x in drift]}")
    assert max(drift) <= 1e-4
    t = nsteps * sus.params.dt
    F = oracle.forces(sus.params, Xg, sus.phi, t)
    check_fp32c(s.mobility(Xg, F).cpu().numpy(), oracle.mobility(sus.params, Xg, F), "final-state velocity")


def test_graph_equals_direct_launches(oracle):
    _torch()
    sus = make_single(300, 100.0, 9)
    out = []
    for graph in (False, True):
        s = P.Simulator(sus.params, [sus.S], precision="fp32c", graph=graph,
                        launch=dict(wg=256, wj=4, ipl=1, jchunk=256))
        s.set_state(sus.X, sus.phi)
        for _ in range(3):  # several replays with eager work between them
            s.step(40)
            s.check()
        out.append(s.get_state()[0].cpu().numpy())
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("launch", [dict(wg=256, wj=4, ipl=1, jchunk=256), FUSED_SINGLE,
                                    {"ipl": 1, "jchunk": 128, "wg": 64, "wj": 1, "posmode": 2, "fused": 2}])
def test_graph_runs_equal_direct_launches_with_records(launch):
    """Runs of steps replay a 16-step graph, single steps the one-step graph,
    and neither crosses a record point: for step counts and record intervals
    that are not multiples of 16, records and final state equal those of
    direct launches bit for bit."""
    _torch()
    sizes = [3, 120, 64, 17] if launch.get("fused") == 2 else [150]
    ens = make_ensemble(nsys=len(sizes), sizes=np.array(sizes, dtype=np.int32))
    out = []
    for graph in (False, True):
        s = P.Simulator(ens.params, sizes, precision="fp32c", graph=graph, launch=launch)
        s.set_state(ens.X, ens.phi)
        recs = []
        for nsteps, every in ((100, 7), (37, 0), (64, 16), (90, 23), (5, 5)):
            cen, com, code = s.run(nsteps, every)
            assert code == 0
            if every:
                recs.append((cen.cpu().numpy(), com.cpu().numpy()))
        X, t0, step = s.get_state()
        assert step == 296
        out.append((recs, X.cpu().numpy()))
    (r0, x0), (r1, x1) = out
    assert np.array_equal(x0, x1)
    for (c0, m0), (c1, m1) in zip(r0, r1):
        assert np.array_equal(c0, c1) and np.array_equal(m0, m1)
    assert [len(c) for c, _ in r0] == [14, 4, 3, 1]


@pytest.mark.parametrize("launch", [dict(wg=256, wj=4, ipl=1, jchunk=256), dict(wg=256, wj=1, ipl=2, jchunk=512),
                                    dict(wg=64, wj=1, ipl=4, jchunk=128, posmode=2),
                                    dict(wg=256, wj=4, ipl=4, jchunk=1000, posmode=2)])
@pytest.mark.parametrize("integrator", ["rk4", "heun"])
def test_step_launch_shapes(oracle, launch, integrator):
    """Stepping in several launch shapes, a single system and a batch: 60
    steps within 1e-9 of the oracle's positions."""
    _torch()
    for sizes in ([700], [3, 120, 64, 17, 250]):
        ens = make_ensemble(nsys=len(sizes), sizes=np.array(sizes, dtype=np.int32))
        s = P.Simulator(ens.params, sizes, precision="fp32c", integrator=integrator, graph=True, launch=launch)
        s.set_state(ens.X, ens.phi)
        cen, com, code = s.run(60, 20)
        assert code == 0
        Xo, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 60, S_per_sys=sizes,
                                 integrator=1 if integrator == "heun" else 0)
        assert np.abs(s.get_state()[0].cpu().numpy() - Xo).max() < 1e-9, (sizes, launch)


def test_deterministic_and_resumable(oracle):
    _torch()
    sus = make_single(200, 80.0, 10)
    res = []
    for _ in range(2):
        s = P.Simulator(sus.params, [sus.S], precision="fp32c")
        s.set_state(sus.X, sus.phi)
        s.step(300)
        res.append(s.get_state()[0].cpu().numpy())
    assert np.array_equal(res[0], res[1])
    s = P.Simulator(sus.params, [sus.S], precision="fp32c")
    s.set_state(sus.X, sus.phi)
    s.step(150)
    Xh, t0, step = s.get_state()
    assert step == 150
    s2 = P.Simulator(sus.params, [sus.S], precision="fp32c")
    s2.set_state(Xh, sus.phi, t0, step)
    s2.step(150)
    assert np.array_equal(s2.get_state()[0].cpu().numpy(), res[0])


# ---------------------------------------------------------------- ensembles

@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_ensemble_matches_oracle(oracle, precision):
    """A batch of uneven suspensions (sizes 1..120 dumbbells) in one launch
    per stage: FP64 bitwise per system, FP32C within the bars."""
    _torch()
    sizes = np.array([1, 16, 120, 3, 57, 64, 33, 90], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    say(f"ensemble {precision}")
    s = P.Simulator(ens.params, sizes, precision=precision, graph=True)
    s.set_state(ens.X, ens.phi)
    nsteps, rec = 400, 100
    cen, com, code = s.run(nsteps, rec)
    assert code == 0
    Xg = s.get_state()[0].cpu().numpy()
    Xo, co, mo, _ = oracle.run(ens.params, ens.X, ens.phi, nsteps, record_every=rec, S_per_sys=sizes)
    if precision == "fp64":
        assert np.array_equal(Xg, Xo)
        assert np.array_equal(com.cpu().numpy(), mo)
    else:
        off = ens.sphere_offsets
        F = np.concatenate([oracle.forces(ens.params, Xg[off[b]:off[b + 1]], ens.phi[off[b] // 2:off[b + 1] // 2], 4.0)
                            for b in range(len(sizes))])
        u = s.mobility(Xg, F).cpu().numpy()
        for b in range(len(sizes)):
            sl = slice(off[b], off[b + 1])
            uo = oracle.mobility(ens.params, Xg[sl], F[sl])
            check_fp32c(u[sl], uo, f"system {b}")
        assert np.abs(Xg - Xo).max() < 1e-6


def test_ensemble_full_size_sampled(oracle):
    """The 512-suspension batch (16..400 dumbbells each) in the default
    launch: mobility of 8 systems against the oracle; 20 steps run clean."""
    _torch()
    ens = make_preset("ens512")
    say(f"ensemble 512 systems, {ens.X.shape[0]} spheres")
    s = P.Simulator(ens.params, ens.S_per_sys, precision="fp32c", graph=True)
    s.set_state(ens.X, ens.phi)
    off = ens.sphere_offsets
    F = np.random.default_rng(2).standard_normal(ens.X.shape)
    u = s.mobility(ens.X, F).cpu().numpy()
    for b in np.random.default_rng(3).choice(ens.nsys, 8, replace=False):
        sl = slice(off[b], off[b + 1])
        check_fp32c(u[sl], oracle.mobility(ens.params, ens.X[sl], F[sl]), f"system {b}")
    cen, com, code = s.run(20, 10)
    assert code == 0 and np.isfinite(com.cpu().numpy()).all()


@pytest.mark.parametrize("fused", [1, 2, 3])
def test_fused_forms_many_systems(oracle, fused):
    """80 uneven systems (the work list then spreads the systems over the
    XCDs, each system's work-groups on one) in each fused form: 30 steps
    within 1e-6 of the oracle per system, relative to the displacement."""
    _torch()
    sizes = np.random.default_rng(17).integers(1, 61, 80).astype(np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    launch = {"ipl": 1, "jchunk": 128, "wg": 64, "wj": 1, "posmode": 2, "fused": fused}
    say(f"80 systems, fused {fused}")
    s = P.Simulator(ens.params, sizes, precision="fp32c", launch=launch, graph=True)
    s.set_state(ens.X, ens.phi)
    _, _, code = s.run(30, 0)
    assert code == 0
    Xg = s.get_state()[0].cpu().numpy()
    Xo, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 30, S_per_sys=sizes)
    off = ens.sphere_offsets
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        check_fp32c(Xg[sl] - ens.X[sl], Xo[sl] - ens.X[sl], f"system {b} displacement")


# ---------------------------------------------------------------- failures

def test_coincident_spheres_raise_flag(oracle):
    _torch()
    sus = make_single(8, 30.0, 3)
    X = sus.X.copy()
    X[5] = X[2]  # two spheres of different dumbbells on top of each other
    for precision in ("fp64", "fp32c"):
        s = P.Simulator(sus.params, [sus.S], precision=precision)
        s.set_state(X, sus.phi)
        _, _, code = s.run(2, 1)
        assert code == P.binding.AD_ENONFINITE, precision


def test_nan_state_raises_flag():
    _torch()
    sus = make_single(8, 30.0, 3)
    X = sus.X.copy()
    X[3, 1] = np.nan
    s = P.Simulator(sus.params, [sus.S], precision="fp32c")
    s.set_state(X, sus.phi)
    _, _, code = s.run(1, 1)
    assert code == P.binding.AD_ENONFINITE
    # a clean state clears it
    s.set_state(sus.X, sus.phi)
    _, _, code = s.run(1, 1)
    assert code == 0


def _steric_suspension():
    """Dense draw with exclusion at 1.5 instead of 2a: steric repulsion is
    active from the start while the Oseen tensor stays regular."""
    p = Params(steric_k=100.0, steric_r=2.0)
    return make_single(30, 16.0, 4, p, rmin=1.5)


def test_steric_trajectory_fp64(oracle):
    """Steric repulsion on (not in the paper): FP64 bitwise against the
    oracle over 200 steps."""
    _torch()
    sus = _steric_suspension()
    F = oracle.forces(sus.params, sus.X, sus.phi, 0.0)
    assert np.abs(F).max() > 1.0  # overlaps present
    Xg, cg, mg, Xo, co, mo = _run_both(oracle, sus, "fp64", 200, 50)
    assert np.array_equal(Xg, Xo)


def test_steric_fp32c(oracle):
    """FP32C with steric forces: velocity error <= 1e-6 at the overlapping
    start, and 200 steps within 1e-6 of the FP64 oracle's positions."""
    _torch()
    sus = _steric_suspension()
    s = P.Simulator(sus.params, [sus.S], precision="fp32c")
    s.set_state(sus.X, sus.phi)
    F = s.forces(sus.X, 0.0).cpu().numpy()
    assert np.array_equal(F, oracle.forces(sus.params, sus.X, sus.phi, 0.0))
    u = s.mobility(sus.X, F).cpu().numpy()
    check_fp32c(u, oracle.mobility(sus.params, sus.X, F), "velocity at the overlapping start")
    Xg, cg, mg, Xo, co, mo = _run_both(oracle, sus, "fp32c", 200, 50)
    err = np.abs(Xg - Xo).max()
    say(f"  steric fp32c max position error after 200 steps {err:.2e}")
    assert err < 1e-6


def test_steric_candidate_overflow_is_reported():
    """More than 16 spheres within 1.5 steric_r of one sphere: the FP32C
    candidate list would be incomplete, and ad_run says so (AD_ERANGE)."""
    _torch()
    p = Params(steric_k=100.0, steric_r=2.0)
    sus = make_single(40, 7.0, 8, p, rmin=1.0)  # up to 23 spheres within 3 of one
    s = P.Simulator(p, [sus.S], precision="fp32c")
    s.set_state(sus.X, sus.phi)
    _, _, code = s.run(1, 1)
    assert code == P.binding.AD_ERANGE


def test_large_steric_workload_runs_clean(oracle):
    """65536 spheres with steric repulsion, FP32C: a few steps with no flag,
    forces bitwise equal to the oracle's at the start."""
    torch = _torch()
    sus = make_preset("n65536")
    say("n65536 steric 4 steps")
    s = P.Simulator(sus.params, [sus.S], precision="fp32c", launch="tuned", graph=True)
    s.set_state(sus.X, sus.phi)
    rows = np.random.default_rng(11).choice(sus.N, 256, replace=False)
    F = s.forces(sus.X, 0.0).cpu().numpy()
    Fo = oracle.forces(sus.params, sus.X, sus.phi, 0.0)
    assert np.array_equal(F[rows], Fo[rows])
    _, _, code = s.run(4, 2)
    assert code == 0
    Xg = s.get_state()[0].cpu().numpy()
    assert np.isfinite(Xg).all() and np.abs(Xg - sus.X).max() < 0.1
    del s
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- RPY-Mazur tensor

@pytest.mark.parametrize("S,side", [(1, 8.0), (8, 40.0), (150, 90.0)])
def test_rpy_mobility_fp64_bitwise(oracle, S, side):
    """Eq. (e:Mazur) with its second line: FP64 bitwise against the oracle."""
    _torch()
    sus = make_single(S, side, 12)
    F = np.random.default_rng(13).standard_normal(sus.X.shape)
    s = P.Simulator(sus.params, [sus.S], precision="fp64", tensor="rpy")
    u = s.mobility(sus.X, F).cpu().numpy()
    assert np.array_equal(u, oracle.mobility(sus.params, sus.X, F, tensor=1))


def test_rpy_trajectory_fp64_bitwise(oracle):
    _torch()
    sus = make_preset("n16")
    s = P.Simulator(sus.params, [sus.S], precision="fp64", tensor="rpy", graph=True)
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(1000, 250)
    assert code == 0
    Xo, co, mo, _ = oracle.run(sus.params, sus.X, sus.phi, 1000, record_every=250, tensor=1)
    assert np.array_equal(s.get_state()[0].cpu().numpy(), Xo)
    assert np.array_equal(com.cpu().numpy(), mo)


# The plain FP64 pair sum runs 1, 2 or 4 targets per work-group (one system
# of 4100 spheres: 4; ensembles of 2048 to 4095 spheres: 2, of 4096 and more:
# 4, with odd dumbbell counts leaving part-filled blocks), in chunks of 128
# sources (4 targets, fewer than 8192 spheres) or 64, the last one part-filled.
@pytest.mark.parametrize("tensor", [0, 1])
@pytest.mark.parametrize("sizes", [[2050], [1, 3, 1025, 999, 33], [7, 1000, 61], [4100, 7]])
def test_fp64_pair_sum_block_shapes_bitwise(oracle, sizes, tensor):
    _torch()
    say(f"fp64 pair sum sizes={sizes} tensor={tensor}")
    sizes = np.array(sizes, dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    F = np.random.default_rng(21).standard_normal(ens.X.shape)
    s = P.Simulator(ens.params, sizes, precision="fp64", tensor="rpy" if tensor else "oseen")
    u = s.mobility(ens.X, F).cpu().numpy()
    off = ens.sphere_offsets
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        assert np.array_equal(u[sl], oracle.mobility(ens.params, ens.X[sl], F[sl], tensor=tensor)), f"system {b}"


# The producer takes short forms of 1/sqrt(r2) only when every r2 of its chunk
# lies in [2^-400, 2^400]; a chunk with any pair outside takes the library's.
# Both must give the oracle's bits: systems scaled far below and above that
# range, and a near-coincident pair (1e-61 apart) in an otherwise plain one.
@pytest.mark.parametrize("tensor", [0, 1])
@pytest.mark.parametrize("case", ["tiny", "huge", "near_pair"])
def test_fp64_pair_sum_outside_short_form_range_bitwise(oracle, case, tensor):
    _torch()
    say(f"fp64 pair sum outside the short-form range: {case} tensor={tensor}")
    S = 2050 if case == "near_pair" else 300
    sus = make_single(S, 240.0 if case == "near_pair" else 90.0, 31)
    X = sus.X.copy()
    F = np.random.default_rng(32).standard_normal(X.shape)
    if case == "tiny":
        X *= 1e-62
    elif case == "huge":
        X *= 1e62
    else:
        # near the origin, where 1e-61 is representable beside the coordinates
        X[3001] = np.array([1e-59, 2e-59, -1e-59])
        X[1000] = X[3001] + np.array([1e-61, -2e-61, 0.5e-61])
    s = P.Simulator(sus.params, [S], precision="fp64", tensor="rpy" if tensor else "oseen")
    u = s.mobility(X, F).cpu().numpy()
    uo = oracle.mobility(sus.params, X, F, tensor=tensor)
    assert np.isfinite(uo).all()
    assert np.array_equal(u, uo)


def test_fp64_bitwise_full_n4096_tuned(oracle):
    """The 4096-sphere workload in the bench's bitwise-FP64 configuration
    (launch "tuned"): 2 RK4 steps bitwise, and the records."""
    _torch()
    sus = make_preset("n4096")
    say("fp64 bitwise n4096 tuned, 2 steps")
    s = P.Simulator(sus.params, [sus.S], precision="fp64", launch="tuned", graph=True)
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(2, 1)
    assert code == 0
    Xo, co, mo, _ = oracle.run(sus.params, sus.X, sus.phi, 2, record_every=1)
    assert np.array_equal(s.get_state()[0].cpu().numpy(), Xo)
    assert np.array_equal(com.cpu().numpy(), mo)


def test_fp64_pair_sum_four_target_blocks_trajectory(oracle):
    """Stepping through the 4-target blocks (part-filled ones included):
    3 RK4 steps bitwise, and the records."""
    _torch()
    sizes = np.array([1, 3, 1025, 999, 33], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    say("fp64 pair sum, 4-target blocks, 3 steps")
    s = P.Simulator(ens.params, sizes, precision="fp64", graph=True)
    s.set_state(ens.X, ens.phi)
    cen, com, code = s.run(3, 1)
    assert code == 0
    Xo, co, mo, _ = oracle.run(ens.params, ens.X, ens.phi, 3, record_every=1, S_per_sys=sizes)
    assert np.array_equal(s.get_state()[0].cpu().numpy(), Xo)
    assert np.array_equal(com.cpu().numpy(), mo)


@pytest.mark.parametrize("precision,launch", [("fp64_tiled", None), ("fp32c", None),
                                              ("fp32c", dict(wg=256, wj=4, ipl=2, jchunk=512, posmode=2)),
                                              ("fp32c", dict(wg=64, wj=1, ipl=4, jchunk=128))])
def test_rpy_mobility_tolerances(oracle, precision, launch):
    _torch()
    sus = make_single(900, 160.0, 14)
    X = perturbed(sus, 0.2)
    F = oracle.forces(sus.params, X, sus.phi, 3.0)
    s = P.Simulator(sus.params, [sus.S], precision=precision, tensor="rpy", launch=launch)
    u, uo = s.mobility(X, F).cpu().numpy(), oracle.mobility(sus.params, X, F, tensor=1)
    if precision == "fp64_tiled":
        assert relerr(u, uo) <= 1e-13
    else:
        check_fp32c(u, uo, f"rpy {launch}")


def test_rpy_trajectory_fp32c(oracle):
    """FP32C with the RPY tensor: 2000 RK4 steps of 512 spheres, centre
    displacement drift <= 1e-4 against the oracle."""
    _torch()
    sus = make_preset("n512")
    s = P.Simulator(sus.params, [sus.S], precision="fp32c", tensor="rpy", graph=True,
                    launch=dict(wg=256, wj=4, ipl=1, jchunk=256))
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(2000, 500)
    assert code == 0
    Xo, co, mo, _ = oracle.run(sus.params, sus.X, sus.phi, 2000, record_every=500, tensor=1)
    R0 = 0.5 * (sus.X[0::2] + sus.X[1::2])
    drift = max(relerr(cen.cpu().numpy()[r] - R0, co[r] - R0) for r in range(len(co)))
    say(f"  rpy fp32c drift {drift:.2e}")
    assert drift <= 1e-4


# ---------------------------------------------------------------- stroke-averaged equations

def _sa_config(S, spread, seed):
    rng = np.random.default_rng(seed)
    R = rng.uniform(-spread, spread, (S, 3))
    N = rng.standard_normal((S, 3))
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    return R, N, rng.uniform(0, 2 * math.pi, S)


def _lattice(n, spacing, seed):
    """n^3 dumbbells on a cubic lattice (Sec. IV.C), random axes and phases."""
    g = (np.arange(n) - (n - 1) / 2) * spacing
    R = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(seed)
    N = rng.standard_normal(R.shape)
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    return R, N, rng.uniform(0, 2 * math.pi, len(R))


@pytest.mark.parametrize("S", [1, 2, 129, 700])
def test_sa_rhs_matches_oracle(oracle, S):
    """Eqs. (e:eom, J, K) on the GPU against the oracle (the phase sine comes
    from the device's sin, hence a tolerance instead of bit equality)."""
    torch = _torch()
    R, N, phi = _sa_config(S, 80.0, S)
    p = Params()
    sa = P.StrokeAveraged(p, R, N, phi)
    dR, dN = (x.cpu().numpy() for x in sa.rhs())
    oR, oN = oracle.sa_rhs(p, R, N, phi)
    if S == 1:
        assert np.abs(dR).max() == 0 and np.abs(dN).max() == 0
        return
    assert relerr(dR, oR) <= 1e-13 and relerr(dN, oN) <= 1e-13


def test_sa_run_lattice_matches_oracle(oracle):
    """5^3 dumbbells at spacing 10 ell (the lattice of Sec. IV.C), 400 RK4
    steps of dt = T/10 of the stroke-averaged equations."""
    _torch()
    R, N, phi = _lattice(5, 40.0, 3)
    p = Params()
    sa = P.StrokeAveraged(p, R, N, phi)
    assert sa.run(10.0, 400) == 0
    Ro, No = oracle.sa_run(p, R, N, phi, 10.0, 400)
    Rg, Ng = sa.R.cpu().numpy(), sa.N.cpu().numpy()
    assert relerr(Rg - R, Ro - R) <= 1e-10
    assert np.abs(Ng - No).max() <= 1e-12
    np.testing.assert_allclose(np.linalg.norm(Ng, axis=1), 1.0, atol=1e-15)


def test_sa_coincident_centres_flagged():
    _torch()
    R, N, phi = _sa_config(5, 30.0, 4)
    R[3] = R[1]
    sa = P.StrokeAveraged(Params(), R, N, phi)
    assert sa.run(1.0, 2) == P.binding.AD_ENONFINITE


# ---------------------------------------------------------------- Brownian noise (Heun)

@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32c", 1e-7)])
def test_heun_noise_matches_oracle(oracle, precision, tol):
    """Additive noise with constant C (Sec. V), Philox4x32-10 + Box-Muller on
    both sides: the same random numbers, so the GPU follows the oracle's
    Brownian trajectory (normals agree to the last bits of log/sin/cos)."""
    _torch()
    sizes = np.array([8, 3, 20], dtype=np.int32)
    ens = make_ensemble(nsys=3, sizes=sizes)
    kT, seed = 0.01, 77
    s = P.Simulator(ens.params, sizes, precision=precision, integrator="heun", kT=kT, seed=seed, graph=True)
    s.set_state(ens.X, ens.phi)
    cen, com, code = s.run(300, 100)
    assert code == 0
    Xg = s.get_state()[0].cpu().numpy()
    Xo, co, mo, _ = oracle.run(ens.params, ens.X, ens.phi, 300, record_every=100, S_per_sys=sizes,
                               integrator=1, kT=kT, seed=seed)
    Xd, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 300, S_per_sys=sizes, integrator=1)
    assert np.abs(Xo - Xd).max() > 1e-3  # the noise matters
    err = np.abs(Xg - Xo).max()
    say(f"  noise {precision} max position error {err:.2e}")
    assert err <= tol


# ---------------------------------------------------------------- fused stage kernel

@pytest.mark.parametrize("launch", [FUSED_SINGLE, FUSED_HILO])
@pytest.mark.parametrize("integrator,tensor", [("rk4", "oseen"), ("heun", "oseen"), ("rk4", "rpy")])
def test_fused_stage_matches_oracle(oracle, launch, integrator, tensor):
    """Pair sum and stage update in one kernel per stage, on systems that are
    not a multiple of the 16-sphere target block or the 64-sphere source
    block: positions after 300 steps within 1e-6 of the oracle's, relative to
    the displacement, and within rounding of the two-kernel path."""
    _torch()
    for S, side in ((5, 20.0), (57, 60.0), (300, 120.0)):
        sus = make_single(S, side, 31)
        say(f"fused {launch['posmode']} {integrator} {tensor} S={S}")
        s = P.Simulator(sus.params, [S], precision="fp32c", integrator=integrator, tensor=tensor,
                        launch=launch, graph=True)
        s.set_state(sus.X, sus.phi)
        _, _, code = s.run(300, 0)
        assert code == 0
        Xf = s.get_state()[0].cpu().numpy()
        plain = dict(launch, fused=0)
        s2 = P.Simulator(sus.params, [S], precision="fp32c", integrator=integrator, tensor=tensor,
                         launch=plain, graph=True)
        s2.set_state(sus.X, sus.phi)
        s2.run(300, 0)
        Xu = s2.get_state()[0].cpu().numpy()
        Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 300, integrator=1 if integrator == "heun" else 0,
                                 tensor=1 if tensor == "rpy" else 0)
        check_fp32c(Xf - sus.X, Xo - sus.X, "displacement vs oracle")
        check_fp32c(Xf - sus.X, Xu - sus.X, "displacement vs two-kernel path")


@pytest.mark.parametrize("launch", [FUSED_SINGLE, FUSED_HILO])
def test_fused_stage_ensemble_matches_oracle(oracle, launch):
    """Fused stages over a batch of uneven systems (1..120 dumbbells), one
    work-group per 16-target block of a system: 400 steps within 1e-6 of the
    oracle per system, relative to the displacement."""
    _torch()
    sizes = np.array([1, 16, 120, 3, 57, 64, 33, 90], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    say(f"fused ensemble posmode {launch['posmode']}")
    s = P.Simulator(ens.params, sizes, precision="fp32c", launch=dict(launch, wg=64, wj=1, jchunk=128),
                    graph=True)
    assert s.launch["fused"] == 1
    s.set_state(ens.X, ens.phi)
    _, _, code = s.run(400, 0)
    assert code == 0
    Xg = s.get_state()[0].cpu().numpy()
    Xo, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 400, S_per_sys=sizes)
    off = ens.sphere_offsets
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        check_fp32c(Xg[sl] - ens.X[sl], Xo[sl] - ens.X[sl], f"system {b} displacement")


@pytest.mark.parametrize("S,posmode", [(3392, 2), (2272, 1)])
def test_fused_stage_at_the_lds_limit(oracle, S, posmode):
    """The largest systems the fused stage takes (6784 spheres with
    single-float positions, 4544 with hi/lo, every source in 160 KiB of LDS):
    two steps against the oracle, relative to the displacement."""
    _torch()
    sus = make_single(S, 280.0, 41)
    launch = dict(FUSED_SINGLE if posmode == 2 else FUSED_HILO)
    say(f"fused at the LDS limit: N = {2 * S}, posmode {posmode}")
    s = P.Simulator(sus.params, [S], precision="fp32c", launch=launch, graph=True)
    s.set_state(sus.X, sus.phi)
    _, _, code = s.run(2, 0)
    assert code == 0
    Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 2)
    check_fp32c(s.get_state()[0].cpu().numpy() - sus.X, Xo - sus.X, "displacement")


def test_fused_stage_deterministic_resumable_and_noise(oracle):
    """Fused stages: two runs give the same bits, split step calls equal one
    call, and the Heun noise follows the oracle's Brownian trajectory."""
    _torch()
    sus = make_preset("n512")
    out = []
    for calls in ((400,), (400,), (150, 250)):
        s = P.Simulator(sus.params, [sus.S], precision="fp32c", launch=FUSED_SINGLE, graph=True)
        s.set_state(sus.X, sus.phi)
        for n in calls:
            _, _, code = s.run(n, 0)
            assert code == 0
        out.append(s.get_state()[0].cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    sus = make_single(20, 40.0, 5)
    kT, seed = 0.01, 77
    s = P.Simulator(sus.params, [sus.S], precision="fp32c", integrator="heun", kT=kT, seed=seed,
                    launch=FUSED_HILO, graph=True)
    s.set_state(sus.X, sus.phi)
    _, _, code = s.run(300, 0)
    assert code == 0
    Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 300, integrator=1, kT=kT, seed=seed)
    assert np.abs(s.get_state()[0].cpu().numpy() - Xo).max() <= 1e-7


WIDE_SINGLE = {"ipl": 1, "jchunk": 128, "wg": 64, "wj": 1, "posmode": 2, "fused": 2}
WIDE_HILO = dict(WIDE_SINGLE, posmode=1)


@pytest.mark.parametrize("launch", [WIDE_SINGLE, WIDE_HILO])
@pytest.mark.parametrize("integrator,tensor", [("rk4", "oseen"), ("heun", "oseen"), ("rk4", "rpy")])
def test_wide_fused_stage_ensemble_matches_oracle(oracle, launch, integrator, tensor):
    """The wide fused stage (64 targets per work-group, one per lane) over
    uneven systems, from 1 dumbbell to blocks with a ragged last block, with a
    system not a multiple of 4 spheres long in its sources: 300 steps within
    1e-6 of the oracle per system, relative to the displacement, and within
    1e-6 of the two-kernel path."""
    _torch()
    sizes = np.array([1, 16, 120, 3, 57, 64, 33, 90, 200], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    say(f"wide fused ensemble posmode {launch['posmode']} {integrator} {tensor}")
    out = {}
    for name, L in (("wide", launch), ("two", dict(launch, fused=0))):
        s = P.Simulator(ens.params, sizes, precision="fp32c", integrator=integrator, tensor=tensor, launch=L,
                        graph=True)
        assert s.launch["fused"] == L["fused"]
        s.set_state(ens.X, ens.phi)
        _, _, code = s.run(300, 0)
        assert code == 0
        out[name] = s.get_state()[0].cpu().numpy()
    Xo, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 300, S_per_sys=sizes,
                             integrator=1 if integrator == "heun" else 0, tensor=1 if tensor == "rpy" else 0)
    off = ens.sphere_offsets
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        check_fp32c(out["wide"][sl] - ens.X[sl], Xo[sl] - ens.X[sl], f"system {b} vs oracle")
        check_fp32c(out["wide"][sl] - ens.X[sl], out["two"][sl] - ens.X[sl], f"system {b} vs two-kernel path")


@pytest.mark.parametrize("S,posmode", [(300, 2), (3412, 2), (2274, 1)])
def test_wide_fused_stage_single_system(oracle, S, posmode):
    """The wide form on one system, up to the largest it takes (6824 spheres
    single-float, 4548 hi/lo): two steps (ten for the small one) against the
    oracle, relative to the displacement."""
    _torch()
    sus = make_single(S, 280.0 if S > 1000 else 120.0, 43)
    n = 10 if S < 1000 else 2
    say(f"wide fused single system N = {2 * S}, posmode {posmode}")
    s = P.Simulator(sus.params, [S], precision="fp32c", launch=dict(WIDE_SINGLE, posmode=posmode), graph=True)
    s.set_state(sus.X, sus.phi)
    _, _, code = s.run(n, 0)
    assert code == 0
    Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, n)
    check_fp32c(s.get_state()[0].cpu().numpy() - sus.X, Xo - sus.X, "displacement")


def test_wide_fused_stage_deterministic_and_resumable():
    """Two runs give the same bits; split step calls equal one call."""
    _torch()
    ens = make_ensemble(nsys=12, sizes=np.array([16, 400, 3, 27, 64, 5, 120, 33, 250, 8, 77, 190], dtype=np.int32))
    out = []
    for calls in ((200,), (200,), (70, 130)):
        s = P.Simulator(ens.params, ens.S_per_sys, precision="fp32c", launch=WIDE_SINGLE, graph=True)
        s.set_state(ens.X, ens.phi)
        for n in calls:
            _, _, code = s.run(n, 0)
            assert code == 0
        out.append(s.get_state()[0].cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


STREAM_SINGLE = {"ipl": 1, "jchunk": 256, "wg": 256, "wj": 4, "posmode": 2, "fused": 3}
STREAM_HILO = dict(STREAM_SINGLE, posmode=1)


@pytest.mark.parametrize("launch", [STREAM_SINGLE, STREAM_HILO])
@pytest.mark.parametrize("integrator,tensor", [("rk4", "oseen"), ("heun", "oseen"), ("rk4", "rpy")])
def test_streamed_fused_stage_matches_oracle(oracle, launch, integrator, tensor):
    """The streamed fused stage on single systems from 1 dumbbell to a size
    that is neither a multiple of the 1024-source padding nor of the 16-target
    block (its own spheres then fall in different splits and chunks), 200
    steps: within 1e-6 of the oracle, relative to the displacement, and
    within 1e-6 of the two-kernel path."""
    _torch()
    for S, side in ((1, 10.0), (5, 20.0), (300, 120.0), (1100, 180.0)):
        sus = make_single(S, side, 51)
        say(f"streamed {launch['posmode']} {integrator} {tensor} S={S}")
        out = {}
        for name, L in (("stream", launch), ("two", dict(launch, fused=0))):
            s = P.Simulator(sus.params, [S], precision="fp32c", integrator=integrator, tensor=tensor, launch=L,
                            graph=True)
            s.set_state(sus.X, sus.phi)
            _, _, code = s.run(200, 0)
            assert code == 0
            out[name] = s.get_state()[0].cpu().numpy()
        Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 200, integrator=1 if integrator == "heun" else 0,
                                 tensor=1 if tensor == "rpy" else 0)
        check_fp32c(out["stream"] - sus.X, Xo - sus.X, "displacement vs oracle")
        check_fp32c(out["stream"] - sus.X, out["two"] - sus.X, "displacement vs two-kernel path")


@pytest.mark.parametrize("S,posmode", [(1500, 2), (1500, 1), (2048, 2), (4100, 2), (4100, 1)])
def test_streamed_fused_stage_large_systems(oracle, S, posmode):
    """Systems at and beyond the size where every source fits one
    work-group's LDS (8200 spheres), and of 3000 spheres (8-target, 8-wave
    work-groups, more than one per compute unit): two steps against the
    oracle."""
    _torch()
    sus = make_single(S, 240.0 * (2 * S / 4096.0) ** (1.0 / 3.0), 53)
    say(f"streamed N = {2 * S}, posmode {posmode}")
    s = P.Simulator(sus.params, [S], precision="fp32c", launch=dict(STREAM_SINGLE, posmode=posmode), graph=True)
    s.set_state(sus.X, sus.phi)
    _, _, code = s.run(2, 0)
    assert code == 0
    Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 2)
    check_fp32c(s.get_state()[0].cpu().numpy() - sus.X, Xo - sus.X, "displacement")


STREAM64 = {"ipl": 1, "jchunk": 256, "wg": 64, "wj": 1, "posmode": 0, "fused": 3}


@pytest.mark.parametrize("integrator,tensor", [("rk4", "oseen"), ("heun", "oseen"), ("rk4", "rpy")])
def test_fp64_streamed_stage_matches_oracle(oracle, integrator, tensor):
    """The FP64 streamed stage (AD_FP64_TILED, fused = 3: rsqrt with one
    Newton step and FMAs, tiled sums) on single systems from 1 dumbbell to
    a size that is neither a multiple of the 1024-source padding nor of any
    target block (4, 8 and 16 targets per work-group all occur), 200 steps:
    within 1e-11 of the oracle relative to the displacement, per system and
    per sphere."""
    _torch()
    for S, side in ((1, 10.0), (5, 20.0), (300, 120.0), (1100, 180.0), (2100, 240.0)):
        sus = make_single(S, side, 61)
        say(f"fp64 streamed {integrator} {tensor} S={S}")
        s = P.Simulator(sus.params, [S], precision="fp64_tiled", integrator=integrator, tensor=tensor,
                        launch=STREAM64, graph=True)
        s.set_state(sus.X, sus.phi)
        _, _, code = s.run(200, 0)
        assert code == 0
        X = s.get_state()[0].cpu().numpy()
        Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 200, integrator=1 if integrator == "heun" else 0,
                                 tensor=1 if tensor == "rpy" else 0)
        d, do = X - sus.X, Xo - sus.X
        assert relerr(d, do) <= 1e-11, (S, relerr(d, do))
        scale = np.linalg.norm(do, axis=1) + np.median(np.linalg.norm(do, axis=1))
        assert (np.linalg.norm(d - do, axis=1) / scale).max() <= 1e-10, S


def test_fp64_streamed_stage_ensemble_determinism_and_flag(oracle):
    """FP64 streamed stage on an uneven ensemble: 100 steps per system within
    1e-11 of the oracle; two runs give the same bits and split calls equal
    one call; coincident spheres raise the flag."""
    _torch()
    sizes = np.array([1, 16, 120, 3, 57, 64, 33, 90, 200], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    out = []
    for calls in ((100,), (100,), (30, 70)):
        s = P.Simulator(ens.params, sizes, precision="fp64_tiled", launch=STREAM64, graph=True)
        s.set_state(ens.X, ens.phi)
        for n in calls:
            _, _, code = s.run(n, 0)
            assert code == 0
        out.append(s.get_state()[0].cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    Xo, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 100, S_per_sys=sizes)
    off = ens.sphere_offsets
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        assert relerr(out[0][sl] - ens.X[sl], Xo[sl] - ens.X[sl]) <= 1e-11, b
    sus = make_single(8, 30.0, 3)
    X = sus.X.copy()
    X[5] = X[2]
    s = P.Simulator(sus.params, [sus.S], precision="fp64_tiled", launch=STREAM64)
    s.set_state(X, sus.phi)
    _, _, code = s.run(2, 1)
    assert code == P.binding.AD_ENONFINITE


def test_streamed_fused_stage_ensemble_and_determinism(oracle):
    """An ensemble of uneven systems (16-target work list), 200 steps against
    the oracle; two runs give the same bits and split calls equal one call."""
    _torch()
    sizes = np.array([1, 16, 120, 3, 57, 64, 33, 90, 200], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    out = []
    for calls in ((200,), (200,), (70, 130)):
        s = P.Simulator(ens.params, sizes, precision="fp32c", launch=STREAM_SINGLE, graph=True)
        s.set_state(ens.X, ens.phi)
        for n in calls:
            _, _, code = s.run(n, 0)
            assert code == 0
        out.append(s.get_state()[0].cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    Xo, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 200, S_per_sys=sizes)
    off = ens.sphere_offsets
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        check_fp32c(out[0][sl] - ens.X[sl], Xo[sl] - ens.X[sl], f"system {b} displacement")


def test_launch_changes_between_runs_repack(oracle):
    """With single-float positions the fused stages leave the lo parts of the
    next pack unwritten. A change of launch shape between runs re-packs from
    the FP64 state, so no form ever reads stale lo parts: 40 steps in each of
    six forms in turn (single-float and hi/lo, streamed, staged and two
    kernels) stay within 1e-6 of the oracle's 240 steps."""
    _torch()
    sus = make_single(300, 120.0, 61)
    s = P.Simulator(sus.params, [sus.S], precision="fp32c", launch=dict(STREAM_HILO, fused=0), graph=True)
    s.set_state(sus.X, sus.phi)
    ctx = s.ctx
    for L in (dict(STREAM_HILO, fused=0), STREAM_SINGLE, STREAM_HILO, FUSED_SINGLE, FUSED_HILO,
              dict(STREAM_SINGLE, fused=0)):
        s.set_launch(**L)
        assert s.ctx == ctx  # the workspace sufficed: the state was kept
        _, _, code = s.run(40, 0)
        assert code == 0
    X, _, step = s.get_state()
    assert step == 240
    Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 240)
    check_fp32c(X.cpu().numpy() - sus.X, Xo - sus.X, "six forms in turn: displacement")


def test_streamed_fused_stage_noise(oracle):
    """Heun with additive noise through the streamed stage: the GPU follows
    the oracle's Brownian trajectory (same Philox numbers)."""
    _torch()
    sus = make_single(600, 120.0, 57)
    kT, seed = 0.01, 91
    s = P.Simulator(sus.params, [sus.S], precision="fp32c", integrator="heun", kT=kT, seed=seed,
                    launch=STREAM_HILO, graph=True)
    s.set_state(sus.X, sus.phi)
    _, _, code = s.run(100, 0)
    assert code == 0
    Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 100, integrator=1, kT=kT, seed=seed)
    Xd, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 100, integrator=1)
    assert np.abs(Xo - Xd).max() > 1e-3  # the noise matters
    assert np.abs(s.get_state()[0].cpu().numpy() - Xo).max() <= 1e-7


def test_heun_noise_deterministic_and_resumable():
    _torch()
    sus = make_single(50, 40.0, 5)
    kw = dict(precision="fp32c", integrator="heun", kT=0.02, seed=5, graph=True)
    s = P.Simulator(sus.params, [sus.S], **kw)
    s.set_state(sus.X, sus.phi)
    s.step(120)
    a = s.get_state()[0].cpu().numpy()
    s2 = P.Simulator(sus.params, [sus.S], **kw)
    s2.set_state(sus.X, sus.phi)
    s2.step(60)
    Xh, t0, st = s2.get_state()
    s3 = P.Simulator(sus.params, [sus.S], **kw)
    s3.set_state(Xh, sus.phi, t0, st)
    s3.step(60)
    assert np.array_equal(s3.get_state()[0].cpu().numpy(), a)


@pytest.mark.parametrize("precision,steric", [("fp32c", False), ("fp32c", True), ("fp64", True)])
def test_split_step_calls_equal_one_call(oracle, precision, steric):
    """A step call leaves the next step's pack in place; later calls reuse it.
    Four calls of 50 steps, with a mobility apply and a record run in between
    (which must not disturb the state), equal one call of 200 steps bit for
    bit."""
    _torch()
    p = Params(steric_k=100.0, steric_r=2.0) if steric else Params()
    sus = make_single(60, 22.0, 6, p, rmin=1.6 if steric else None)
    one = P.Simulator(p, [sus.S], precision=precision, graph=True)
    one.set_state(sus.X, sus.phi)
    one.step(200)
    parts = P.Simulator(p, [sus.S], precision=precision, graph=True)
    parts.set_state(sus.X, sus.phi)
    parts.step(50)
    parts.mobility(sus.X, np.ones_like(sus.X))
    parts.step(50)
    _, _, code = parts.run(50, 25)
    assert code == 0
    parts.step(50)
    assert np.array_equal(one.get_state()[0].cpu().numpy(), parts.get_state()[0].cpu().numpy())


# ---------------------------------------------------------------- resident form (small systems)

RESIDENT = {"ipl": 1, "jchunk": 256, "wg": 64, "wj": 1, "posmode": 1, "fused": 4}
RESIDENT_SINGLE = dict(RESIDENT, posmode=2)


@pytest.mark.parametrize("integrator,tensor", [("rk4", "oseen"), ("heun", "oseen"), ("rk4", "rpy")])
def test_resident_fp64_bitwise(oracle, integrator, tensor):
    """The resident form in plain FP64: the 16-sphere workload over 2000
    steps (records every 250), and a batch of uneven small systems over 300
    steps (one of 128 spheres, whose terms take several column chunks),
    bitwise equal to the oracle: state, centres and centre of mass."""
    _torch()
    it, te = (1 if integrator == "heun" else 0), (1 if tensor == "rpy" else 0)
    sus = make_preset("n16")
    s = P.Simulator(sus.params, [sus.S], precision="fp64", integrator=integrator, tensor=tensor,
                    launch=RESIDENT, graph=True)
    assert s.launch["fused"] == 4
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(2000, 250)
    assert code == 0
    Xo, co, mo, _ = oracle.run(sus.params, sus.X, sus.phi, 2000, record_every=250, integrator=it, tensor=te)
    assert np.array_equal(s.get_state()[0].cpu().numpy(), Xo)
    assert np.array_equal(cen.cpu().numpy(), co) and np.array_equal(com.cpu().numpy(), mo)
    sizes = np.array([1, 8, 27, 64, 3, 40], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    s = P.Simulator(ens.params, sizes, precision="fp64", integrator=integrator, tensor=tensor, launch=RESIDENT)
    s.set_state(ens.X, ens.phi)
    cen, com, code = s.run(300, 100)
    assert code == 0
    Xo, co, mo, _ = oracle.run(ens.params, ens.X, ens.phi, 300, record_every=100, S_per_sys=sizes, integrator=it,
                               tensor=te)
    assert np.array_equal(s.get_state()[0].cpu().numpy(), Xo)
    assert np.array_equal(cen.cpu().numpy(), co) and np.array_equal(com.cpu().numpy(), mo)


def test_resident_fp64_full_n16(oracle):
    """The plain FP64 workload in full in the resident form, which is what
    launch="tuned" picks for it: 16 spheres, 1e4 RK4 steps, records every
    1000, bitwise."""
    _torch()
    sus = make_preset("n16")
    s = P.Simulator(sus.params, [sus.S], precision="fp64", launch="tuned")
    assert s.launch["fused"] == 4
    s.set_state(sus.X, sus.phi)
    cen, com, code = s.run(10_000, 1000)
    assert code == 0
    Xo, co, mo, _ = oracle.run(sus.params, sus.X, sus.phi, 10_000, record_every=1000)
    assert np.array_equal(s.get_state()[0].cpu().numpy(), Xo)
    assert np.array_equal(cen.cpu().numpy(), co) and np.array_equal(com.cpu().numpy(), mo)


@pytest.mark.parametrize("launch", [RESIDENT, RESIDENT_SINGLE])
@pytest.mark.parametrize("integrator,tensor", [("rk4", "oseen"), ("heun", "oseen"), ("rk4", "rpy")])
def test_resident_fp32c_matches_oracle(oracle, launch, integrator, tensor):
    """The resident form in FP32C on uneven systems from 1 dumbbell to 128
    (256 spheres: 512 threads, two lanes per target; a 2-sphere system
    there has 32 lanes per target) and the paper's 27-dumbbell lattice size:
    300 steps against the oracle per system, relative to the displacement,
    and within the bars of the two-kernel path."""
    _torch()
    sizes = np.array([1, 27, 128, 3, 57, 8, 100], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    it, te = (1 if integrator == "heun" else 0), (1 if tensor == "rpy" else 0)
    out = {}
    for name, L in (("res", launch), ("two", dict(launch, fused=0))):
        s = P.Simulator(ens.params, sizes, precision="fp32c", integrator=integrator, tensor=tensor, launch=L,
                        graph=True)
        s.set_state(ens.X, ens.phi)
        _, _, code = s.run(300, 0)
        assert code == 0
        out[name] = s.get_state()[0].cpu().numpy()
    Xo, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 300, S_per_sys=sizes, integrator=it, tensor=te)
    off = ens.sphere_offsets
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        check_fp32c(out["res"][sl] - ens.X[sl], Xo[sl] - ens.X[sl], f"system {b} (S={sizes[b]}) vs oracle")
        check_fp32c(out["res"][sl] - ens.X[sl], out["two"][sl] - ens.X[sl], f"system {b} vs two-kernel path")


@pytest.mark.parametrize("sizes", [[8], [16], [8, 1, 5, 2], [12, 16, 3]])
def test_resident_fp32c_thread_counts_match_oracle(oracle, sizes):
    """The FP32C resident form at each of its thread counts: one wave up to
    16 spheres (4 lanes per sphere at 16 spheres, 32 at 2), 256 threads for
    17 to 32 spheres (8 lanes per sphere), 512 above; the uneven ensembles
    put systems of different sizes, and so different lane counts, in one
    launch. 300 RK4 steps against the oracle per system, norm and per-sphere
    bars."""
    _torch()
    sizes = np.array(sizes, dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    s = P.Simulator(ens.params, sizes, precision="fp32c", launch=RESIDENT_SINGLE, graph=True)
    s.set_state(ens.X, ens.phi)
    _, _, code = s.run(300, 0)
    assert code == 0
    X = s.get_state()[0].cpu().numpy()
    Xo, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 300, S_per_sys=sizes)
    off = ens.sphere_offsets
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        check_fp32c(X[sl] - ens.X[sl], Xo[sl] - ens.X[sl], f"system {b} (S={sizes[b]})")


def test_resident_noise_determinism_and_split_calls(oracle):
    """Resident form: Heun with Brownian noise follows the oracle's
    trajectory (same Philox numbers); two runs give the same bits; split
    calls and record points (which split the launches) equal one call;
    switching to a staged form and back keeps the state."""
    _torch()
    sus = make_single(20, 40.0, 5)
    kT, seed = 0.01, 77
    s = P.Simulator(sus.params, [sus.S], precision="fp32c", integrator="heun", kT=kT, seed=seed, launch=RESIDENT)
    s.set_state(sus.X, sus.phi)
    _, _, code = s.run(300, 0)
    assert code == 0
    Xo, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 300, integrator=1, kT=kT, seed=seed)
    assert np.abs(s.get_state()[0].cpu().numpy() - Xo).max() <= 1e-7
    sizes = np.array([16, 27, 3, 60], dtype=np.int32)
    ens = make_ensemble(nsys=len(sizes), sizes=sizes)
    out = []
    for calls in ((200,), (200,), (70, 130), ((200, 30),)):
        s = P.Simulator(ens.params, sizes, precision="fp32c", launch=RESIDENT)
        s.set_state(ens.X, ens.phi)
        for n in calls:
            nsteps, every = (n if isinstance(n, tuple) else (n, 0))
            _, _, code = s.run(nsteps, every)
            assert code == 0
        out.append(s.get_state()[0].cpu().numpy())
    for o in out[1:]:
        assert np.array_equal(out[0], o)
    # the streamed form needs the largest workspace of the three: created with
    # it, the context keeps its state through every change of form
    s = P.Simulator(ens.params, sizes, precision="fp32c", launch=STREAM_SINGLE)
    s.set_state(ens.X, ens.phi)
    ctx = s.ctx
    for L in (RESIDENT, STREAM_SINGLE, RESIDENT, dict(RESIDENT, fused=0), RESIDENT):
        s.set_launch(**L)
        assert s.ctx == ctx
        _, _, code = s.run(40, 0)
        assert code == 0
    Xo, _, _, _ = oracle.run(ens.params, ens.X, ens.phi, 200, S_per_sys=sizes)
    off = ens.sphere_offsets
    X = s.get_state()[0].cpu().numpy()
    for b in range(len(sizes)):
        sl = slice(off[b], off[b + 1])
        check_fp32c(X[sl] - ens.X[sl], Xo[sl] - ens.X[sl], f"forms in turn, system {b}")


def test_resident_coincident_spheres_raise_flag():
    _torch()
    sus = make_single(8, 30.0, 3)
    X = sus.X.copy()
    X[5] = X[2]
    for precision in ("fp64", "fp32c"):
        s = P.Simulator(sus.params, [sus.S], precision=precision, launch=RESIDENT)
        s.set_state(X, sus.phi)
        _, _, code = s.run(2, 1)
        assert code == P.binding.AD_ENONFINITE, precision
