"""Pins of the oracle's Brownian option: additive noise with a constant C
(Sec. V; Eq. e:langevin with Eq. e:cholesky on the diagonal of H), drawn from
Philox4x32-10 and Box-Muller. Pinned to the generator's published
known-answer vectors, to the statistics of the normals and to
free diffusion of isolated dumbbells, whose centre moves only by the noise
(the spring forces cancel in the centre velocity), so that its mean square
displacement is 3 kT t/(6 pi eta a)."""
import math

import numpy as np
import pytest

from oracle.adref import OracleError
from workload import Params, make_ensemble


def test_normals_statistics(oracle):
    z = np.array([oracle.gauss3(11, i, n) for i in range(3000) for n in range(4)]).reshape(-1)
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 6 * math.sqrt(2 / z.size)
    # fourth moment of a standard normal is 3
    assert abs((z ** 4).mean() - 3) < 0.15
    # neighbouring counters are uncorrelated
    a = np.array([oracle.gauss3(11, i, 0) for i in range(3000)])
    b = np.array([oracle.gauss3(11, i + 1, 0) for i in range(3000)])
    c = np.array([oracle.gauss3(11, i, 1) for i in range(3000)])
    for x, y in ((a, b), (a, c), (a[:, 0], a[:, 1])):
        r = np.corrcoef(np.ravel(x), np.ravel(y))[0, 1]
        assert abs(r) < 4 / math.sqrt(3000 * (1 if np.ndim(x) == 1 else 3))
    # keys matter
    assert not np.array_equal(oracle.gauss3(11, 5, 7), oracle.gauss3(12, 5, 7))


def test_isolated_dumbbells_diffuse_freely(oracle):
    """400 isolated passive dumbbells (one per system), Heun with noise:
    mean square centre displacement 3 kT t/(6 pi eta a) within sampling
    error; without noise the centres do not move."""
    p = Params(lam=0.0, dt=0.01)
    sizes = np.ones(400, dtype=np.int32)
    ens = make_ensemble(nsys=400, sizes=sizes, params=p)
    kT, nsteps = 0.05, 200
    R0 = 0.5 * (ens.X[0::2] + ens.X[1::2])
    X, cen, _, _ = oracle.run(p, ens.X, ens.phi, nsteps, record_every=nsteps, S_per_sys=sizes,
                              integrator=1, kT=kT, seed=3)
    msd = ((cen[-1] - R0) ** 2).sum(1).mean()
    expect = 3 * kT * (1 / (6 * math.pi * p.eta * p.a)) * nsteps * p.dt
    assert abs(msd / expect - 1) < 0.15, msd / expect
    X0, cen0, _, _ = oracle.run(p, ens.X, ens.phi, nsteps, record_every=nsteps, S_per_sys=sizes, integrator=1)
    assert np.abs(cen0[-1] - R0).max() < 1e-12


def test_noise_reproducible_and_resumable(oracle):
    p = Params()
    ens = make_ensemble(nsys=3, sizes=np.array([4, 7, 2], dtype=np.int32), params=p)
    kw = dict(S_per_sys=[4, 7, 2], integrator=1, kT=0.01, seed=9)
    a = oracle.run(p, ens.X, ens.phi, 100, **kw)[0]
    b = oracle.run(p, ens.X, ens.phi, 100, **kw)[0]
    assert np.array_equal(a, b)
    h = oracle.run(p, ens.X, ens.phi, 50, **kw)[0]
    c = oracle.run(p, h, ens.phi, 50, step0=50, **kw)[0]
    assert np.array_equal(a, c)
    d = oracle.run(p, ens.X, ens.phi, 100, **dict(kw, seed=10))[0]
    assert not np.array_equal(a, d)


def test_noise_needs_heun(oracle):
    p = Params()
    ens = make_ensemble(nsys=1, sizes=np.array([3], dtype=np.int32), params=p)
    with pytest.raises(OracleError):
        oracle.run(p, ens.X, ens.phi, 2, integrator=0, kT=0.1)


def test_philox_known_answers(oracle, golden_dir):
    """The oracle's Philox4x32-10 block against the generator's published
    known-answer vectors (fixture tests/golden/philox4x32_10_kat.json)."""
    import json
    kat = json.loads((golden_dir / "philox4x32_10_kat.json").read_text())
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["counter"]]
        key = [int(x, 16) for x in v["key"]]
        assert oracle.philox(ctr, key) == [int(x, 16) for x in v["output"]]
