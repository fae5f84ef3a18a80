"""The seeded input generator: distributions and exclusion (recipe in
workload/suspensions.py)."""
import math

import numpy as np

from workload import Params, make_ensemble, make_single, place_dumbbells
from workload.suspensions import ensemble_sizes, min_pair_distance


def test_single_system_recipe():
    sus = make_single(256, 120.0, 0)
    assert sus.X.shape == (512, 3) and sus.phi.shape == (256,)
    R = 0.5 * (sus.X[0::2] + sus.X[1::2])
    assert np.all(np.abs(R) <= 60.0)
    d = np.linalg.norm(sus.X[1::2] - sus.X[0::2], axis=1)
    L0 = sus.params.ell + sus.params.lam * np.sin(sus.phi)
    np.testing.assert_allclose(d, L0, rtol=1e-14)
    assert np.all((sus.phi >= 0) & (sus.phi < 2 * math.pi))
    assert min_pair_distance(sus.X) >= 2 * sus.params.a


def test_orientations_uniform_on_sphere():
    sus = make_single(4000, 2000.0, 1)
    n = sus.X[1::2] - sus.X[0::2]
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    # first and second moments of the uniform distribution on S^2
    assert np.abs(n.mean(0)).max() < 0.05
    np.testing.assert_allclose(n.T @ n / len(n), np.eye(3) / 3, atol=0.03)
    assert abs(sus.phi.mean() - math.pi) < 0.1


def test_seeded_and_reproducible():
    a, b = make_single(64, 50.0, 7), make_single(64, 50.0, 7)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.phi, b.phi)
    assert not np.array_equal(a.X, make_single(64, 50.0, 8).X)


def test_exclusion_switch():
    # dense enough that the literal uniform draw overlaps
    lit = make_single(300, 25.0, 3, exclusion=False)
    rsa = make_single(300, 25.0, 3)
    assert min_pair_distance(lit.X) < 2.0 <= min_pair_distance(rsa.X)


def test_ensemble_recipe():
    S = ensemble_sizes(512)
    assert S.min() >= 16 and S.max() <= 400
    ens = make_ensemble(nsys=6, sizes=S[:6])
    assert ens.X.shape[0] == 2 * int(S[:6].sum())
    for b in range(6):
        sys_b = ens.system(b)
        ref = make_single(int(S[b]), (2 * float(S[b]) / 0.02) ** (1 / 3), 1 + b)
        assert np.array_equal(sys_b.X, ref.X)


def test_place_dumbbells_rest_length():
    p = Params()
    X = place_dumbbells([[0, 0, 0]], [[0, 0, 2.0]], [math.pi / 2], p)
    np.testing.assert_allclose(X, [[0, 0, -2.5], [0, 0, 2.5]])
