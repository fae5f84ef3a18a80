"""The pair and array experiments of Sec. IV on the oracle: the input
generators, the observables, and the paper's claims about how the
microscopic model and the stroke-averaged equations compare.

Every observable is taken over whole stroke periods after one settling period
(reading of the paper: it does not say when its measurements start; from rest
the springs first settle onto the stroke, and that transient moves the centres
at first order in the interaction, which would swamp the second-order
swimming signal). The stroke-averaged run starts from the microscopic state at
the end of the settling period.

Claims checked (values are not printed in the paper, so these are the shapes):
* Sec. IV.C, Fig. 3: the mean square displacement per period scales as
  (ell rho^(1/3))^(2 nu) with nu = -4, for both models;
* Sec. IV.C, Figs. 3-4: checkerboard phases give a larger mean square
  displacement than random phases;
* Sec. IV.C, Figs. 3-4 captions: the shift between the models is the one the
  aligned pair shows at the same a/ell (Fig. 1c);
* Sec. IV.B, Fig. 2: the stroke-averaged equations reproduce the microscopic
  change of the relative orientation Delta q, up to the same shift.
"""
import math

import numpy as np
import pytest

from paper_1004_1932_amd import observables as obs
from workload import array_runs, checkerboard_phases, fig1_params, lattice_array, place_dumbbells, rotation_pairs
from workload.arrays import lattice_indices

SPP = 5000  # steps per period (dt = 2e-4 T)


def test_checkerboard_lattice():
    """Nearest lattice neighbours hold the other phase; the lattice has the
    requested spacing, is centred at the origin, and the axes are unit."""
    x, sp = 5, 7.0
    R, N, phi = lattice_array(x, sp, 3, "checkerboard")
    assert R.shape == (125, 3) and set(np.unique(phi)) == {0.0, 0.5 * math.pi}
    np.testing.assert_allclose(R.mean(0), 0.0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(N, axis=1), 1.0, atol=1e-15)
    d = np.linalg.norm(R[:, None] - R[None], axis=-1)
    nb = np.isclose(d, sp)
    assert nb.sum() == 2 * 3 * x * x * (x - 1)  # neighbour pairs of a cubic lattice, both orders
    assert np.all(phi[:, None] != phi[None, :], where=nb)
    idx = lattice_indices(3)
    assert checkerboard_phases(idx)[0] == 0.0 and checkerboard_phases(idx)[1] == 0.5 * math.pi
    _, _, pr = lattice_array(x, sp, 3, "random")
    assert pr.min() >= 0 and pr.max() < 2 * math.pi and len(np.unique(pr)) == 125
    with pytest.raises(ValueError):
        lattice_array(2, 1.0, 0, "optimal")


def test_observables_by_hand():
    R0 = np.array([[0.0, 0, 0], [1, 0, 0], [0, 0, 0], [0, 2, 0]])
    R1 = np.array([[1.0, 0, 0], [1, 0, 0], [0, 0, 3], [0, 2, 4]])
    np.testing.assert_allclose(obs.msd_per_system(R1, R0, [2, 2]), [0.5, 12.5])
    assert obs.ensemble_msd(R1, R0, [2, 2]) == 6.5
    np.testing.assert_allclose(obs.pair_mean_displacement(R1, R0), [[0.5, 0, 0], [0, 0, 3.5]])
    np.testing.assert_allclose(obs.pair_separation_change(R1, R0), [[-1, 0, 0], [0, 0, 1]])
    X = np.array([[0.0, 0, 0], [2, 0, 0], [0, 0, 0], [0, 0, 5]])
    np.testing.assert_allclose(obs.centres(X), [[1, 0, 0], [0, 0, 2.5]])
    np.testing.assert_allclose(obs.axes(X), [[1, 0, 0], [0, 0, 1]])
    np.testing.assert_allclose(obs.pair_projection(obs.axes(X)), [0.0])
    with pytest.raises(ValueError):
        obs.msd_per_system(R1, R0, [3, 2])


def micro_then_sa(oracle, ens, phi_runs, periods):
    """One settling period, then `periods` periods of the microscopic model
    (oracle, all runs as one ensemble) and of the stroke-averaged equations
    from the settled state. Returns (R_T, N_T, R_mic, N_mic, R_sa, N_sa),
    dumbbells of all runs concatenated."""
    p = ens.params
    S = ens.S_per_sys
    X1, _, _, _ = oracle.run(p, ens.X, ens.phi, SPP, S_per_sys=S)
    X2, _, _, _ = oracle.run(p, X1, ens.phi, periods * SPP, t0=0.0, step0=SPP, S_per_sys=S)
    R1, N1 = obs.centres(X1), obs.axes(X1)
    Rs, Ns, o = [], [], 0
    for b, Sb in enumerate(S):
        r, n = oracle.sa_run(p, R1[o:o + Sb], N1[o:o + Sb], phi_runs[b], p.T / 20, 20 * periods)
        Rs.append(r)
        Ns.append(n)
        o += Sb
    return R1, N1, obs.centres(X2), obs.axes(X2), np.concatenate(Rs), np.concatenate(Ns)


@pytest.fixture(scope="module")
def array_msd(oracle):
    """<<R(T)^2>> of 3x3x3 arrays, W = 4 runs, for both models, both phase
    kinds and spacings 10 ell and 20 ell."""
    p = fig1_params(0.2, SPP)
    out = {}
    for phases in ("checkerboard", "random"):
        for sp in (10, 20):
            ens, _, _, phi = array_runs(3, sp * p.ell, 4, phases, seed=11, params=p)
            R1, _, Rm, _, Rs, _ = micro_then_sa(oracle, ens, phi, 1)
            out[phases, sp] = (obs.ensemble_msd(Rm, R1, ens.S_per_sys), obs.ensemble_msd(Rs, R1, ens.S_per_sys))
    return out


def test_array_msd_scales_with_density(array_msd):
    """Doubling the spacing divides <<R(T)^2>> by 2^8 (nu = -4): exactly for
    the stroke-averaged equations (every velocity scales as D^-4), up to
    near-field corrections of order ell/D for the microscopic model."""
    for phases in ("checkerboard", "random"):
        (m10, s10), (m20, s20) = array_msd[phases, 10], array_msd[phases, 20]
        assert abs(math.log2(s10 / s20) - 8) < 0.02, (phases, s10 / s20)
        assert abs(math.log2(m10 / m20) - 8) < 0.2, (phases, m10 / m20)


def test_checkerboard_beats_random_phases(array_msd):
    for sp in (10, 20):
        for model in (0, 1):
            assert array_msd["checkerboard", sp][model] > 1.3 * array_msd["random", sp][model]


def test_model_shift_matches_the_aligned_pair(oracle, array_msd):
    """sqrt of the microscopic / stroke-averaged ratio of <<R(T)^2>> equals,
    within 10 %, the ratio of the two models' displacements of an aligned
    pair at the same a/ell and distance (the shift of Fig. 1c)."""
    p = fig1_params(0.2, SPP)
    R = np.array([[0.0, 0, 0], [10 * p.ell, 0, 0]])
    N = np.array([[1.0, 0, 0], [1.0, 0, 0]])
    phi = np.array([0.0, 0.5 * math.pi])
    X1, _, _, _ = oracle.run(p, place_dumbbells(R, N, phi, p), phi, SPP)
    X2, _, _, _ = oracle.run(p, X1, phi, SPP, t0=0.0, step0=SPP)
    R1 = obs.centres(X1)
    Rs, _ = oracle.sa_run(p, R1, obs.axes(X1), phi, p.T / 20, 20)
    d_mic = np.linalg.norm(obs.pair_mean_displacement(obs.centres(X2), R1))
    d_sa = np.linalg.norm(obs.pair_mean_displacement(Rs, R1))
    shift = d_mic / d_sa
    assert 1.1 < shift < 1.6, shift  # a/ell = 0.2 is far from the a/ell -> 0 limit
    for key, (m, s) in array_msd.items():
        assert abs(math.sqrt(m / s) / shift - 1) < 0.1, (key, math.sqrt(m / s), shift)


def test_pair_rotation_follows_the_stroke_averaged_law(oracle):
    """Fig. 2 setup: Delta q over five periods for pairs at distance 5 ell,
    q(0) = 0 and 1, several angles: the microscopic change has the sign of
    the stroke-averaged one and the same shift as the translations."""
    p = fig1_params(0.2, SPP)
    for q0, degs in ((0.0, (15, 75, 105, 165)), (1.0, (15, 45, 75))):
        ens, _, _, phi = rotation_pairs(np.radians(degs), q0, 5 * p.ell, params=p)
        _, N1, _, Nm, _, Ns = micro_then_sa(oracle, ens, phi, 5)
        q1 = obs.pair_projection(N1)
        dq_mic = obs.pair_projection(Nm) - q1
        dq_sa = obs.pair_projection(Ns) - q1
        ratio = dq_mic / dq_sa
        assert np.all(ratio > 1.1) and np.all(ratio < 1.8), (q0, ratio)
