"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it follows. None re-types the oracle's own sum:
the checks are closed forms (Stokeslet values, the single-dumbbell length
equation of App. A), invariants (symmetry, positive definiteness, zero
divergence, translation/rotation/permutation invariance, inversion symmetry),
brute force (the dense 3N x 3N tensor), convergence orders, and the paper's
far-field aligned-pair law (Sec. IV.A, Fig. 1).
"""
import json
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from workload import Params, make_single, place_dumbbells

PI = math.pi


def rot(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def small_suspension(S=12, side=30.0, seed=3, **kw):
    return make_single(S, side, seed, Params(**kw))


# ---------------------------------------------------------------- closed forms

def test_stokeslet_pair_closed_form(oracle):
    """Sec. II, Eq. (e:Mazur): two spheres, force on one. The velocity of the
    other is the Stokeslet: 1/(4 pi eta r) along the line of centres and
    1/(8 pi eta r) across it; the loaded sphere moves with 1/(6 pi eta a)."""
    p = Params(a=1.0, eta=1.0)
    e = np.array([2.0, -1.0, 2.0]) / 3.0          # unit axis
    r = 3.0
    X = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3]]) + np.array([[0, 0, 0], r * e])
    perp = np.array([1.0, 2.0, 0.0]) / math.sqrt(5.0)
    assert abs(perp @ e) < 1e-15
    for direction, coef in ((e, 0.026525823848649224),        # 1/(4 pi * 3)
                            (perp, 0.013262911924324612)):     # 1/(8 pi * 3)
        F = np.array([[0.0, 0.0, 0.0], 2.5 * direction])
        u = oracle.mobility(p, X, F)
        np.testing.assert_allclose(u[0], 2.5 * coef * direction, rtol=0, atol=1e-15)
        np.testing.assert_allclose(u[1], 2.5 * 0.05305164769729845 * direction, rtol=0, atol=1e-15)


def test_single_dumbbell_coefficients(oracle, golden_dir):
    """App. A.2, Eq. (e:h-symm): for a dumbbell of length L, the oracle's
    mobility contracted with the axis gives h_self = 4 kappa/(3a) and
    h_partner = 2 kappa/L."""
    g = json.loads((golden_dir / "single_dumbbell_coefficients.json").read_text())
    p = Params(a=g["a"], eta=g["mu"])
    n = np.array([0.0, 0.6, 0.8])
    X = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 1.0] + g["L"] * n])
    u = oracle.mobility(p, X, np.array([[0.0, 0.0, 0.0], n]))
    assert abs(u[1] @ n - g["h_self"]) < 1e-16
    assert abs(u[0] @ n - g["h_partner"]) < 1e-16


def test_isolated_dumbbell_length_follows_app_a(oracle, golden_dir):
    """App. A.2: an isolated dumbbell's length obeys dd/dt = b(d) k (d - L(t)),
    b(d) = (4 kappa/d)(1 - 2d/(3a)). Integrate that scalar ODE independently
    and compare the oracle's 3d RK4 trajectory. Scallop theorem (Sec. I,
    Sec. V): the centre and the axis do not move."""
    g = json.loads((golden_dir / "single_dumbbell_coefficients.json").read_text())
    kappa = g["kappa"]
    p = Params(a=1.0, eta=1.0, k=1.0, ell=4.0, lam=1.0, T=100.0, dt=0.01)
    # start off the potential minimum so the length relaxes as well as follows L(t)
    R = np.array([3.0, -2.0, 5.0])
    n = np.array([1.0, 2.0, -2.0]) / 3.0
    phi = 0.7
    d0 = 4.6
    X = np.array([R - 0.5 * d0 * n, R + 0.5 * d0 * n])
    omega = 2 * PI / p.T

    def rhs(t, y):
        d = y[0]
        b = (4 * kappa / d) * (1 - 2 * d / (3 * p.a))
        return [b * p.k * (d - (p.ell + p.lam * math.sin(omega * t + phi)))]

    nsteps, rec = 5000, 500
    Xn, cen, _, _ = oracle.run(p, X, np.array([phi]), nsteps, record_every=rec)
    times = np.arange(1, nsteps // rec + 1) * rec * p.dt
    sol = solve_ivp(rhs, (0, times[-1]), [d0], t_eval=times, rtol=1e-12, atol=1e-14, method="DOP853")
    # lengths at the record times, by advancing in record-sized pieces
    Xr = X.copy()
    lengths = []
    for _ in range(len(times)):
        Xr, _, _, _ = oracle.run(p, Xr, np.array([phi]), rec, t0=0.0, step0=len(lengths) * rec)
        lengths.append(np.linalg.norm(Xr[1] - Xr[0]))
    np.testing.assert_allclose(lengths, sol.y[0], rtol=0, atol=1e-10)
    # centre fixed and axis fixed (only rounding)
    assert np.abs(cen - R).max() < 1e-12
    axis = (Xn[1] - Xn[0]) / np.linalg.norm(Xn[1] - Xn[0])
    assert np.abs(axis - n).max() < 1e-12


def test_rest_length_is_paper_formula(oracle):
    """Eq. (e:swimmer_potential): L(t) = ell + lam sin(omega t + phi), here via
    the addition theorem; equal to the direct form within the rounding of
    the phase argument (a few ulp of omega t + phi)."""
    p = Params()
    rng = np.random.default_rng(0)
    eps = np.finfo(float).eps
    for t, phi in zip(rng.uniform(0, 1e4, 200), rng.uniform(0, 2 * PI, 200)):
        arg = 2 * PI / p.T * t
        direct = p.ell + p.lam * math.sin(arg + phi)
        bound = 4 * eps * (abs(arg) + 2 * PI) * p.lam + 4 * eps * p.ell
        assert abs(oracle.rest_length(p, t, phi) - direct) < bound


# ---------------------------------------------------------------- forces

def test_forces_internal_and_central(oracle):
    """Sec. II and App. A (force-free, torque-free swimmers): the two spring
    forces of a dumbbell cancel exactly and act along its axis; at d = L(t)
    they vanish; their magnitude is k |d - L|."""
    sus = small_suspension()
    p = sus.params
    t = 13.7
    X = sus.X + np.random.default_rng(1).normal(scale=0.05, size=sus.X.shape)
    F = oracle.forces(p, X, sus.phi, t)
    assert np.array_equal(F[0::2], -F[1::2])
    n = X[1::2] - X[0::2]
    d = np.linalg.norm(n, axis=1)
    L = p.ell + p.lam * np.sin(2 * PI / p.T * t + sus.phi)
    assert np.abs(np.cross(F[1::2], n)).max() < 1e-15
    np.testing.assert_allclose(np.linalg.norm(F[1::2], axis=1), p.k * np.abs(d - L), rtol=1e-12, atol=1e-15)
    # force on sphere 2s+1 pulls it back toward L: sign of -(d - L) along n
    np.testing.assert_array_equal(np.sign(np.einsum("ij,ij->i", F[1::2], n)), -np.sign(d - L))
    # at the potential minimum the forces vanish (initial state at t = 0)
    F0 = oracle.forces(p, sus.X, sus.phi, 0.0)
    assert np.abs(F0).max() < 1e-14


def test_spring_energy_hand_values(oracle):
    """Eq. (e:swimmer_potential): U = sum_s k/2 (d_s - L_s(t))^2. Two
    dumbbells with k = 3: d = 5 against L = 4 (phase 0, t = 0) gives 3/2;
    d = 3 against L = 5 (phase pi/2) gives 6; a quarter period later the
    first rest length is 5 as well (d - L = 0) and the second 4 (d - L =
    -1, 3/2)."""
    p = Params(k=3.0)
    X = np.array([[1.0, 2.0, 3.0], [6.0, 2.0, 3.0], [-4.0, 0.0, 0.0], [-4.0, 0.0, 3.0]])
    phi = np.array([0.0, PI / 2])
    assert abs(oracle.energy(p, X, phi, 0.0) - 7.5) < 1e-13
    assert abs(oracle.energy(p, X, phi, p.T / 4) - 1.5) < 1e-13


def test_forces_are_minus_energy_gradient(oracle):
    """F = -grad U (Sec. II): central differences of the oracle's energy
    against the oracle's forces, sphere by sphere."""
    sus = small_suspension(S=5)
    p = Params(k=2.5)
    X = sus.X + np.random.default_rng(4).normal(scale=0.3, size=sus.X.shape)
    t, h = 21.3, 1e-6
    F = oracle.forces(p, X, sus.phi, t)
    G = np.empty_like(X)
    for i in range(X.shape[0]):
        for a in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[i, a] += h
            Xm[i, a] -= h
            G[i, a] = -(oracle.energy(p, Xp, sus.phi, t) - oracle.energy(p, Xm, sus.phi, t)) / (2 * h)
    assert np.abs(F).max() > 0.1
    np.testing.assert_allclose(G, F, rtol=0, atol=1e-7)


def test_steric_repulsion(oracle):
    """Steric option: equal and opposite, along the separation, k_s (r_c - r)
    in magnitude below r_c, zero beyond."""
    p = Params(steric_k=100.0, steric_r=2.0, lam=0.0)
    # two dumbbells at rest length 4, spheres 1 and 2 at distance 1.5
    X = np.array([[0, 0, 0], [4, 0, 0], [4, 1.5, 0], [8, 1.5, 0]], dtype=float)
    phi = np.zeros(2)
    F = oracle.forces(p, X, phi, 0.0)
    np.testing.assert_allclose(F[1], [0, -50.0, 0], atol=1e-12)
    np.testing.assert_allclose(F[2], [0, 50.0, 0], atol=1e-12)
    np.testing.assert_allclose(F[0], 0, atol=1e-12)
    X2 = X.copy()
    X2[2:, 1] = 2.0
    assert np.abs(oracle.forces(p, X2, phi, 0.0)).max() < 1e-12


# ---------------------------------------------------------------- invariants

def test_mobility_symmetric(oracle):
    """Sec. II: H_ij = H_ji (Eq. e:Mazur is symmetric), so v.Mw = w.Mv."""
    sus = small_suspension(S=20)
    rng = np.random.default_rng(5)
    v, w = rng.standard_normal((2, sus.N, 3))
    Mv, Mw = oracle.mobility(sus.params, sus.X, v), oracle.mobility(sus.params, sus.X, w)
    a, b = np.sum(v * Mw), np.sum(w * Mv)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_mobility_linear(oracle):
    sus = small_suspension(S=20)
    rng = np.random.default_rng(6)
    v, w = rng.standard_normal((2, sus.N, 3))
    lhs = oracle.mobility(sus.params, sus.X, 2.5 * v - 0.75 * w)
    rhs = 2.5 * oracle.mobility(sus.params, sus.X, v) - 0.75 * oracle.mobility(sus.params, sus.X, w)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-14 * np.abs(rhs).max())


def test_mobility_positive_definite(oracle):
    """Sec. II: H is positive definite when all sphere distances exceed 2a
    (checked on the assembled tensor)."""
    sus = small_suspension(S=16, side=60.0)
    from workload.suspensions import min_pair_distance
    assert min_pair_distance(sus.X) > 2 * sus.params.a
    N = sus.N
    H = np.stack([oracle.mobility(sus.params, sus.X, e.reshape(N, 3)).reshape(-1)
                  for e in np.eye(3 * N)], axis=1)
    assert np.abs(H - H.T).max() < 1e-15
    assert np.linalg.eigvalsh(H).min() > 0


def test_mobility_divergence_free(oracle):
    """Sec. II: d/dx_(beta j) H_(alpha i)(beta j) = 0. Central differences of
    the velocity of sphere i with respect to the position of sphere j, for a
    unit force on j along each axis, summed over the axis."""
    p = Params()
    rng = np.random.default_rng(2)
    X = rng.uniform(-6, 6, (5, 3))
    h = 1e-5
    for i in range(5):
        for j in range(5):
            if i == j:
                continue
            div = np.zeros(3)
            for b in range(3):
                F = np.zeros((5, 3))
                F[j, b] = 1.0
                Xp, Xm = X.copy(), X.copy()
                Xp[j, b] += h
                Xm[j, b] -= h
                div += (oracle.mobility(p, Xp, F)[i] - oracle.mobility(p, Xm, F)[i]) / (2 * h)
            assert np.abs(div).max() < 1e-8


def test_dense_tensor_equals_matrix_free(oracle):
    """Brute force: the assembled 3N x 3N tensor (the paper's own design,
    Sec. V) times F equals the matrix-free pair loop."""
    for tensor in (0, 1):
        sus = small_suspension(S=32, side=40.0)
        F = np.random.default_rng(8).standard_normal(sus.X.shape)
        a = oracle.mobility(sus.params, sus.X, F, tensor=tensor)
        b = oracle.mobility_dense(sus.params, sus.X, F, tensor=tensor)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.abs(a).max())


def test_translation_and_rotation_invariance(oracle):
    """Free space (Sec. IV): shifting the suspension leaves velocities
    unchanged; rotating it rotates them."""
    sus = small_suspension()
    p = sus.params
    F = oracle.forces(p, sus.X + 0.03, sus.phi, 7.0)
    u = oracle.mobility(p, sus.X, F)
    shift = np.array([13.25, -7.5, 2.125])
    np.testing.assert_allclose(oracle.mobility(p, sus.X + shift, F), u, rtol=0, atol=1e-14 * np.abs(u).max())
    Q = rot(4)
    uq = oracle.mobility(p, sus.X @ Q.T, F @ Q.T)
    np.testing.assert_allclose(uq, u @ Q.T, rtol=0, atol=1e-13 * np.abs(u).max())
    # trajectories too
    X1, _, _, _ = oracle.run(p, sus.X, sus.phi, 200)
    X2, _, _, _ = oracle.run(p, sus.X @ Q.T + shift, sus.phi, 200)
    np.testing.assert_allclose(X2, X1 @ Q.T + shift, rtol=0, atol=1e-11)


def test_permutation_invariance(oracle):
    """Relabelling dumbbells permutes the output."""
    sus = small_suspension(S=10)
    p = sus.params
    perm = np.random.default_rng(9).permutation(sus.S)
    sph = np.stack([2 * perm, 2 * perm + 1], 1).reshape(-1)
    X1, _, _, _ = oracle.run(p, sus.X, sus.phi, 300)
    X2, _, _, _ = oracle.run(p, sus.X[sph], sus.phi[perm], 300)
    np.testing.assert_allclose(X2, X1[sph], rtol=0, atol=1e-12)


def test_passive_dumbbells(oracle):
    """Sec. II: lam = 0 gives passive dumbbells. At rest length nothing moves;
    from a stretched state the spring energy decays monotonically (gradient
    flow with a positive-definite mobility)."""
    p = Params(lam=0.0)
    sus = make_single(10, 40.0, 11, p)
    F = oracle.forces(p, sus.X, sus.phi, 5.0)
    assert np.abs(oracle.mobility(p, sus.X, F)).max() < 1e-15
    rng = np.random.default_rng(3)
    X = sus.X + rng.normal(scale=0.2, size=sus.X.shape)
    energies = [oracle.energy(p, X, sus.phi, 0.0)]
    for n in range(20):
        X, _, _, _ = oracle.run(p, X, sus.phi, 50, step0=50 * n)
        energies.append(oracle.energy(p, X, sus.phi, 0.0))
    assert np.all(np.diff(energies) < 0)


def test_inversion_symmetric_suspension_keeps_com(oracle):
    """Pairs (R, N, phi) and (-R, N, phi): the velocity field is odd under
    inversion, so the centre of mass stays at the origin."""
    rng = np.random.default_rng(12)
    S2 = 8
    R = rng.uniform(-20, 20, (S2, 3))
    Nv = rng.standard_normal((S2, 3))
    phi = rng.uniform(0, 2 * PI, S2)
    p = Params()
    # the mirror image of a dumbbell is the same dumbbell with its spheres swapped
    # (its sphere k sits at minus the position of the original's other sphere)
    X = place_dumbbells(np.concatenate([R, -R]), np.concatenate([Nv, Nv]), np.concatenate([phi, phi]), p)
    X[2 * S2:] = -X[:2 * S2].reshape(S2, 2, 3)[:, ::-1].reshape(-1, 3)
    Xn, _, com, _ = oracle.run(p, X, np.concatenate([phi, phi]), 2000, record_every=500)
    assert np.abs(com).max() < 1e-13
    assert np.abs(Xn - X).max() > 1e-3


def test_ensemble_equals_independent_systems(oracle):
    """Independent suspensions batched together evolve exactly as alone."""
    p = Params()
    a = make_single(6, 25.0, 1, p)
    b = make_single(9, 30.0, 2, p)
    X = np.concatenate([a.X, b.X])
    phi = np.concatenate([a.phi, b.phi])
    Xe, cen, com, _ = oracle.run(p, X, phi, 400, record_every=100, S_per_sys=[6, 9])
    Xa, ca, ma, _ = oracle.run(p, a.X, a.phi, 400, record_every=100)
    Xb, cb, mb, _ = oracle.run(p, b.X, b.phi, 400, record_every=100)
    assert np.array_equal(Xe, np.concatenate([Xa, Xb]))
    assert np.array_equal(cen, np.concatenate([ca, cb], axis=1))
    assert np.array_equal(com[:, 0], ma[:, 0]) and np.array_equal(com[:, 1], mb[:, 0])


def test_thread_count_does_not_change_results(oracle):
    sus = small_suspension(S=40, side=50.0)
    n0 = oracle.max_threads()
    oracle.set_threads(1)
    X1, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 100)
    oracle.set_threads(max(2, n0))
    X2, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 100)
    oracle.set_threads(n0)
    assert np.array_equal(X1, X2)


def test_resume_is_exact(oracle):
    """Step n starts at t0 + n dt: 2m steps equal m steps, then m more from
    step index m."""
    sus = small_suspension()
    X2, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 600)
    Xa, _, _, _ = oracle.run(sus.params, sus.X, sus.phi, 300)
    Xb, _, _, _ = oracle.run(sus.params, Xa, sus.phi, 300, step0=300)
    assert np.array_equal(X2, Xb)


# ---------------------------------------------------------------- integrators

def _convergence(oracle, integrator, steps_list, Tend):
    p0 = Params(k=5.0)
    sus = make_single(4, 16.0, 21, p0)
    X = sus.X + np.random.default_rng(0).normal(scale=0.1, size=sus.X.shape)
    from dataclasses import replace
    ref_steps = steps_list[-1] * 8
    ref, _, _, _ = oracle.run(replace(p0, dt=Tend / ref_steps), X, sus.phi, ref_steps, integrator=0)
    errs = []
    for n in steps_list:
        Xn, _, _, _ = oracle.run(replace(p0, dt=Tend / n), X, sus.phi, n, integrator=integrator)
        errs.append(np.abs(Xn - ref).max())
    return np.array(errs)


def test_rk4_is_fourth_order(oracle):
    errs = _convergence(oracle, 0, [25, 50, 100], 20.0)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 13) and np.all(ratios < 19), ratios


def test_heun_is_second_order(oracle):
    """Sec. V: the paper's Heun predictor-corrector, second order."""
    errs = _convergence(oracle, 1, [50, 100, 200], 20.0)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 3.5) and np.all(ratios < 4.5), ratios


# ---------------------------------------------------------------- RPY

def test_rpy_correction_is_textbook_rpy(oracle):
    """Eq. (e:Mazur_offdiagonal) with both lines equals the textbook
    Rotne-Prager-Yamakawa tensor (1/(8 pi eta r))[(1 + 2a^2/(3r^2)) I +
    (1 - 2a^2/r^2) rr/r^2] for r >= 2a."""
    p = Params(a=1.0, eta=1.3)
    rng = np.random.default_rng(4)
    for _ in range(5):
        r = rng.uniform(2.0, 9.0)
        e = rng.standard_normal(3)
        e /= np.linalg.norm(e)
        X = np.array([[0, 0, 0], r * e])
        F = np.zeros((2, 3))
        F[1] = rng.standard_normal(3)
        u = oracle.mobility(p, X, F, tensor=1)[0]
        a = p.a
        ref = (1 / (8 * PI * p.eta * r)) * ((1 + 2 * a * a / (3 * r * r)) * F[1]
                                            + (1 - 2 * a * a / (r * r)) * e * (e @ F[1]))
        np.testing.assert_allclose(u, ref, rtol=1e-14, atol=1e-17)


# ---------------------------------------------------------------- far field (Fig. 1)

def _aligned_pair_displacement(oracle, g, a_over_ell, D_over_ell, dphi, periods=2, steps_per_period=10000):
    ell = g["ell_m"]
    omega = g["omega_per_s"]
    T = 2 * PI / omega
    p = Params(a=a_over_ell * ell, eta=g["mu_kg_per_m_s"], k=g["k0_kg_per_s2"], ell=ell,
               lam=g["lam_over_ell"] * ell, T=T, dt=T * g["dt_over_T"])
    assert abs(p.dt - T / steps_per_period) < 1e-20
    D = D_over_ell * ell
    phi = np.array([0.0, dphi])
    X = place_dumbbells([[0, 0, 0], [D, 0, 0]], [[1, 0, 0], [1, 0, 0]], phi, p)
    # Sec. V: the first period is discarded (settling of the springs)
    _, cen, _, _ = oracle.run(p, X, phi, periods * steps_per_period, record_every=steps_per_period)
    disp = cen[-1] - cen[-2]
    sa = g["far_field_prefactor"] * p.a * omega * (p.lam / ell) ** 2 * (ell / D) ** 4 * T
    return disp, sa


@pytest.mark.parametrize("dummy", [0])
def test_aligned_pair_far_field_law(oracle, golden_dir, dummy):
    """Sec. IV.A, Eq. (e:stroke_averaged) and Fig. 1: both dumbbells swim the
    same way with equal speed, in the direction set by the phase difference
    (+x for phi_2 - phi_1 = pi/2 with dumbbell 2 at larger x); the
    displacement per stroke decays as |D|^-4; the ratio to the stroke-averaged
    law tends to 1 as a/ell -> 0 at lam = 0.1 ell."""
    g = json.loads((golden_dir / "fig1_aligned_pair.json").read_text())
    dphi = PI / 2
    d10, sa10 = _aligned_pair_displacement(oracle, g, g["a_over_ell"], 10.0, dphi)
    # same direction, same speed, transverse components zero
    assert d10[0, 0] > 0 and d10[1, 0] > 0
    assert abs(d10[0, 0] - d10[1, 0]) < 1e-3 * d10[0, 0]
    assert np.abs(d10[:, 1:]).max() < 1e-6 * d10[0, 0]
    # |D|^-4
    d20, sa20 = _aligned_pair_displacement(oracle, g, g["a_over_ell"], 20.0, dphi)
    ratio = d10[0, 0] / d20[0, 0]
    assert 16 * 0.95 < ratio < 16 * 1.05, ratio
    # reversing the phase difference reverses the motion
    dneg, _ = _aligned_pair_displacement(oracle, g, g["a_over_ell"], 10.0, -dphi)
    assert dneg[0, 0] < 0 and abs(dneg[0, 0] + d10[0, 0]) < 0.05 * d10[0, 0]
    # Fig. 1(c): microscopic / stroke-averaged -> 1 as a/ell -> 0
    ratios = []
    for al in (0.2, 0.1, 0.05, 0.02):
        d, sa = _aligned_pair_displacement(oracle, g, al, 10.0, dphi)
        ratios.append(d[0, 0] / sa)
    dev = np.abs(np.array(ratios) - 1)
    assert np.all(np.diff(dev) < 0), ratios
    assert dev[-1] < 0.06, ratios
    assert dev[0] < 0.5, ratios


def test_aligned_pair_in_phase_does_not_swim(oracle, golden_dir):
    """Eq. (e:stroke_averaged): sin(0) = 0 -- equal phases give no collective
    motion; by mirror symmetry the mean position is exactly fixed."""
    g = json.loads((golden_dir / "fig1_aligned_pair.json").read_text())
    d, sa = _aligned_pair_displacement(oracle, g, g["a_over_ell"], 10.0, 0.0)
    assert abs(d[0, 0] + d[1, 0]) < 1e-6 * sa


def test_library_call_names_are_the_same_functions(oracle):
    """adref_mobility_apply and adref_step, the oracle's entries under the
    library's call names, give the bits of adref_mobility and of adref_run
    without records."""
    import ctypes as C
    L = oracle.lib()
    sus = make_single(12, 40.0, 4)
    p = C.byref(oracle._params(sus.params))
    X = np.ascontiguousarray(sus.X, dtype=np.float64)
    F = oracle.forces(sus.params, X, sus.phi, 0.7)
    u = oracle.mobility(sus.params, X, F)
    u2 = np.zeros_like(u)
    assert L.adref_mobility_apply(p, X.shape[0], oracle._d(X), oracle._d(F), oracle._d(u2)) == 0
    assert np.array_equal(u, u2)
    Xr, _, _, _ = oracle.run(sus.params, X, sus.phi, 25, t0=0.3, step0=7)
    Xs = X.copy()
    off = np.array([0, X.shape[0]], dtype=np.int64)
    assert L.adref_step(p, 1, off.ctypes.data_as(C.POINTER(C.c_int64)), oracle._d(Xs), oracle._d(sus.phi), 0.3,
                        7, 25) == 0
    assert np.array_equal(Xr, Xs)
