"""Pins of the oracle's stroke-averaged far-field equations (Sec. III,
Eqs. e:eom, J, K) against the paper: the 1d aligned-pair law it prints
separately (Eq. e:stroke_averaged), the symmetries and decay laws stated
after Eq. K, head-tail symmetry of symmetric dumbbells, and the microscopic
dynamics of the same pair (Sec. IV compares the two)."""
import json
import math

import numpy as np
import pytest

from workload import Params, place_dumbbells

PI = math.pi


def unit(v):
    v = np.asarray(v, dtype=float)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def rand_config(seed, S=6, spread=60.0):
    rng = np.random.default_rng(seed)
    return (rng.uniform(-spread, spread, (S, 3)), unit(rng.standard_normal((S, 3))),
            rng.uniform(0, 2 * PI, S))


def test_aligned_pair_reduces_to_the_1d_law(oracle, golden_dir):
    """Eq. (J) with N_s = N_r = +-Dhat (s, r, q = +-1) gives Eq.
    (e:stroke_averaged): (9/16) a w sin(phi_s - phi_r) (lam/ell)^2 (ell/D)^4 Dhat."""
    g = json.loads((golden_dir / "fig1_aligned_pair.json").read_text())
    p = Params(a=1.0, ell=4.0, lam=1.0, T=100.0)
    w = 2 * PI / p.T
    for D in (20.0, 37.5):
        for n1, n2 in (([1, 0, 0], [1, 0, 0]), ([-1, 0, 0], [1, 0, 0]), ([-1, 0, 0], [-1, 0, 0])):
            R = np.array([[0.0, 0, 0], [D, 0, 0]])
            N = np.array([n1, n2], dtype=float)
            phi = np.array([0.2, 1.3])
            dR, dN = oracle.sa_rhs(p, R, N, phi)
            law = g["far_field_prefactor"] * p.a * w * (p.lam / p.ell) ** 2 * (p.ell / D) ** 4
            # dumbbell 0: Dhat = R0 - R1 = -x; dumbbell 1: Dhat = +x
            np.testing.assert_allclose(dR[0], law * math.sin(0.2 - 1.3) * np.array([-1, 0, 0]), rtol=1e-13,
                                       atol=1e-30)
            np.testing.assert_allclose(dR[1], law * math.sin(1.3 - 0.2) * np.array([1, 0, 0]), rtol=1e-13,
                                       atol=1e-30)
            assert np.abs(dN).max() == 0.0  # aligned: no rotation


def test_phase_locked_pairs_do_not_interact(oracle):
    """Sec. III: J and K vanish when the phases differ by a multiple of pi."""
    R, N, _ = rand_config(1)
    p = Params()
    dR0, dN0 = oracle.sa_rhs(p, R, N, np.random.default_rng(9).uniform(0, 2 * PI, len(R)))
    for base in (0.0, 1.1):
        for k in (0, 1, 2):
            phi = base + k * PI * np.array([0, 1, 0, 1, 1, 0])
            dR, dN = oracle.sa_rhs(p, R, N, phi)
            # sin(k pi) is zero only up to the rounding of k pi
            assert np.abs(dR).max() < 1e-14 * np.abs(dR0).max()
            assert np.abs(dN).max() < 1e-14 * np.abs(dN0).max()


def test_decay_laws(oracle):
    """Sec. III: translation ~ |D|^-4, rotation ~ |D|^-5."""
    p = Params()
    N = unit(np.array([[1.0, 2.0, 0.5], [-0.3, 1.0, 2.0]]))
    phi = np.array([0.0, 0.9])
    e = unit([0.3, -0.5, 0.8])
    out = []
    for D in (30.0, 60.0):
        dR, dN = oracle.sa_rhs(p, np.array([[0.0, 0, 0], D * e]), N, phi)
        out.append((dR[0], dN[0]))
    np.testing.assert_allclose(out[0][0] / out[1][0], 16.0, rtol=1e-12)
    np.testing.assert_allclose(out[0][1] / out[1][1], 32.0, rtol=1e-12)


def test_head_tail_symmetry_and_unit_axes(oracle):
    """Symmetric dumbbells have no head: flipping any axis leaves dR/dt
    unchanged and flips that axis' dN/dt; dN/dt is orthogonal to N."""
    R, N, phi = rand_config(2)
    p = Params()
    dR, dN = oracle.sa_rhs(p, R, N, phi)
    assert np.abs(np.einsum("ij,ij->i", dN, N)).max() < 1e-12 * np.abs(dN).max()
    for k in range(len(N)):
        Nf = N.copy()
        Nf[k] = -Nf[k]
        dR2, dN2 = oracle.sa_rhs(p, R, Nf, phi)
        np.testing.assert_allclose(dR2, dR, rtol=1e-12, atol=1e-14 * np.abs(dR).max())
        sign = np.ones(len(N))
        sign[k] = -1
        np.testing.assert_allclose(dN2, dN * sign[:, None], rtol=1e-12, atol=1e-14 * np.abs(dN).max())


def test_translation_and_rotation(oracle):
    R, N, phi = rand_config(3)
    p = Params()
    dR, dN = oracle.sa_rhs(p, R, N, phi)
    dR2, dN2 = oracle.sa_rhs(p, R + np.array([5.0, -7.0, 2.5]), N, phi)
    np.testing.assert_allclose(dR2, dR, rtol=1e-12, atol=1e-15 * np.abs(dR).max())
    q, r = np.linalg.qr(np.random.default_rng(4).standard_normal((3, 3)))
    Q = q * np.sign(np.diag(r))
    dR3, dN3 = oracle.sa_rhs(p, R @ Q.T, N @ Q.T, phi)
    np.testing.assert_allclose(dR3, dR @ Q.T, rtol=1e-11, atol=1e-13 * np.abs(dR).max())
    np.testing.assert_allclose(dN3, dN @ Q.T, rtol=1e-11, atol=1e-13 * np.abs(dN).max())


def test_rk4_keeps_unit_axes_and_converges(oracle):
    """Fast strokes (T = 2, lam = 2) in a tight cluster, so the averaged
    dynamics move the dumbbells by about one length: RK4's error falls ~16x
    per halving of dt, and the axes stay unit vectors."""
    R, N, phi = rand_config(5, S=4, spread=8.0)
    p = Params(T=2.0, lam=2.0)
    tend = 100.0
    ref = oracle.sa_run(p, R, N, phi, tend / 6400, 6400)
    assert np.abs(ref[0] - R).max() > 1.0
    errs = []
    for n in (200, 400, 800):
        Rn, Nn = oracle.sa_run(p, R, N, phi, tend / n, n)
        np.testing.assert_allclose(np.linalg.norm(Nn, axis=1), 1.0, atol=1e-15)
        errs.append(np.abs(Rn - ref[0]).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 14) and np.all(ratios < 19), ratios


@pytest.mark.parametrize("a_over_ell,tol", [(0.05, 0.10), (0.02, 0.05)])
def test_microscopic_pair_follows_the_stroke_averaged_law(oracle, a_over_ell, tol):
    """Sec. IV: the stroke-averaged equations describe the microscopic
    dynamics of a pair at a few body lengths, better as a/ell -> 0. A 3d pair
    at random orientations, Fig. 1 parameters (ell = 5 um, w = 500/s,
    lam = 0.1 ell, stiff springs), distance 8 ell: the displacement of the
    centres over one stroke (after the settling period) matches J T in
    direction and, within tol, in length."""
    ell = 5e-6
    om = 500.0
    T = 2 * PI / om
    spp = 10000
    p = Params(a=a_over_ell * ell, eta=1e-3, k=1e-3, ell=ell, lam=0.1 * ell, T=T, dt=T / spp)
    rng = np.random.default_rng(0)
    n = unit(rng.standard_normal((2, 3)))
    dvec = unit(rng.standard_normal(3))
    R = np.array([[0.0, 0, 0], 8 * ell * dvec])
    phi = np.array([0.3, 0.3 + PI / 2])
    X = place_dumbbells(R, n, phi, p)
    Xn, cen, _, _ = oracle.run(p, X, phi, 2 * spp, record_every=spp)
    disp = cen[1] - cen[0]
    axes = unit(Xn[1::2] - Xn[0::2])
    dR, _ = oracle.sa_rhs(p, cen[0], axes, phi)
    for k in range(2):
        cosang = disp[k] @ dR[k] / np.linalg.norm(disp[k]) / np.linalg.norm(dR[k])
        assert cosang > 0.999
        assert abs(np.linalg.norm(disp[k]) / np.linalg.norm(dR[k] * T) - 1) < tol
