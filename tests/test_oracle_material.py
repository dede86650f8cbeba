"""Pins of the oracle's fixed-corotated elasticity and Newtonian viscosity (the
paper's material model, Sec. III-B; reading R31) against the mathematics: the polar
decomposition from an SVD (a library routine), zero stress at rotations,
objectivity and isotropy, the stress as the derivative of the energy, the small-
strain (Hooke) limit, closed-form viscous stresses."""
import numpy as np
import pytest

import oracle

E, NU = 2.0e4, 0.4
MU = E / (2 * (1 + NU))
LAM = E * NU / ((1 + NU) * (1 - 2 * NU))


def _rand_F(rng, s=0.3):
    while True:
        F = np.eye(3) + s * rng.normal(size=(3, 3))
        if np.linalg.det(F) > 0.2:
            return F


def _rand_rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_polar_matches_svd():
    rng = np.random.default_rng(1)
    for _ in range(50):
        F = _rand_F(rng)
        R, S = oracle.polar(F)
        U, s, Vt = np.linalg.svd(F)
        assert np.allclose(R, U @ Vt, atol=1e-12)
        assert np.allclose(S, Vt.T @ np.diag(s) @ Vt, atol=1e-12)


def test_fcr_zero_at_rotations():
    rng = np.random.default_rng(2)
    for _ in range(10):
        assert np.abs(oracle.fcr_P(E, NU, _rand_rot(rng))).max() < 1e-9 * E


def test_fcr_objectivity_and_isotropy():
    rng = np.random.default_rng(3)
    for _ in range(10):
        F, Q = _rand_F(rng), _rand_rot(rng)
        P = oracle.fcr_P(E, NU, F)
        assert np.allclose(oracle.fcr_P(E, NU, Q @ F), Q @ P, rtol=1e-10, atol=1e-8)
        assert np.allclose(oracle.fcr_P(E, NU, F @ Q), P @ Q, rtol=1e-10, atol=1e-8)


def test_fcr_stress_is_energy_gradient():
    rng = np.random.default_rng(4)
    for _ in range(5):
        F = _rand_F(rng)
        P = oracle.fcr_P(E, NU, F)
        h = 1e-6
        G = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                Fp, Fm = F.copy(), F.copy()
                Fp[i, j] += h
                Fm[i, j] -= h
                G[i, j] = (oracle.fcr_psi(E, NU, Fp) - oracle.fcr_psi(E, NU, Fm)) / (2 * h)
        assert np.allclose(P, G, rtol=1e-6, atol=1e-6 * E)


def test_fcr_small_strain_is_hooke():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(3, 3))
    eps = 1e-6 * (A + A.T)
    P = oracle.fcr_P(E, NU, np.eye(3) + eps)
    hooke = 2 * MU * eps + LAM * np.trace(eps) * np.eye(3)
    assert np.allclose(P, hooke, rtol=1e-4, atol=1e-9 * E)


def test_fcr_uniaxial_closed_form():
    """F = diag(a, 1, 1): R = I, P11 = 2 mu (a - 1) + lambda (a - 1), P22 = P33 =
    lambda (a - 1) a."""
    a = 1.2
    P = oracle.fcr_P(E, NU, np.diag([a, 1.0, 1.0]))
    assert np.allclose(np.diag(P), [2 * MU * (a - 1) + LAM * (a - 1), LAM * (a - 1) * a, LAM * (a - 1) * a],
                       rtol=1e-12)
    assert np.abs(P - np.diag(np.diag(P))).max() < 1e-9


def test_viscous_stress_closed_forms():
    eta, g = 3.0, 2.5
    # simple shear rate at F = I: sigma = eta (l + l^T)
    Fd = np.zeros((3, 3))
    Fd[0, 1] = g
    P = oracle.visc_P(eta, np.eye(3), Fd)
    expect = np.zeros((3, 3))
    expect[0, 1] = expect[1, 0] = eta * g
    assert np.allclose(P, expect, atol=1e-12)
    # rigid rotation rate: Fdot = W F with W skew gives no viscous stress
    rng = np.random.default_rng(6)
    F = _rand_F(rng)
    W = np.array([[0.0, -0.3, 0.2], [0.3, 0.0, -0.7], [-0.2, 0.7, 0.0]])
    assert np.abs(oracle.visc_P(eta, F, W @ F)).max() < 1e-10
    # general: P = J sigma F^-T with sigma = eta (l + l^T), l = Fdot F^-1
    Fd = rng.normal(size=(3, 3))
    l = Fd @ np.linalg.inv(F)
    sig = eta * (l + l.T)
    assert np.allclose(oracle.visc_P(eta, F, Fd), np.linalg.det(F) * sig @ np.linalg.inv(F).T, rtol=1e-10)


def test_fcr_scene_uniform_translation_and_rest():
    """A free body in fixed-corotated elasticity with viscosity at rest and without
    gravity stays at rest; moving uniformly it translates without strain."""
    from paper_2609_27342_amd import workloads as W
    sc = W.box_scene(n_cells=(3, 3, 3), dx=0.01, E=E, nu=NU, v0=(0.3, -0.1, 0.2))
    sc["params"].update(material=1, viscosity=0.5, floor_on=0, gravity=[0.0, 0.0, 0.0])
    o = oracle.OracleScene(sc)
    x0 = o.get()["x"].copy()
    for _ in range(5):
        assert o.step([])[0] == 0
    st = o.get()
    assert np.allclose(st["v"], [0.3, -0.1, 0.2], atol=1e-12)
    assert np.allclose(st["x"] - x0, 5 * 1e-4 * np.array([0.3, -0.1, 0.2]), atol=1e-12)
    assert np.allclose(st["F"], np.eye(3), atol=1e-12)
