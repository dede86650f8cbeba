"""Pins of the rigid-tool oracle (two-way coupling, reading R30) and the product's
host-side rigid step against it.

The oracle's integrator is checked against closed forms of its own scheme and
against invariants of rigid-body motion; its impulse response against the C
oracle's per-contact inverse effective mass (Sec. III-E, Eq. 15); the product's
tlmpm_rigid_step / tlmpm_rigid_tool (host code, no GPU) against the oracle.
"""
import math

import numpy as np
import pytest

import oracle
from oracle.rigid import Body, qrot
from paper_2609_27342_amd import workloads as W


def _rot(axis, ang):
    axis = np.asarray(axis, np.float64) / np.linalg.norm(axis)
    return np.concatenate(([math.cos(ang / 2)], math.sin(ang / 2) * axis))


def test_free_fall_discrete_closed_form():
    """Symplectic Euler under constant acceleration a: v_n = v0 + n h a,
    x_n = x0 + n h v0 + h^2 a n (n + 1) / 2."""
    g = np.array([0.3, -0.2, -9.81])
    F = np.array([0.05, 0.0, 0.1])
    b = Body([0.1, 0.2, 0.3], _rot([1, 2, 3], 0.7), [0.5, -0.1, 0.2], [0, 0, 0], 0.25, [1e-3, 2e-3, 3e-3])
    h, n = 1e-3, 250
    for _ in range(n):
        b.step(np.concatenate((F, np.zeros(3))), g, h)
    a = F / 0.25 + g
    assert np.allclose(b.v, [0.5, -0.1, 0.2] + n * h * a, rtol=0, atol=1e-12)
    assert np.allclose(b.x, np.array([0.1, 0.2, 0.3]) + n * h * np.array([0.5, -0.1, 0.2]) + h * h * a * n * (n + 1) / 2,
                       rtol=0, atol=1e-12)


def test_rotation_matrix_is_orthonormal_and_rotates_axis_angle():
    q = _rot([0, 0, 1], math.pi / 3)
    R = qrot(q)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-15)
    assert np.allclose(R @ [1, 0, 0], [0.5, math.sqrt(3) / 2, 0], atol=1e-15)


def test_constant_torque_about_principal_axis():
    """Spin about a principal axis under a torque along it: no gyroscopic term, so
    omega_n = omega_0 + n h tau / I exactly and the axis stays fixed."""
    I = np.array([1e-3, 2e-3, 3e-3])
    q0 = _rot([1, 1, 0], 0.4)
    R0 = qrot(q0)
    axis = R0 @ [0, 0, 1]
    b = Body([0, 0, 0], q0, [0, 0, 0], 2.0 * axis, 0.1, I)
    tau = 1e-3 * axis
    h, n = 1e-3, 400
    for _ in range(n):
        b.step(np.concatenate((np.zeros(3), tau)), [0, 0, 0], h)
    assert np.allclose(b.w, (2.0 + n * h * 1e-3 / 3e-3) * axis, rtol=1e-12, atol=1e-12)
    assert np.allclose(qrot(b.q) @ [0, 0, 1], axis, atol=1e-12)


def test_symmetric_top_keeps_spin_component():
    """Torque-free symmetric top (I1 = I2): Euler's third equation gives a constant
    body-axis spin omega_3."""
    b = Body([0, 0, 0], _rot([0.3, 1, 0.2], 0.9), [0, 0, 0], [0.4, -0.7, 2.0], 0.1, [2e-3, 2e-3, 1e-3])
    w3 = (qrot(b.q).T @ b.w)[2]
    for _ in range(500):
        b.step(np.zeros(6), [0, 0, 0], 1e-3)
    assert abs((qrot(b.q).T @ b.w)[2] - w3) < 1e-12


def test_torque_free_energy_and_momentum_drift_first_order():
    """Torque-free asymmetric body: kinetic energy and |L| are invariants of the
    motion; the scheme keeps them to first order in h (drift halves with h)."""
    def drift(h, T=0.5):
        b = Body([0, 0, 0], _rot([1, 0.2, 0.1], 0.3), [0, 0, 0], [1.0, 0.5, -0.8], 0.1, [1e-3, 2e-3, 3.5e-3])
        def inv(b):
            wb = qrot(b.q).T @ b.w
            return 0.5 * wb @ (b.I * wb), np.linalg.norm(b.I * wb)
        E0, L0 = inv(b)
        for _ in range(int(round(T / h))):
            b.step(np.zeros(6), [0, 0, 0], h)
        E1, L1 = inv(b)
        return abs(E1 - E0) / E0, abs(L1 - L0) / L0
    e1, l1 = drift(1e-3)
    e2, l2 = drift(5e-4)
    assert e1 < 1e-2 and l1 < 1e-2
    assert 1.6 < e1 / e2 < 2.4 and 1.6 < l1 / l2 < 2.4


def test_tool_blade_velocity_is_rigid_point_velocity():
    """The blade edge point of the tool record moves with v + omega x r: a short
    torque-free step moves it by h times that velocity to first order."""
    b = Body([0.01, -0.02, 0.05], _rot([0, 1, 0], 0.4), [0.1, 0.0, -0.3], [0.5, 2.0, -1.0], 0.1, [3e-5, 1e-4, 7e-5])
    blade = W.knife_blade_body(0.05, 0.03)
    t0 = b.tool(blade)
    h = 1e-7
    b.step(np.zeros(6), [0, 0, 0], h)
    t1 = b.tool(blade)
    fd = (t1["blade"]["x_e"] - t0["blade"]["x_e"]) / h
    assert np.allclose(fd, t0["blade"]["v_e"], rtol=1e-5, atol=1e-9)
    for k in ("n", "e", "d"):
        assert abs(np.linalg.norm(t0["blade"][k]) - 1.0) < 1e-14
    assert abs(t0["blade"]["n"] @ t0["blade"]["e"]) < 1e-14 and abs(t0["blade"]["e"] @ t0["blade"]["d"]) < 1e-14


def test_impulse_response_equals_inverse_effective_mass():
    """An impulse j n at a point p of a body at rest, applied as a wrench over one
    step, changes the normal velocity of p by j times the inverse effective mass."""
    b = Body([0.0, 0.0, 0.0], _rot([1, 2, 0.5], 1.1), [0, 0, 0], [0, 0, 0], 0.2, [1e-3, 4e-3, 2e-3])
    p = np.array([0.03, -0.01, 0.02])
    n = np.array([0.2, -0.5, 0.84])
    n = n / np.linalg.norm(n)
    w = b.inverse_effective_mass(p, n)
    j, h = 1e-3, 1e-4
    F = j / h * n
    x0 = b.x.copy()
    b.step(np.concatenate((F, np.cross(p - x0, F))), [0, 0, 0], h)
    # velocity change of the material point at p (from rest, no gyroscopic term)
    dvp = b.v + np.cross(b.w, p - x0)
    assert abs((dvp @ n) / j - w) < 1e-12 * w


def test_oracle_contact_uses_tool_inverse_effective_mass():
    """Sec. III-E, Eq. 15: a particle pressed against a free tool receives
    J_n = s_n m_eff / dt max(-phi_hat, 0) with m_eff = (1/m + w)^-1 and w the tool's
    inverse effective mass at the contact point along the normal."""
    p = W.base_params(0.01, (-0.05, -0.05, -0.05), (10, 10, 10), 1e-4, 0.3, floor_on=0, gravity=[0.0, 0.0, 0.0])
    V0 = np.float32(0.01 ** 3 / 8)
    m = float(np.float32(V0 * 1000))
    s = dict(params=p, X=np.array([[0.0025, 0.0025, 0.0025]], np.float32), v0=None, vol0=np.array([V0], np.float32),
             mass=np.array([m], np.float32), E=np.array([1e4], np.float32))
    o = oracle.OracleScene(s)
    R = 0.5 * float(V0) ** (1.0 / 3.0)
    body = Body([0.013, -0.007, 0.021], [1, 0, 0, 0], [0, 0, 0], [0, 0, 0], 0.05, [2e-6, 5e-6, 4e-6])
    # blade edge along x just above the particle (front direction -z), tool at rest
    b = W.blade(0, (0.0, 0.0, 0.0005 + R * 0.5), (0, 1, 0), (0, 0, -1), (0, 0, 0), 0.05, 0.03, 0.04, 0.01)
    T = dict(W.tool(b, labels=False, contact=True, cutting=False, x_B=body.x, v_B=(0, 0, 0)), contact=1, cutting=0,
             inv_mass=1.0 / body.M, inv_inertia=body.inv_inertia_world().reshape(9))
    xc = np.array([0.0, 0.0, 0.0005 + R * 0.5])
    nB = np.array([0.0, 0.0, -1.0])
    w = body.inverse_effective_mass(xc, nB)
    assert w > 1.5 / body.M  # the arm adds a rotational part
    vz = 3.0  # moving up into the edge
    o.set(x=np.zeros((1, 3)), v=np.array([[0.0, 0.0, vz]]))
    st, wr = o.step([T])
    dt = 1e-4
    gap = 0.0005 + 0.5 * R - R
    phihat = gap + dt * min(-vz, 0.0)
    meff = 1.0 / (1.0 / m + w)
    Jn = 0.5 * meff / dt * max(-phihat, 0.0)
    dv = o.get()["v"][0] - [0.0, 0.0, vz]
    assert Jn > 0
    assert np.allclose(m * dv, [0.0, 0.0, -Jn], rtol=1e-9, atol=1e-15)
    assert np.allclose(wr[0][:3] * dt, [0.0, 0.0, Jn], rtol=1e-9)


def test_product_rigid_step_matches_oracle():
    """tlmpm_rigid_step and tlmpm_rigid_tool (host code of the library) follow the
    oracle's scheme: the same trajectory under a varying wrench to rounding."""
    from paper_2609_27342_amd import tlmpm
    if not __import__("os").path.exists(tlmpm.LIB_PATH):
        pytest.skip("library not built")
    rng = np.random.default_rng(3)
    x0, q0, v0, w0 = [0.01, 0.02, 0.1], _rot([1, -1, 2], 0.8), [0.1, 0.0, -0.4], [1.0, -0.5, 0.3]
    M, I = 0.1, [8.4e-5, 2.1e-4, 1.3e-4]
    ob = Body(x0, q0, v0, w0, M, I)
    pb = tlmpm.RigidBody(x0, q0, v0, w0, M, I)
    blade = W.knife_blade_body(0.05, 0.03)
    g = [0.0, 0.0, -9.81]
    for k in range(300):
        wr = rng.normal(size=6) * [0.5, 0.5, 0.5, 0.01, 0.01, 0.01]
        ob.step(wr, g, 1e-3)
        pb.step(wr, g, 1e-3)
        if k % 50 == 0:
            to, tp = ob.tool(blade), pb.tool(blade)
            for key in ("x_e", "n", "e", "d", "v_e"):
                assert np.allclose(tp["blade"][key], to["blade"][key], rtol=1e-12, atol=1e-13), key
            assert np.allclose(tp["inv_inertia"], to["inv_inertia"], rtol=1e-11)
            assert abs(tp["inv_mass"] - 1.0 / M) < 1e-15
    st = pb.state()
    assert np.allclose(st["x"], ob.x, rtol=1e-12, atol=1e-14)
    assert np.allclose(st["v"], ob.v, rtol=1e-12, atol=1e-13)
    assert np.allclose(st["omega"], ob.w, rtol=1e-11, atol=1e-12)
    assert np.allclose(st["q"] * np.sign(st["q"][0]), ob.q * np.sign(ob.q[0]), rtol=1e-12, atol=1e-13)
