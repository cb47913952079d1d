"""Pins of the oracle's vector-Jacobian product of the direct sum and of its
trajectory gradient through the leapfrog, against central finite
differences of the (separately pinned) force and integrator, invariants and
closed forms."""
import numpy as np
import pytest

import ics


def _fd_dir(f, x, d, h):
    return (f(x + h * d) - f(x - h * d)) / (2 * h)


@pytest.mark.parametrize("with_phi", [False, True])
def test_vjp_vs_central_fd(orc, with_phi):
    n, eps = 256, 0.05
    p, _ = ics.plummer(n, 40)
    p[:, 3] *= np.linspace(0.5, 1.5, n)
    g = ics.rng(41)
    abar = g.standard_normal((n, 3))
    pbar = g.standard_normal(n) if with_phi else None
    xb, mb = orc.vjp(p, eps, abar, pbar)

    def scal(pm):
        a, ph = orc.accel(pm, eps)
        s = (a * abar).sum()
        if pbar is not None:
            s += (ph * pbar).sum()
        return s

    # random directions in positions and masses: <grad, d> = FD directional derivative
    for k in range(4):
        d = np.zeros((n, 4))
        d[:, :3] = g.standard_normal((n, 3))
        fd = _fd_dir(scal, p, d, 1e-6)
        an = (xb * d[:, :3]).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9
        dm = np.zeros((n, 4))
        dm[:, 3] = g.standard_normal(n)
        fd = _fd_dir(scal, p, dm, 1e-6)
        an = (mb * dm[:, 3]).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9
    # 32 single coordinates
    for k in range(32):
        i, c = int(g.integers(n)), int(g.integers(4))
        d = np.zeros((n, 4))
        d[i, c] = 1.0
        fd = _fd_dir(scal, p, d, 1e-6)
        an = xb[i, c] if c < 3 else mb[i]
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.abs(xb).max())


def test_vjp_invariants(orc):
    n, eps = 300, 0.02
    p, _ = ics.plummer(n, 42)
    p[:, 3] *= np.linspace(0.2, 2.0, n)
    g = ics.rng(43)
    abar = g.standard_normal((n, 3))
    pbar = g.standard_normal(n)
    xb, mb = orc.vjp(p, eps, abar, pbar)
    # translation invariance of a and phi: sum_k xbar_k = 0
    assert np.abs(xb.sum(axis=0)).max() <= 1e-12 * np.abs(xb).sum()
    # a and phi are homogeneous of degree one in the masses:
    # sum_k m_k mbar_k = sum_i abar_i . a_i + phibar_i phi_i
    a, ph = orc.accel(p, eps)
    lhs = (p[:, 3] * mb).sum()
    rhs = (abar * a).sum() + (pbar * ph).sum()
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(p[:, 3] * mb).sum())


def test_vjp_two_body_closed_form(orc):
    # two bodies, abar only on body 0 along x: a0 = m1 d w, d = x1 - x0
    # with eps = 0 and d = (2,0,0): w = 1/8, da0x/dx1 = m1 (w - 3 d^2 w / r^2) = m1 (1/8 - 3/8) = -m1/4
    p = np.array([[0.0, 0, 0, 1.0], [2.0, 0, 0, 3.0]])
    abar = np.array([[1.0, 0, 0], [0, 0, 0]])
    xb, mb = orc.vjp(p, 0.0, abar)
    np.testing.assert_allclose(xb[1], [-0.75, 0, 0], rtol=1e-15)
    np.testing.assert_allclose(xb[0], [0.75, 0, 0], rtol=1e-15)
    # da0x/dm1 = d_x w = 2/8; da1x/dm0 enters only through abar_1 = 0
    np.testing.assert_allclose(mb, [0.0, 0.25], rtol=1e-15, atol=0)


def test_traj_grad_vs_fd(orc):
    n, eps, dt, steps = 12, 0.1, 0.02, 15
    p, v = ics.plummer(n, 44)
    p[:, 3] *= np.linspace(0.5, 1.5, n)
    y = ics.perturbed_snapshot(p, 45, 0.1)
    L, gx, gv, gm = orc.traj_grad(p, v, y, eps, dt, steps)

    def loss(pm, vv):
        return float(((orc.leapfrog(pm, vv, eps, dt, steps)["x"] - y) ** 2).sum())

    assert abs(loss(p, v) - L) <= 1e-14 * L
    g = ics.rng(46)
    for k in range(6):
        dx = np.zeros((n, 4)); dx[:, :3] = g.standard_normal((n, 3))
        dv = np.zeros((n, 4)); dv[:, :3] = g.standard_normal((n, 3))
        dm = np.zeros((n, 4)); dm[:, 3] = g.standard_normal(n)
        h = 1e-6
        fdx = (loss(p + h * dx, v) - loss(p - h * dx, v)) / (2 * h)
        fdv = (loss(p, v + h * dv) - loss(p, v - h * dv)) / (2 * h)
        fdm = (loss(p + h * dm, v) - loss(p - h * dm, v)) / (2 * h)
        for fd, an in [(fdx, (gx * dx[:, :3]).sum()), (fdv, (gv * dv[:, :3]).sum()), (fdm, (gm * dm[:, 3]).sum())]:
            assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (fd, an)


def test_traj_grad_closed_forms(orc):
    p, v = ics.plummer(9, 47)
    y = ics.perturbed_snapshot(p, 48)
    # zero steps: L = |x0 - y|^2, dL/dx0 = 2 (x0 - y), no dependence on v0 or m
    L, gx, gv, gm = orc.traj_grad(p, v, y, 0.1, 0.01, 0)
    np.testing.assert_allclose(gx, 2 * (p[:, :3] - y), rtol=1e-15)
    assert np.all(gv == 0) and np.all(gm == 0)
    # G = 0: x(T) = x0 + T v0, dL/dv0 = 2 T (x(T) - y), dL/dm = 0
    T = 8 * 0.125
    L, gx, gv, gm = orc.traj_grad(p, v, y, 0.1, 0.125, 8, G=0.0)
    xT = p[:, :3] + T * v[:, :3]
    np.testing.assert_allclose(gx, 2 * (xT - y), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(gv, 2 * T * (xT - y), rtol=1e-13, atol=1e-13)
    assert np.all(gm == 0)


def _energy_T(orc, pm, vv, eps, dt, steps):
    """Total energy K + U of the final state of the FP64 leapfrog."""
    r = orc.leapfrog(pm, vv, eps, dt, steps)
    m = np.asarray(pm)[:, 3]
    return 0.5 * float((m * (r["v"] ** 2).sum(1)).sum()) + 0.5 * float((m * r["pot"]).sum()), r


def test_energy_gradient_vs_fd(orc):
    """Gradient of the final total energy E(T) = 1/2 sum m v^2 + 1/2 sum m phi
    through the leapfrog: cotangents vbar_T = m v_T and phibar_T = m / 2 on the
    final potential (the potential path of the reverse mode), plus the
    explicit mass terms 1/2 v^2 + 1/2 phi; checked against central finite
    differences of E(T)."""
    n, eps, dt, steps = 10, 0.1, 0.02, 12
    p, v = ics.plummer(n, 61)
    p[:, 3] *= np.linspace(0.5, 1.5, n)
    E, r = _energy_T(orc, p, v, eps, dt, steps)
    m = p[:, 3]
    gx, gv, gm = orc.traj_grad_cot(p, v, eps, dt, steps, np.zeros((n, 3)), m[:, None] * r["v"], 0.5 * m)
    gm = gm + 0.5 * (r["v"] ** 2).sum(1) + 0.5 * r["pot"]
    g = ics.rng(62)
    for k in range(5):
        dx = np.zeros((n, 4)); dx[:, :3] = g.standard_normal((n, 3))
        dv = np.zeros((n, 4)); dv[:, :3] = g.standard_normal((n, 3))
        dm = np.zeros((n, 4)); dm[:, 3] = g.standard_normal(n)
        h = 1e-6
        fdx = (_energy_T(orc, p + h * dx, v, eps, dt, steps)[0] - _energy_T(orc, p - h * dx, v, eps, dt, steps)[0]) / (2 * h)
        fdv = (_energy_T(orc, p, v + h * dv, eps, dt, steps)[0] - _energy_T(orc, p, v - h * dv, eps, dt, steps)[0]) / (2 * h)
        fdm = (_energy_T(orc, p + h * dm, v, eps, dt, steps)[0] - _energy_T(orc, p - h * dm, v, eps, dt, steps)[0]) / (2 * h)
        for fd, an in [(fdx, (gx * dx[:, :3]).sum()), (fdv, (gv * dv[:, :3]).sum()), (fdm, (gm * dm[:, 3]).sum())]:
            assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (fd, an)


def test_traj_grad_cot_reduces_to_position_loss(orc):
    """With xbar_T = 2 (x_T - y) and no other cotangent the general reverse
    mode gives the position-loss gradient bit for bit."""
    n, eps, dt, steps = 9, 0.1, 0.02, 7
    p, v = ics.plummer(n, 63)
    y = ics.perturbed_snapshot(p, 64, 0.1)
    L, gx, gv, gm = orc.traj_grad(p, v, y, eps, dt, steps)
    xT = orc.leapfrog(p, v, eps, dt, steps)["x"]
    hx, hv, hm = orc.traj_grad_cot(p, v, eps, dt, steps, 2.0 * (xT - y), np.zeros((n, 3)))
    assert np.array_equal(gx, hx) and np.array_equal(gv, hv) and np.array_equal(gm, hm)
