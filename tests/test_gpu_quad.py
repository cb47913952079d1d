"""Quadrupole tree cells on the device (the expansion of the paper's
reference [20] through l = 2, evaluated directly) against the oracle.

The device forms Q = 3 S - trace(S) I from FP64 second moments built
bottom-up (parallel-axis rule); the oracle sums Q over each cell's bodies.
Records agree to FP32 rounding; forces are FP32 arithmetic over the oracle's
lists, held to the tree-code bars (RMS 1e-6 relative in the compensated
modes)."""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, max_rel, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu


def _orb_input(torch, nb, pm, leaf):
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    perm = nb.orb_order(p, leaf)
    q = nb.permute(p, perm)
    torch.cuda.synchronize()
    return q, q.cpu().numpy()


@pytest.mark.parametrize("n,leaf,kind", [(1, 1, "plummer"), (9, 8, "plummer"), (1000, 4, "plummer"),
                                         (4099, 8, "plummer"), (20001, 16, "ball"), (70001, 4, "collide")])
def test_quad_records_match_oracle(orc, n, leaf, kind):
    torch, nb = gpu()
    if kind == "plummer":
        pm, _ = ics.plummer(max(n, 2), 500 + n)
    elif kind == "ball":
        pm, _ = ics.uniform_ball(n, 501)
    else:
        pm, _ = ics.colliding_pair(n + 3, 502)
    pm = pm[:n]
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_quad(q, leaf))
    mo = orc.tree_moments(qh, leaf)
    Q = orc.tree_quad(widen32(qh), leaf)
    assert got.shape == (Q.shape[0], 3, 4)
    np.testing.assert_array_equal(got[:, 0, :3], mo["com"].astype(np.float32).astype(np.float64))
    np.testing.assert_array_equal(got[:, 0, 3], mo["mass"].astype(np.float32).astype(np.float64))
    gq = np.c_[got[:, 1, :], got[:, 2, :2]]          # Qxx, Qyy, Qzz, Qxy, Qxz, Qyz
    scale = np.abs(Q).max(axis=1, keepdims=True)
    assert np.all(np.abs(gq - Q) <= 2.0 ** -22 * scale + 1e-300)
    assert np.all(got[:, 2, 2:] == 0)


@pytest.mark.parametrize("prec,tol_rms,tol_max", [("F32_F64ACC", 1e-6, 2e-5), ("F32_KAHAN", 1e-6, 2e-5),
                                                  ("F32", 2e-6, 1e-4)])
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_force_matches_oracle(orc, prec, tol_rms, tol_max, theta):
    torch, nb = gpu()
    n, leaf, eps = 12000, 4, 0.01
    pm, _ = ics.plummer(n, 510)
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_accel(q, eps, theta, leaf, prec=getattr(nb, prec), cells=nb.CELLS_QUADRUPOLE))
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps, cells=3)
    assert rms_rel(got[:, :3], a) < tol_rms
    assert max_rel(got[:, :3], a) < tol_max
    assert rms_rel(got[:, 3], p) < tol_rms


def test_accuracy_against_direct_and_the_other_cells(orc):
    """theta = 0 is the direct sum; at theta 0.5, 0.7, 1.0 the error against the
    exact sum is within a factor 2 of the pseudo-particle cells' and below half
    the monopole cells'."""
    torch, nb = gpu()
    n, leaf, eps = 9000, 4, 0.005
    pm, _ = ics.colliding_pair(n, 520)
    q, qh = _orb_input(torch, nb, pm, leaf)
    ad, pd = orc.accel(widen32(qh), eps)
    t0 = host(nb.tree_accel(q, eps, 0.0, leaf, prec=nb.F32_F64ACC, cells=nb.CELLS_QUADRUPOLE))
    assert rms_rel(t0[:, :3], ad) < 1e-6 and rms_rel(t0[:, 3], pd) < 1e-6
    for theta in (0.5, 0.7, 1.0):
        e = {}
        for cells in (nb.CELLS_MONOPOLE, nb.CELLS_PSEUDO, nb.CELLS_QUADRUPOLE):
            t = host(nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, cells=cells))
            e[cells] = rms_rel(t[:, :3], ad)
        print(f"theta {theta}: rms error vs direct: monopole {e[0]:.3e}, pseudo {e[2]:.3e}, quadrupole {e[3]:.3e}")
        assert e[3] < e[0] / 2
        assert 0.5 < e[3] / e[2] < 2.0


@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 65, 129, 1000])
def test_small_and_ragged(orc, n):
    torch, nb = gpu()
    pm, _ = ics.uniform_ball(max(n, 2), 530 + n)
    pm = pm[:n].copy()
    pm[:, 3] = 1.0 / n
    q, qh = _orb_input(torch, nb, pm, 4)
    got = host(nb.tree_accel(q, 0.05, 0.8, 4, prec=nb.F32_F64ACC, cells=nb.CELLS_QUADRUPOLE))
    if n == 1:
        assert np.all(got == 0.0)
        return
    a, p = orc.tree_accel(widen32(qh), 4, 64, 0.8, 0.05, cells=3)
    assert rms_rel(got[:, :3], a) < 1e-6
    assert rms_rel(got[:, 3], p) < 1e-6


def test_massless_bodies_and_eps_zero(orc):
    torch, nb = gpu()
    n = 6000
    pm, _ = ics.plummer(n, 540)
    pm = pm.copy()
    pm[::4, 3] = 0.0
    pm[pm[:, 0] < -0.5, 3] = 0.0  # whole cells without mass
    q, qh = _orb_input(torch, nb, pm, 4)
    got = host(nb.tree_accel(q, 0.0, 0.6, 4, prec=nb.F32_F64ACC, cells=nb.CELLS_QUADRUPOLE))
    a, p = orc.tree_accel(widen32(qh), 4, 64, 0.6, 0.0, cells=3)
    assert np.isfinite(got).all()
    assert rms_rel(got[:, :3], a) < 1e-6


def test_large_sampled(orc):
    """N = 2^20 colliding pair at theta 0.7, leaf 4 (the benchmark's launch):
    sampled targets against the oracle, and the truncation for the record."""
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    n, eps, leaf, theta = w["n"], w["eps"], 4, 0.7
    pm, _ = ics.colliding_pair(n, w["seed"])
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, cells=nb.CELLS_QUADRUPOLE))
    tg = np.random.default_rng(9).choice(n, 256, replace=False)
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps, targets=tg, cells=3)
    assert rms_rel(got[tg, :3], a) < 1e-6
    assert rms_rel(got[tg, 3], p) < 1e-6
    ad, _ = orc.accel(widen32(qh), eps, targets=tg)
    trunc = rms_rel(got[tg, :3], ad)
    print(f"quadrupole tree theta {theta}: rms relative error against the direct sum {trunc:.3e}")
    assert trunc < 0.02 * theta ** 3


def test_cell_models_alternate_with_the_same_bits():
    torch, nb = gpu()
    pm, _ = ics.plummer(5000, 550)
    q, _ = _orb_input(torch, nb, pm, 4)
    models = (nb.CELLS_QUADRUPOLE, nb.CELLS_MONOPOLE, nb.CELLS_PSEUDO)
    first = [host(nb.tree_accel(q, 0.01, 0.7, 4, cells=c)) for c in models]
    again = [host(nb.tree_accel(q, 0.01, 0.7, 4, cells=c)) for c in models]
    for a, b in zip(first, again):
        assert np.array_equal(a, b)
    assert not np.array_equal(first[0], first[2])


def test_tree_leapfrog_quadrupole_cells(orc):
    """Three steps one at a time: each force is the oracle's quadrupole-cell
    tree force at the integrator's positions and each step is the KDK
    recurrence."""
    torch, nb = gpu()
    n, leaf, theta, eps, dt = 3000, 4, 0.6, 0.01, 1e-3
    pm, v0 = ics.plummer(n, 560)
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    perm = nb.orb_order(p, leaf)
    q = nb.permute(p, perm)
    v = nb.permute(to_dev(torch, np.c_[v0[:, :3], np.zeros(n)].astype(np.float32), torch.float32), perm)
    a = nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, cells=nb.CELLS_QUADRUPOLE)
    h = 0.5 * dt
    for _ in range(3):
        xk, vk, ak = host(q), host(v), host(a)
        at, _ = orc.tree_accel(xk, leaf, 64, theta, eps, cells=3)
        assert rms_rel(ak[:, :3], at) < 1e-6
        nb.tree_leapfrog(q, v, a, eps, theta, dt, 1, leaf, acc_valid=True, prec=nb.F32_F64ACC,
                         cells=nb.CELLS_QUADRUPOLE)
        x1, v1, a1 = host(q), host(v), host(a)
        np.testing.assert_allclose(x1[:, :3], xk[:, :3] + dt * (vk[:, :3] + h * ak[:, :3]), rtol=0, atol=1e-6)
        np.testing.assert_allclose(v1[:, :3], vk[:, :3] + h * (ak[:, :3] + a1[:, :3]), rtol=0, atol=1e-6)
