"""Order-2 tree cells on the device (the pseudo-particle multipole method of
Makino 1999, the paper's reference [20], cited in Section VI) against the
oracle.

The device builds each cell's 12 pseudo-particles from FP64 second moments
(parallel-axis rule, bottom-up); the oracle sums the method's mass formula
over the cell's bodies.  Positions are FP32 roundings of the same FP64 value
(within one FP32 unit); masses agree to FP32 rounding relative to the cell
mass.  Forces are FP32 pair arithmetic over the oracle's lists, held to the
tree-code bars (RMS 1e-6 relative in the compensated modes)."""
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
def test_pseudo_particles_match_oracle(orc, n, leaf, kind):
    torch, nb = gpu()
    if kind == "plummer":
        pm, _ = ics.plummer(max(n, 2), 400 + n)
    elif kind == "ball":
        pm, _ = ics.uniform_ball(n, 401)
    else:
        pm, _ = ics.colliding_pair(n + 3, 402)
    pm = pm[:n]
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_pseudo(q, leaf))
    want = orc.tree_pseudo(widen32(qh), leaf)
    assert got.shape == want.shape
    mo = orc.tree_moments(qh, leaf)
    # positions: FP32 of com + a s_j
    ulp = np.spacing(np.abs(want[:, :, :3]).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got[:, :, :3] - want[:, :, :3]) <= ulp)
    # masses: FP32 rounding relative to the cell's mass
    M = mo["mass"][:, None]
    err = np.abs(got[:, :, 3] - want[:, :, 3])
    assert np.all(err <= 2.0 ** -23 * (np.abs(want[:, :, 3]) + M / 12) + 1e-300)
    np.testing.assert_allclose(got[:, :, 3].astype(np.float64).sum(1), M[:, 0], rtol=1e-5)


@pytest.mark.parametrize("prec,tol_rms,tol_max", [("F32_F64ACC", 1e-6, 2e-5), ("F32_KAHAN", 1e-6, 2e-5),
                                                  ("F32", 2e-6, 1e-4)])
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_force_matches_oracle(orc, prec, tol_rms, tol_max, theta):
    torch, nb = gpu()
    n, leaf, eps = 12000, 4, 0.01
    pm, _ = ics.plummer(n, 410)
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_accel(q, eps, theta, leaf, prec=getattr(nb, prec), cells=nb.CELLS_PSEUDO))
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps, cells=2)
    assert rms_rel(got[:, :3], a) < tol_rms
    assert max_rel(got[:, :3], a) < tol_max
    assert rms_rel(got[:, 3], p) < tol_rms


def test_theta_zero_equals_direct_and_order_two_beats_monopole(orc):
    torch, nb = gpu()
    n, leaf, eps = 9000, 4, 0.005
    pm, _ = ics.colliding_pair(n, 420)
    q, qh = _orb_input(torch, nb, pm, leaf)
    ad, pd = orc.accel(widen32(qh), eps)
    t0 = host(nb.tree_accel(q, eps, 0.0, leaf, prec=nb.F32_F64ACC, cells=nb.CELLS_PSEUDO))
    assert rms_rel(t0[:, :3], ad) < 1e-6 and rms_rel(t0[:, 3], pd) < 1e-6
    for theta in (0.5, 0.7, 1.0):
        e = {}
        for order in (0, 2):
            t = host(nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, cells=order))
            e[order] = rms_rel(t[:, :3], ad)
        print(f"theta {theta}: rms error against the direct sum, monopole {e[0]:.3e}, order 2 {e[2]:.3e}")
        assert e[2] < e[0] / 2


@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 65, 129, 1000])
def test_small_and_ragged(orc, n):
    torch, nb = gpu()
    pm, _ = ics.uniform_ball(max(n, 2), 430 + n)
    pm = pm[:n].copy()
    pm[:, 3] = 1.0 / n
    q, qh = _orb_input(torch, nb, pm, 4)
    got = host(nb.tree_accel(q, 0.05, 0.8, 4, prec=nb.F32_F64ACC, cells=nb.CELLS_PSEUDO))
    if n == 1:
        assert np.all(got == 0.0)
        return
    a, p = orc.tree_accel(widen32(qh), 4, 64, 0.8, 0.05, cells=2)
    assert rms_rel(got[:, :3], a) < 1e-6
    assert rms_rel(got[:, 3], p) < 1e-6


def test_massless_bodies_and_eps_zero(orc):
    torch, nb = gpu()
    n = 6000
    pm, _ = ics.plummer(n, 440)
    pm = pm.copy()
    pm[::4, 3] = 0.0
    pm[pm[:, 0] < -0.5, 3] = 0.0  # whole cells without mass
    q, qh = _orb_input(torch, nb, pm, 4)
    got = host(nb.tree_accel(q, 0.0, 0.6, 4, prec=nb.F32_F64ACC, cells=nb.CELLS_PSEUDO))
    a, p = orc.tree_accel(widen32(qh), 4, 64, 0.6, 0.0, cells=2)
    assert np.isfinite(got).all()
    assert rms_rel(got[:, :3], a) < 1e-6


def test_large_sampled(orc):
    """N = 2^20 colliding pair at theta 0.7, leaf 4 (the benchmark's order-2
    launch): sampled targets against the oracle's order-2 tree force, and
    the truncation against the exact sum for the record."""
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    n, eps, leaf, theta = w["n"], w["eps"], 4, 0.7
    pm, _ = ics.colliding_pair(n, w["seed"])
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, cells=nb.CELLS_PSEUDO))
    tg = np.random.default_rng(8).choice(n, 256, replace=False)
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps, targets=tg, cells=2)
    assert rms_rel(got[tg, :3], a) < 1e-6
    assert rms_rel(got[tg, 3], p) < 1e-6
    ad, _ = orc.accel(widen32(qh), eps, targets=tg)
    trunc = rms_rel(got[tg, :3], ad)
    print(f"order-2 tree theta {theta}: rms relative error against the direct sum {trunc:.3e}")
    assert trunc < 0.02 * theta ** 3


def test_order_switch_and_repeat_same_bits():
    """Order 0 and order 2 share the tables: alternating them gives the same
    bits each time."""
    torch, nb = gpu()
    pm, _ = ics.plummer(5000, 450)
    q, _ = _orb_input(torch, nb, pm, 4)
    r2 = host(nb.tree_accel(q, 0.01, 0.7, 4, cells=nb.CELLS_PSEUDO))
    r0 = host(nb.tree_accel(q, 0.01, 0.7, 4, cells=0))
    assert np.array_equal(r2, host(nb.tree_accel(q, 0.01, 0.7, 4, cells=nb.CELLS_PSEUDO)))
    assert np.array_equal(r0, host(nb.tree_accel(q, 0.01, 0.7, 4, cells=0)))
    assert not np.array_equal(r0, r2)


def test_tree_leapfrog_order_two(orc):
    """Three steps one at a time: each force is the oracle's order-2 tree force
    at the integrator's positions and each step is the KDK recurrence."""
    torch, nb = gpu()
    n, leaf, theta, eps, dt = 3000, 4, 0.6, 0.01, 1e-3
    pm, v0 = ics.plummer(n, 460)
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    perm = nb.orb_order(p, leaf)
    q = nb.permute(p, perm)
    v = nb.permute(to_dev(torch, np.c_[v0[:, :3], np.zeros(n)].astype(np.float32), torch.float32), perm)
    a = nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, cells=2)
    h = 0.5 * dt
    for _ in range(3):
        xk, vk, ak = host(q), host(v), host(a)
        at, _ = orc.tree_accel(xk, leaf, 64, theta, eps, cells=2)
        assert rms_rel(ak[:, :3], at) < 1e-6
        nb.tree_leapfrog(q, v, a, eps, theta, dt, 1, leaf, acc_valid=True, prec=nb.F32_F64ACC, cells=2)
        x1, v1, a1 = host(q), host(v), host(a)
        np.testing.assert_allclose(x1[:, :3], xk[:, :3] + dt * (vk[:, :3] + h * ak[:, :3]), rtol=0, atol=1e-6)
        np.testing.assert_allclose(v1[:, :3], vk[:, :3] + h * (ak[:, :3] + a1[:, :3]), rtol=0, atol=1e-6)
