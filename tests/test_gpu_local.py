"""Group local expansions on the device (the fast multipole method's M2L and
L2P steps at the level of the target groups, with quadrupole cells) against
the oracle.

The walk's decisions are FP64 expressions of the definitions, so the
per-group list sizes must equal the oracle's exactly. Forces are FP32 (the
ten expansion coefficients are summed per lane and then over the wave) and
are held to the tree-code bars against the oracle's FP64 evaluation of the
same lists."""
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


def _own_leaves(orc, n, leaf):
    """Leaves inside each group (the oracle lists them as near; the device
    sums them as the group's own range)."""
    nodes = orc.tree_nodes(n, leaf)
    L = orc.tree_lists(np.zeros((n, 4)) + np.arange(n)[:, None] * 1e-3, leaf, 64, 0.0)
    leaves = nodes[nodes[:, 2] < 0]
    out = []
    for gid in L["group_id"]:
        gb, ge = nodes[gid, :2]
        out.append(int(np.sum((leaves[:, 0] >= gb) & (leaves[:, 1] <= ge))))
    return np.array(out)


@pytest.mark.parametrize("n,leaf,theta,kind", [
    (3000, 8, 0.5, "plummer"), (3000, 4, 0.7, "plummer"), (20000, 4, 0.7, "collide"),
    (20000, 4, 0.4, "ball"), (9000, 16, 1.0, "plummer"), (776, 1, 0.8, "collide"), (5000, 8, 0.0, "ball"),
    (70001, 4, 0.6, "plummer")])
def test_counts_match_oracle(orc, n, leaf, theta, kind):
    torch, nb = gpu()
    gen = {"plummer": ics.plummer, "collide": ics.colliding_pair, "ball": ics.uniform_ball}[kind]
    pm, _ = gen(n, 600 + n)
    q, qh = _orb_input(torch, nb, pm, leaf)
    lc, fc, ncnt = (host(t).astype(np.int64) for t in nb.tree_local_counts(q, theta, leaf))
    want = orc.tree_local_counts(qh, leaf, 64, theta)
    assert np.array_equal(lc, want["loc_cnt"])
    assert np.array_equal(fc, want["far_cnt"])
    assert np.array_equal(ncnt, want["near_cnt"] - _own_leaves(orc, n, leaf))
    if theta == 0.0:
        assert lc.sum() == 0 and fc.sum() == 0


@pytest.mark.parametrize("prec,tol_rms,tol_max", [("F32_F64ACC", 1e-6, 2e-5), ("F32_KAHAN", 1e-6, 2e-5),
                                                  ("F32", 2e-6, 1e-4)])
@pytest.mark.parametrize("theta", [0.0, 0.5, 0.7])
def test_force_matches_oracle(orc, prec, tol_rms, tol_max, theta):
    torch, nb = gpu()
    n, leaf, eps = 12000, 4, 0.01
    pm, _ = ics.plummer(n, 610)
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_accel(q, eps, theta, leaf, prec=getattr(nb, prec), cells=nb.CELLS_LOCAL))
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps, cells=4)
    assert rms_rel(got[:, :3], a) < tol_rms
    assert max_rel(got[:, :3], a) < tol_max
    assert rms_rel(got[:, 3], p) < tol_rms


def test_accuracy_against_direct_and_the_other_cells(orc):
    """theta = 0 is the direct sum; at theta 0.5 and 0.7 the error against the
    exact sum is below the monopole cells' (measured 0.47x and 0.57x)."""
    torch, nb = gpu()
    n, leaf, eps = 20000, 4, 0.005
    pm, _ = ics.colliding_pair(n, 620)
    q, qh = _orb_input(torch, nb, pm, leaf)
    ad, pd = orc.accel(widen32(qh), eps)
    t0 = host(nb.tree_accel(q, eps, 0.0, leaf, prec=nb.F32_F64ACC, cells=nb.CELLS_LOCAL))
    assert rms_rel(t0[:, :3], ad) < 1e-6 and rms_rel(t0[:, 3], pd) < 1e-6
    for theta in (0.5, 0.7):
        e = {}
        for cells in (nb.CELLS_MONOPOLE, nb.CELLS_QUADRUPOLE, nb.CELLS_LOCAL):
            t = host(nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, cells=cells))
            e[cells] = rms_rel(t[:, :3], ad)
        print(f"theta {theta}: rms error vs direct: monopole {e[0]:.3e}, quadrupole {e[3]:.3e}, local {e[4]:.3e}")
        # quadrupole cells with a third-order group expansion: below the
        # monopole cells; the local test admits a combined size-to-distance
        # ratio of up to sqrt(2) theta, so at equal theta the error lies above
        # the quadrupole cells' (measured 3.8x at theta 0.5, 3.2x at 0.7)
        assert e[4] < 0.7 * e[0]


@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 65, 129, 1000])
def test_small_and_ragged(orc, n):
    torch, nb = gpu()
    pm, _ = ics.uniform_ball(max(n, 2), 630 + n)
    pm = pm[:n].copy()
    pm[:, 3] = 1.0 / n
    q, qh = _orb_input(torch, nb, pm, 4)
    got = host(nb.tree_accel(q, 0.05, 0.7, 4, prec=nb.F32_F64ACC, cells=nb.CELLS_LOCAL))
    if n == 1:
        assert np.all(got == 0.0)
        return
    a, p = orc.tree_accel(widen32(qh), 4, 64, 0.7, 0.05, cells=4)
    assert rms_rel(got[:, :3], a) < 1e-6
    assert rms_rel(got[:, 3], p) < 1e-6


def test_massless_bodies_and_eps_zero(orc):
    torch, nb = gpu()
    n = 6000
    pm, _ = ics.plummer(n, 640)
    pm = pm.copy()
    pm[::4, 3] = 0.0
    pm[pm[:, 0] < -0.5, 3] = 0.0  # whole cells without mass
    q, qh = _orb_input(torch, nb, pm, 4)
    got = host(nb.tree_accel(q, 0.0, 0.6, 4, prec=nb.F32_F64ACC, cells=nb.CELLS_LOCAL))
    a, p = orc.tree_accel(widen32(qh), 4, 64, 0.6, 0.0, cells=4)
    assert np.isfinite(got).all()
    assert rms_rel(got[:, :3], a) < 1e-6


def test_large_sampled(orc):
    """N = 2^20 colliding pair at theta 0.7, leaf 4: sampled targets against
    the oracle, and the truncation against the exact sum for the record."""
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    n, eps, leaf, theta = w["n"], w["eps"], 4, 0.7
    pm, _ = ics.colliding_pair(n, w["seed"])
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, cells=nb.CELLS_LOCAL))
    tg = np.random.default_rng(10).choice(n, 256, replace=False)
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps, targets=tg, cells=4)
    assert rms_rel(got[tg, :3], a) < 1e-6
    assert rms_rel(got[tg, 3], p) < 1e-6
    ad, _ = orc.accel(widen32(qh), eps, targets=tg)
    trunc = rms_rel(got[tg, :3], ad)
    print(f"local-expansion tree theta {theta}: rms relative error against the direct sum {trunc:.3e}")
    assert trunc < 0.03 * theta ** 3


def test_repeat_same_bits():
    torch, nb = gpu()
    pm, _ = ics.plummer(5000, 650)
    q, _ = _orb_input(torch, nb, pm, 4)
    r1 = host(nb.tree_accel(q, 0.01, 0.7, 4, cells=nb.CELLS_LOCAL))
    _ = host(nb.tree_accel(q, 0.01, 0.7, 4, cells=nb.CELLS_QUADRUPOLE))
    r2 = host(nb.tree_accel(q, 0.01, 0.7, 4, cells=nb.CELLS_LOCAL))
    assert np.array_equal(r1, r2)


def test_tree_leapfrog_local_cells(orc):
    torch, nb = gpu()
    n, leaf, theta, eps, dt = 3000, 4, 0.6, 0.01, 1e-3
    pm, v0 = ics.plummer(n, 660)
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    perm = nb.orb_order(p, leaf)
    q = nb.permute(p, perm)
    v = nb.permute(to_dev(torch, np.c_[v0[:, :3], np.zeros(n)].astype(np.float32), torch.float32), perm)
    a = nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, cells=nb.CELLS_LOCAL)
    h = 0.5 * dt
    for _ in range(3):
        xk, vk, ak = host(q), host(v), host(a)
        at, _ = orc.tree_accel(xk, leaf, 64, theta, eps, cells=4)
        assert rms_rel(ak[:, :3], at) < 1e-6
        nb.tree_leapfrog(q, v, a, eps, theta, dt, 1, leaf, acc_valid=True, prec=nb.F32_F64ACC,
                         cells=nb.CELLS_LOCAL)
        x1, v1, a1 = host(q), host(v), host(a)
        np.testing.assert_allclose(x1[:, :3], xk[:, :3] + dt * (vk[:, :3] + h * ak[:, :3]), rtol=0, atol=1e-6)
        np.testing.assert_allclose(v1[:, :3], vk[:, :3] + h * (ak[:, :3] + a1[:, :3]), rtol=0, atol=1e-6)


@pytest.mark.parametrize("cells", ["CELLS_PSEUDO", "CELLS_QUADRUPOLE", "CELLS_LOCAL"])
def test_higher_order_cells_replay_in_a_captured_graph(cells):
    """After the first call for a shape, a tree force with any cell model is
    kernel launches only (moments, second moments, cell records, walk):
    captured in a HIP graph it replays bit for bit like eager calls, with
    eager work in between."""
    torch, nb = gpu()
    cm = getattr(nb, cells)
    pm, _ = ics.plummer(20000, 670)
    q, _ = _orb_input(torch, nb, pm, 4)
    out_e = nb.tree_accel(q, 0.01, 0.6, 4, prec=nb.F32_F64ACC, cells=cm)
    out_g = torch.empty_like(q)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        nb.tree_accel(q, 0.01, 0.6, 4, prec=nb.F32_F64ACC, out=out_g, cells=cm)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        nb.tree_accel(q, 0.01, 0.6, 4, prec=nb.F32_F64ACC, out=out_g, cells=cm)
    for rep in range(3):
        out_g.zero_()
        graph.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()
        ref = nb.tree_accel(q, 0.01, 0.6, 4, prec=nb.F32_F64ACC, cells=cm)
        torch.cuda.synchronize()
        assert torch.equal(out_g, ref) and torch.equal(ref, out_e), rep
        del junk
