"""Tree code on the ORB cells (paper Section IV.A walk and monopole cells over
the Section IV.B ORB recursion) on the device against the oracle.

Moments and interaction lists are integer/decision work defined in FP64 with
a fixed operation order, so they must match the oracle bit for bit; forces
are FP32 pair arithmetic over the same lists and are held to an RMS relative
error of 1e-6 in the compensated modes (2e-6 in plain FP32), inside the 2e-6
bar of the direct-sum parity tests (the oracle evaluates the same lists in
FP64 with the cells at their exact FP64 centres of mass).
"""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, max_rel, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu


def _orb_input(torch, nb, pm, leaf):
    """Bodies gathered into the device ORB order (FP32), plus the host copy."""
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    perm = nb.orb_order(p, leaf)
    q = nb.permute(p, perm)
    torch.cuda.synchronize()
    return q, q.cpu().numpy()


@pytest.mark.parametrize("n,leaf", [(1, 1), (5, 8), (64, 8), (65, 8), (1000, 1), (3000, 8), (20001, 16),
                                    (50000, 4), (4096, 64)])
def test_moments_bitexact(orc, n, leaf):
    torch, nb = gpu()
    pm, _ = ics.plummer(max(n, 2), 300 + n)
    q, qh = _orb_input(torch, nb, pm[:n], leaf)
    mom, box = nb.tree_moments(q, leaf)
    torch.cuda.synchronize()
    mom, box = mom.cpu().numpy(), box.cpu().numpy()
    want = orc.tree_moments(qh, leaf)
    assert np.array_equal(mom[:, 0], want["mass"])
    assert np.array_equal(mom[:, 1:4], want["com"])
    assert np.array_equal(mom[:, 4], want["diag2"])
    assert np.array_equal(box[:, :3].astype(np.float64), want["lo"])
    assert np.array_equal(box[:, 3:].astype(np.float64), want["hi"])


def test_moments_zero_masses_and_repeat(orc):
    """Massless cells take the box centre; a second call on the same shape
    (counters reset by the first) gives the same bits."""
    torch, nb = gpu()
    pm, _ = ics.uniform_ball(4000, 310)
    pm = pm.copy()
    pm[::3, 3] = 0.0
    pm[pm[:, 0] < -0.4, 3] = 0.0  # a massless region: whole cells without mass
    q, qh = _orb_input(torch, nb, pm, 8)
    want = orc.tree_moments(qh, 8)
    for _ in range(2):
        mom, _ = nb.tree_moments(q, 8)
        torch.cuda.synchronize()
        mom = mom.cpu().numpy()
        assert np.array_equal(mom[:, 0], want["mass"])
        assert np.array_equal(mom[:, 1:4], want["com"])
    assert (want["mass"] == 0).any()


def _oracle_sets(orc, qh, leaf, theta):
    """Oracle lists per group, without the leaves inside the group (the
    device sums those as the group's own range)."""
    nodes = orc.tree_nodes(qh.shape[0], leaf)
    L = orc.tree_lists(qh, leaf, 64, theta)
    fo = np.r_[0, np.cumsum(L["far_cnt"])]
    no = np.r_[0, np.cumsum(L["near_cnt"])]
    far, near = [], []
    for g, gid in enumerate(L["group_id"]):
        gb, ge = nodes[gid, :2]
        far.append(set(L["far"][fo[g]:fo[g + 1]].tolist()))
        near.append({int(c) for c in L["near"][no[g]:no[g + 1]] if not (gb <= nodes[c, 0] and nodes[c, 1] <= ge)})
    return far, near


@pytest.mark.parametrize("n,leaf,theta,kind", [
    (3000, 8, 0.5, "plummer"), (3000, 8, 1.2, "plummer"), (20000, 8, 0.7, "collide"),
    (20000, 4, 0.4, "ball"), (9000, 16, 3.0, "plummer"), (776, 1, 0.8, "collide"), (5000, 8, 0.0, "ball")])
def test_lists_match_oracle(orc, n, leaf, theta, kind):
    torch, nb = gpu()
    gen = {"plummer": ics.plummer, "collide": ics.colliding_pair, "ball": ics.uniform_ball}[kind]
    pm, _ = gen(n, 320 + n)
    q, qh = _orb_input(torch, nb, pm, leaf)
    fc, ncnt, _, _ = nb.tree_lists(q, theta, leaf)
    torch.cuda.synchronize()
    mf, mn = int(fc.max().item()), int(ncnt.max().item())
    fc, ncnt, fi, ni = nb.tree_lists(q, theta, leaf, max(mf, 1), max(mn, 1))
    torch.cuda.synchronize()
    fc, ncnt, fi, ni = fc.cpu().numpy(), ncnt.cpu().numpy(), fi.cpu().numpy(), ni.cpu().numpy()
    far, near = _oracle_sets(orc, qh, leaf, theta)
    assert len(far) == fc.shape[0]
    for g in range(fc.shape[0]):
        assert fc[g] == len(far[g]) and ncnt[g] == len(near[g]), g
        assert set(fi[g, :fc[g]].tolist()) == far[g], g
        assert set(ni[g, :ncnt[g]].tolist()) == near[g], g
    if theta == 0.0:
        assert fc.sum() == 0


@pytest.mark.parametrize("prec,tol_rms,tol_max", [("F32_F64ACC", 1e-6, 2e-5), ("F32_KAHAN", 1e-6, 2e-5),
                                                  ("F32", 2e-6, 1e-4)])
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_force_matches_oracle(orc, prec, tol_rms, tol_max, theta):
    torch, nb = gpu()
    n, leaf, eps = 12000, 8, 0.01
    pm, _ = ics.plummer(n, 330)
    q, qh = _orb_input(torch, nb, pm, leaf)
    out = nb.tree_accel(q, eps, theta, leaf, prec=getattr(nb, prec))
    torch.cuda.synchronize()
    got = host(out)
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps)
    assert rms_rel(got[:, :3], a) < tol_rms
    assert max_rel(got[:, :3], a) < tol_max
    assert rms_rel(got[:, 3], p) < tol_rms


def test_theta_zero_equals_direct_sum(orc):
    """theta = 0 accepts no cell: the tree force is the exact direct sum."""
    torch, nb = gpu()
    n, leaf, eps = 9000, 8, 0.005
    pm, _ = ics.colliding_pair(n, 340)
    q, qh = _orb_input(torch, nb, pm, leaf)
    tr = host(nb.tree_accel(q, eps, 0.0, leaf, prec=nb.F32_F64ACC))
    di = host(nb.accel(q, eps, prec=nb.F32_F64ACC))
    ad, pd = orc.accel(widen32(qh), eps)
    assert rms_rel(tr[:, :3], ad) < 1e-6 and rms_rel(di[:, :3], ad) < 1e-6
    assert rms_rel(tr[:, :3], di[:, :3]) < 1e-6
    assert rms_rel(tr[:, 3], pd) < 1e-6


@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 65, 129, 1000])
def test_small_and_ragged(orc, n):
    torch, nb = gpu()
    pm, _ = ics.uniform_ball(max(n, 2), 350 + n)
    pm = pm[:n].copy()
    pm[:, 3] = 1.0 / n
    q, qh = _orb_input(torch, nb, pm, 4)
    got = host(nb.tree_accel(q, 0.05, 0.8, 4, prec=nb.F32_F64ACC))
    a, p = orc.tree_accel(widen32(qh), 4, 64, 0.8, 0.05)
    if n == 1:
        assert np.all(got == 0.0)
        return
    assert rms_rel(got[:, :3], a) < 1e-6
    assert rms_rel(got[:, 3], p) < 1e-6


def test_eps_zero_and_massless(orc):
    """eps = 0 with distinct positions and a share of massless bodies (test
    particles feel the field, exert none)."""
    torch, nb = gpu()
    n = 6000
    pm, _ = ics.plummer(n, 360)
    pm = pm.copy()
    pm[::4, 3] = 0.0
    q, qh = _orb_input(torch, nb, pm, 8)
    got = host(nb.tree_accel(q, 0.0, 0.6, 8, prec=nb.F32_F64ACC))
    a, p = orc.tree_accel(widen32(qh), 8, 64, 0.6, 0.0)
    assert np.isfinite(got).all()
    assert rms_rel(got[:, :3], a) < 1e-6


def test_large_sampled_and_error_against_direct(orc):
    """N = 2^20 colliding pair, the launch the benchmark times: sampled
    targets against the oracle's tree force, and the monopole truncation
    against the exact sum reported for the record."""
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    n, eps, leaf, theta = w["n"], w["eps"], 8, 0.7
    pm, _ = ics.colliding_pair(n, w["seed"])
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC))
    tg = np.random.default_rng(7).choice(n, 384, replace=False)
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps, targets=tg)
    assert rms_rel(got[tg, :3], a) < 1e-6
    assert rms_rel(got[tg, 3], p) < 1e-6
    ad, _ = orc.accel(widen32(qh), eps, targets=tg)
    trunc = rms_rel(got[tg, :3], ad)
    print(f"tree theta {theta}: rms relative error against the direct sum {trunc:.3e}")
    assert trunc < 0.1 * theta ** 2


def test_repeat_and_shape_change_same_bits():
    """Cached tables: the same call twice gives the same bits, also after a
    call of another shape in between."""
    torch, nb = gpu()
    pm, _ = ics.plummer(5000, 370)
    q, _ = _orb_input(torch, nb, pm, 8)
    pm2, _ = ics.plummer(3000, 371)
    q2, _ = _orb_input(torch, nb, pm2, 16)
    r1 = host(nb.tree_accel(q, 0.01, 0.7, 8))
    _ = host(nb.tree_accel(q2, 0.01, 0.7, 16))
    r2 = host(nb.tree_accel(q, 0.01, 0.7, 8))
    assert np.array_equal(r1, r2)
