"""The multi-level FMM on the device (nbody_fmm_accel, nbody_fmm_lists)
against the oracle's FMM (Section VI's O(N) method).

The traversal's decisions are the FP64 expressions of the definitions, so
every node's M2L, M2P and P2P lists equal the oracle's as sets (the device
walk visits them in its own fixed order).  Forces are FP32 (M2L sums, M2P
cells and P2P pairs in FP32, L2L and L2P in FP64) and are held to the
tree-code bars against the oracle's FP64 evaluation of the same lists."""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, max_rel, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu

GEN = {"plummer": ics.plummer, "collide": ics.colliding_pair, "ball": ics.uniform_ball}


def _orb_input(torch, nb, pm, leaf):
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    q = nb.permute(p, nb.orb_order(p, leaf))
    torch.cuda.synchronize()
    return q, q.cpu().numpy()


def _per_node_sorted(ids, cnt):
    node = np.repeat(np.arange(cnt.shape[0]), cnt)
    return ids[np.lexsort((ids, node))]


@pytest.mark.parametrize("n,leaf,theta,kind", [
    (1, 8, 0.5, "plummer"), (7, 8, 0.5, "plummer"), (300, 4, 0.6, "plummer"), (3000, 8, 0.5, "plummer"),
    (3000, 8, 0.0, "ball"), (5000, 5, 0.7, "collide"), (776, 1, 0.9, "collide"), (20000, 16, 0.5, "collide"),
    (9001, 12, 1.0, "plummer"), (4097, 64, 0.4, "ball"), (70001, 8, 0.6, "plummer"), (5000, 8, 5.0, "plummer")])
def test_lists_match_oracle(orc, n, leaf, theta, kind):
    torch, nb = gpu()
    pm, _ = GEN[kind](max(n, 4), 700 + n)
    q, qh = _orb_input(torch, nb, pm[:n], leaf)
    got = dict(zip(("m2l_cnt", "m2p_cnt", "p2p_cnt", "m2l", "m2p", "p2p"),
                   (host(t).astype(np.int64) for t in nb.fmm_lists(q, theta, leaf))))
    want = orc.fmm_lists(qh, leaf, theta)
    for kind in ("m2l", "m2p", "p2p"):
        c = got[kind + "_cnt"]
        assert np.array_equal(c, want[kind + "_cnt"]), kind
        # each node's entries as a set (the device walk visits them in its
        # own fixed order)
        assert np.array_equal(_per_node_sorted(got[kind], c),
                              _per_node_sorted(want[kind], want[kind + "_cnt"])), kind
    if theta == 0.0:
        assert got["m2l_cnt"].sum() == 0 and got["m2p_cnt"].sum() == 0


@pytest.mark.parametrize("n,leaf,theta,kind", [(262144, 8, 0.5, "collide"), (300001, 4, 0.6, "plummer")])
def test_lists_match_oracle_two_targets_per_wave(orc, n, leaf, theta, kind):
    """Depths of 32768 nodes or more are walked two target nodes per wave,
    two siblings (the union of their inherited sources, each tagged with the
    targets that need it): every node's lists still equal the oracle's as
    sets, and the forces on sampled targets match the oracle's FMM."""
    torch, nb = gpu()
    pm, _ = GEN[kind](n, 790 + n)
    q, qh = _orb_input(torch, nb, pm, leaf)
    nodes = nb.tree_shape(n, leaf, nodes=True)[2]
    depth = np.zeros(nodes.shape[0], dtype=np.int64)
    for a in range(nodes.shape[0]):  # preorder: parents first
        for ch in nodes[a, 2:]:
            if ch >= 0:
                depth[ch] = depth[a] + 1
    per_depth = np.bincount(depth)
    assert per_depth.max() >= 32768
    got = dict(zip(("m2l_cnt", "m2p_cnt", "p2p_cnt", "m2l", "m2p", "p2p"),
                   (host(t).astype(np.int64) for t in nb.fmm_lists(q, theta, leaf))))
    want = orc.fmm_lists(qh, leaf, theta)
    for k in ("m2l", "m2p", "p2p"):
        c = got[k + "_cnt"]
        assert np.array_equal(c, want[k + "_cnt"]), k
        assert np.array_equal(_per_node_sorted(got[k], c), _per_node_sorted(want[k], want[k + "_cnt"])), k
    out = host(nb.fmm_accel(q, 0.01, theta, leaf, prec=nb.F32_F64ACC))
    tg = ics.sample_targets(n, 128, 3)
    a, p = orc.fmm_accel(widen32(qh), leaf, theta, 0.01, targets=tg)
    assert rms_rel(out[tg, :3], a) < 1e-6
    assert rms_rel(out[tg, 3], p) < 1e-6


@pytest.mark.parametrize("prec,tol_rms,tol_max", [("F32_F64ACC", 1e-6, 2e-5), ("F32_KAHAN", 1e-6, 2e-5),
                                                  ("F32", 2e-6, 1e-4)])
@pytest.mark.parametrize("theta,leaf", [(0.0, 8), (0.5, 8), (0.7, 4), (0.6, 16)])
def test_force_matches_oracle(orc, prec, tol_rms, tol_max, theta, leaf):
    torch, nb = gpu()
    n, eps = 12000, 0.01
    pm, _ = ics.plummer(n, 710)
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.fmm_accel(q, eps, theta, leaf, prec=getattr(nb, prec)))
    a, p = orc.fmm_accel(widen32(qh), leaf, theta, eps)
    assert rms_rel(got[:, :3], a) < tol_rms
    assert max_rel(got[:, :3], a) < tol_max
    assert rms_rel(got[:, 3], p) < tol_rms


@pytest.mark.parametrize("n,leaf", [(1, 8), (2, 1), (5, 8), (64, 64), (65, 64), (1001, 3), (4096, 32)])
def test_edge_sizes(orc, n, leaf):
    """One body (no force), fewer bodies than a leaf, ragged last leaves,
    leaf sizes that are not powers of two, the largest leaf."""
    torch, nb = gpu()
    pm, _ = ics.uniform_ball(max(n, 2), 720 + n)
    q, qh = _orb_input(torch, nb, pm[:n], leaf)
    got = host(nb.fmm_accel(q, 0.01, 0.6, leaf, prec=nb.F32_F64ACC))
    if n == 1:
        assert np.all(got == 0)
        return
    a, p = orc.fmm_accel(widen32(qh), leaf, 0.6, 0.01)
    assert rms_rel(got[:, :3], a) < 1e-6
    assert rms_rel(got[:, 3], p) < 1e-6


def test_far_flung_leaf(orc):
    """A dense ball and 8 bodies strung far out along x: their leaf takes M2P
    cells rather than every leaf; lists and forces match the oracle."""
    torch, nb = gpu()
    g = np.random.default_rng(17)
    v = g.normal(size=(2000, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    ball = v * g.uniform(size=(2000, 1)) ** (1 / 3)
    line = np.column_stack([np.linspace(20, 60, 8), g.normal(0, 0.5, (8, 2))])
    x = np.vstack([ball, line])
    pm = np.hstack([x, g.uniform(0.5, 1.5, (x.shape[0], 1))]).astype(np.float32)
    q, qh = _orb_input(torch, nb, pm, 8)
    mc, cc, pc = (host(t).astype(np.int64) for t in nb.fmm_lists(q, 0.5, 8)[:3])
    want = orc.fmm_lists(qh, 8, 0.5)
    assert np.array_equal(cc, want["m2p_cnt"]) and np.array_equal(pc, want["p2p_cnt"])
    assert cc.sum() > 0
    got = host(nb.fmm_accel(q, 0.0, 0.5, 8, prec=nb.F32_F64ACC))
    a, p = orc.fmm_accel(widen32(qh), 8, 0.5, 0.0)
    assert rms_rel(got[:, :3], a) < 1e-6
    assert rms_rel(got[:, 3], p) < 1e-6


def test_theta_zero_is_the_direct_sum(orc):
    torch, nb = gpu()
    n = 3000
    pm, _ = ics.colliding_pair(n, 730)
    q, qh = _orb_input(torch, nb, pm, 8)
    got = host(nb.fmm_accel(q, 0.005, 0.0, 8, prec=nb.F32_F64ACC))
    a, p = orc.accel(widen32(qh), 0.005)
    assert rms_rel(got[:, :3], a) < 1e-6
    assert rms_rel(got[:, 3], p) < 1e-6


def test_repeat_calls_and_buffer_growth(orc):
    """A small call, then a much larger one (the list buffers grow), then the
    small one again: every result equals its first evaluation bit for bit."""
    torch, nb = gpu()
    outs = []
    for n in (2000, 60000, 2000):
        pm, _ = ics.plummer(n, 740 + n)
        q, _ = _orb_input(torch, nb, pm, 8)
        outs.append(nb.fmm_accel(q, 0.01, 0.3, 8).clone())
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[2])


def test_collide1m_sampled_against_oracle(orc):
    """The full-size colliding pair (2^20 bodies, leaf 8, theta 0.5): lists
    sizes equal the oracle's, sampled forces at FP32 tolerance; error
    against the exact sum reported."""
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    pm, _ = ics.colliding_pair(w["n"], w["seed"])
    q, qh = _orb_input(torch, nb, pm, 8)
    got = host(nb.fmm_accel(q, w["eps"], 0.5, 8, prec=nb.F32_F64ACC))
    tg = ics.sample_targets(w["n"], 256, w["seed"] + 3)
    a, p = orc.fmm_accel(widen32(qh), 8, 0.5, w["eps"], targets=tg)
    assert rms_rel(got[tg, :3], a) < 1e-6
    assert rms_rel(got[tg, 3], p) < 1e-6
    ad, _ = orc.accel(widen32(qh), w["eps"], targets=tg)
    print(f"fmm collide1m theta 0.5 leaf 8: vs oracle FMM {rms_rel(got[tg, :3], a):.2e}, "
          f"vs exact sum {rms_rel(got[tg, :3], ad):.2e}")


def test_coincident_bodies_and_g(orc):
    """Every body at one point: no expansion is ever used, forces are exactly
    zero and the potential is -G (M - m_i) / eps; G scales the result."""
    torch, nb = gpu()
    n, leaf = 200, 4
    pm = np.zeros((n, 4), dtype=np.float32)
    pm[:, :3] = [0.25, -1.5, 3.0]
    pm[:, 3] = np.linspace(0.5, 1.5, n)
    q, qh = _orb_input(torch, nb, pm, leaf)
    for theta in (0.5, 5.0):
        mc, cc, pc = (host(t) for t in nb.fmm_lists(q, theta, leaf)[:3])
        assert mc.sum() == 0 and cc.sum() == 0
        got = host(nb.fmm_accel(q, 0.1, theta, leaf, G=2.0, prec=nb.F32_F64ACC))
        assert np.all(got[:, :3] == 0)
        _, p = orc.fmm_accel(widen32(qh), leaf, theta, 0.1, G=2.0)
        assert rms_rel(got[:, 3], p) < 1e-6


def test_g_scales_the_result(orc):
    torch, nb = gpu()
    pm, _ = ics.plummer(6000, 760)
    q, qh = _orb_input(torch, nb, pm, 8)
    got = host(nb.fmm_accel(q, 0.01, 0.6, 8, G=2.5, prec=nb.F32_F64ACC))
    a, p = orc.fmm_accel(widen32(qh), 8, 0.6, 0.01, G=2.5)
    assert rms_rel(got[:, :3], a) < 1e-6
    assert rms_rel(got[:, 3], p) < 1e-6


@pytest.mark.parametrize("n", [20000, 262144])
def test_compact_lists_equal_the_slot_layout(orc, n):
    """With the slot layout's memory budget set to nothing, the traversal
    counts, scans and fills compact lists instead; the lists and the forces
    are the same, bit for bit (at 2^18 also with the deep depths walked two
    target nodes per wave)."""
    import os
    torch, nb = gpu()
    pm, _ = ics.plummer(n, 770)
    q, _ = _orb_input(torch, nb, pm, 8)
    nb.release()
    slot = nb.fmm_accel(q, 0.01, 0.5, 8, prec=nb.F32_F64ACC).clone()
    slot_lists = [t.clone() for t in nb.fmm_lists(q, 0.5, 8)]
    os.environ["NBODY_FMM_SLOT_MB"] = "0"
    try:
        nb.release()
        compact = nb.fmm_accel(q, 0.01, 0.5, 8, prec=nb.F32_F64ACC).clone()
        compact_lists = nb.fmm_lists(q, 0.5, 8)
    finally:
        del os.environ["NBODY_FMM_SLOT_MB"]
        nb.release()
    torch.cuda.synchronize()
    assert torch.equal(slot, compact)
    for a, b in zip(slot_lists, compact_lists):
        assert torch.equal(a, b)
