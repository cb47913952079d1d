"""Pins of the oracle's tree code (paper Section IV.A: a distant group of
bodies acts as one body of its total mass at its centre of mass, found by a
walk from the root; the cells are those of the Section IV.B ORB recursion).

Each check is independent of the oracle's own formulas: structural
invariants of the node table, moments against numpy reductions, the
partition of every interaction list, the geometric meaning of acceptance
checked body by body, theta = 0 against the direct sum, a two-body monopole
closed form on both sides of the acceptance threshold, and the error falling
with theta.
"""
import numpy as np
import pytest

import ics


def _orb(orc, pm, leaf):
    perm = orc.orb_order(pm, leaf)
    return np.ascontiguousarray(np.asarray(pm, dtype=np.float32)[perm])


@pytest.mark.parametrize("n,leaf", [(1, 1), (7, 8), (8, 8), (9, 8), (100, 8), (1000, 3), (4096, 16), (777, 64)])
def test_node_table_structure(orc, n, leaf):
    nodes = orc.tree_nodes(n, leaf)
    nleaves = -(-n // leaf)
    assert nodes.shape == (2 * nleaves - 1, 4)
    assert tuple(nodes[0, :2]) == (0, n)
    sizes = nodes[:, 1] - nodes[:, 0]
    is_leaf = nodes[:, 2] < 0
    assert np.all((nodes[:, 2] < 0) == (nodes[:, 3] < 0))
    # leaves: at most `leaf` bodies, all full except the last, aligned, in order
    lv = nodes[is_leaf]
    assert np.all(sizes[is_leaf] <= leaf) and np.all(sizes[is_leaf] >= 1)
    order = np.argsort(lv[:, 0])
    assert np.array_equal(lv[order, 0], np.arange(nleaves) * leaf)
    assert np.all(sizes[is_leaf][order][:-1] == leaf)
    # inner nodes: preorder (left child follows its parent), children tile the parent
    for k in np.nonzero(~is_leaf)[0]:
        b, e, l, r = nodes[k]
        assert l == k + 1 and r > l
        assert nodes[l, 0] == b and nodes[l, 1] == nodes[r, 0] and nodes[r, 1] == e
        # about equal halves (the left part rounded up to whole leaves)
        assert (nodes[l, 1] - nodes[l, 0]) % leaf == 0
        assert 0 <= (nodes[l, 1] - nodes[l, 0]) - (nodes[r, 1] - nodes[r, 0]) < 2 * leaf


def test_moments_against_numpy(orc):
    pm, _ = ics.plummer(3000, 11)
    q = _orb(orc, pm, 8)
    x = q[:, :3].astype(np.float64)
    m = q[:, 3].astype(np.float64)
    nodes = orc.tree_nodes(q.shape[0], 8)
    mo = orc.tree_moments(q, 8)
    for k in range(nodes.shape[0]):
        b, e = nodes[k, :2]
        M = m[b:e].sum()
        assert mo["mass"][k] == pytest.approx(M, rel=1e-14)
        np.testing.assert_allclose(mo["com"][k], (m[b:e, None] * x[b:e]).sum(0) / M, rtol=1e-12, atol=1e-15)
        assert np.array_equal(mo["lo"][k], x[b:e].min(0))
        assert np.array_equal(mo["hi"][k], x[b:e].max(0))
        assert mo["diag2"][k] == pytest.approx(((x[b:e].max(0) - x[b:e].min(0)) ** 2).sum(), rel=1e-14)


def test_zero_mass_cell_uses_box_centre(orc):
    pm = np.zeros((16, 4), dtype=np.float32)
    pm[:, 0] = np.arange(16, dtype=np.float32)
    pm[8:, 3] = 1.0  # first half massless
    q = _orb(orc, pm, 8)
    nodes = orc.tree_nodes(16, 8)
    mo = orc.tree_moments(q, 8)
    k = int(np.nonzero((nodes[:, 0] == 0) & (nodes[:, 1] == 8))[0][0])
    assert mo["mass"][k] == 0.0
    assert np.array_equal(mo["com"][k], 0.5 * (mo["lo"][k] + mo["hi"][k]))


def _ranges(nodes, ids):
    return sorted((int(nodes[c, 0]), int(nodes[c, 1])) for c in ids)


@pytest.mark.parametrize("theta", [0.0, 0.4, 0.8, 1.5, 4.0])
def test_lists_partition_the_bodies(orc, theta):
    n, leaf, group = 5000, 8, 64
    pm, _ = ics.colliding_pair(n, 21)
    q = _orb(orc, pm, leaf)
    nodes = orc.tree_nodes(n, leaf)
    L = orc.tree_lists(q, leaf, group, theta)
    fo = np.r_[0, np.cumsum(L["far_cnt"])]
    no = np.r_[0, np.cumsum(L["near_cnt"])]
    assert L["group_id"].shape[0] == len(fo) - 1
    # groups: maximal nodes of at most `group` bodies, tiling [0, n) in order
    gr = [tuple(nodes[g, :2]) for g in L["group_id"]]
    assert gr[0][0] == 0 and gr[-1][1] == n and all(a[1] == b[0] for a, b in zip(gr, gr[1:]))
    for g, (gb, ge) in zip(L["group_id"], gr):
        assert ge - gb <= group or nodes[g, 2] < 0
    for q_ in range(len(gr)):
        cells = _ranges(nodes, L["far"][fo[q_]:fo[q_ + 1]]) + _ranges(nodes, L["near"][no[q_]:no[q_ + 1]])
        cells.sort()
        assert cells[0][0] == 0 and cells[-1][1] == n
        assert all(a[1] == b[0] for a, b in zip(cells, cells[1:])), "cells overlap or leave a gap"
        gb, ge = gr[q_]
        for c in L["far"][fo[q_]:fo[q_ + 1]]:
            assert nodes[c, 1] <= gb or nodes[c, 0] >= ge, "accepted cell overlaps its group"
        for c in L["near"][no[q_]:no[q_ + 1]]:
            assert nodes[c, 2] < 0, "near entries are leaves"
    if theta == 0.0:
        assert L["far_cnt"].sum() == 0


@pytest.mark.parametrize("theta", [0.3, 0.7, 1.2])
def test_accepted_cells_are_distant_body_by_body(orc, theta):
    """Every body of an accepted cell lies within s of its centre of mass and
    every body of the group lies farther than s / theta from it: the
    size-to-distance ratio is below theta for each target (Section IV.A's
    'distant enough'), checked from the coordinates directly."""
    n, leaf, group = 2048, 4, 32
    pm, _ = ics.plummer(n, 5)
    q = _orb(orc, pm, leaf)
    x = q[:, :3].astype(np.float64)
    nodes = orc.tree_nodes(n, leaf)
    mo = orc.tree_moments(q, leaf)
    L = orc.tree_lists(q, leaf, group, theta)
    fo = np.r_[0, np.cumsum(L["far_cnt"])]
    checked = 0
    for qi, g in enumerate(L["group_id"]):
        gb, ge = nodes[g, :2]
        for c in L["far"][fo[qi]:fo[qi + 1]]:
            b, e = nodes[c, :2]
            com = mo["com"][c]
            size = np.sqrt(((x[b:e].max(0) - x[b:e].min(0)) ** 2).sum())
            assert np.linalg.norm(x[b:e] - com, axis=1).max() <= size * (1 + 1e-12)
            dmin = np.linalg.norm(x[gb:ge] - com, axis=1).min()
            assert size < theta * dmin * (1 + 1e-12)
            checked += 1
    assert checked > 100


def test_maximal_acceptance_brute_force(orc):
    """On a small tree, the far list of each group is exactly the set of
    acceptable cells none of whose ancestors is acceptable, and the near list
    the remaining leaves outside the group: the walk visits children only of
    cells it could not accept."""
    n, leaf, group, theta = 96, 2, 8, 0.9
    pm, _ = ics.uniform_ball(n, 9)
    q = _orb(orc, pm, leaf)
    x = q[:, :3].astype(np.float64)
    nodes = orc.tree_nodes(n, leaf)
    mo = orc.tree_moments(q, leaf)
    L = orc.tree_lists(q, leaf, group, theta)
    parent = -np.ones(nodes.shape[0], dtype=np.int64)
    for k in range(nodes.shape[0]):
        if nodes[k, 2] >= 0:
            parent[nodes[k, 2]] = parent[nodes[k, 3]] = k
    fo = np.r_[0, np.cumsum(L["far_cnt"])]
    no = np.r_[0, np.cumsum(L["near_cnt"])]
    for qi, g in enumerate(L["group_id"]):
        gb, ge = nodes[g, :2]
        glo, ghi = x[gb:ge].min(0), x[gb:ge].max(0)

        def ok(c):
            b, e = nodes[c, :2]
            if b < ge and gb < e:
                return False
            com = mo["com"][c]
            d = np.maximum(0.0, np.maximum(glo - com, com - ghi))
            return bool(mo["diag2"][c] < theta * theta * float(d @ d))

        def any_anc_ok(c):
            p = parent[c]
            while p >= 0:
                if ok(p):
                    return True
                p = parent[p]
            return False

        far = {c for c in range(nodes.shape[0]) if ok(c) and not any_anc_ok(c)}
        near = {c for c in range(nodes.shape[0]) if nodes[c, 2] < 0 and not ok(c) and not any_anc_ok(c)}
        assert set(L["far"][fo[qi]:fo[qi + 1]].tolist()) == far
        assert set(L["near"][no[qi]:no[qi + 1]].tolist()) == near


def test_theta_zero_is_the_direct_sum(orc):
    n = 1500
    pm, _ = ics.plummer(n, 13)
    q = _orb(orc, pm, 8)
    a, p = orc.tree_accel(q, 8, 64, 0.0, 0.01)
    ad, pd = orc.accel(q, 0.01)
    np.testing.assert_allclose(a, ad, rtol=1e-12, atol=1e-14 * np.abs(ad).max())
    np.testing.assert_allclose(p, pd, rtol=1e-13)


def test_pair_monopole_closed_form(orc):
    """Two bodies of mass m at x = -s and x = +s, a light target at x = D:
    once the pair is accepted the target feels -2 G m / D^2 (the pair's mass
    at its centre), before that the exact -G m [1/(D-s)^2 + 1/(D+s)^2]."""
    s, D, m, G = 0.25, 4.0, 0.5, 1.0
    pm = np.array([[-s, 0, 0, m], [s, 0, 0, m], [D, 0, 0, 1e-30]], dtype=np.float32)
    q = _orb(orc, pm, 1)
    assert q[2, 0] == D  # ORB along x: the pair forms one node, the target another
    thr = 2 * s / D  # diagonal 2s against the distance D
    for theta, expect in [(thr * 1.01, -2 * G * m / D**2),
                          (thr * 0.99, -G * m * (1 / (D - s) ** 2 + 1 / (D + s) ** 2))]:
        a, p = orc.tree_accel(q, 1, 1, theta, 0.0, G=G, targets=[2])
        assert a[0, 0] == pytest.approx(expect, rel=1e-14)
        assert a[0, 1] == 0.0 and a[0, 2] == 0.0
        pexp = -2 * G * m / D if theta > thr else -G * m * (1 / (D - s) + 1 / (D + s))
        assert p[0] == pytest.approx(pexp, rel=1e-14)


def test_error_falls_with_theta(orc):
    n = 8192
    pm, _ = ics.plummer(n, 17)
    q = _orb(orc, pm, 4)
    tg = np.random.default_rng(3).choice(n, 400, replace=False)
    ad, pd = orc.accel(q, 0.01, targets=tg)
    errs = []
    for theta in [0.3, 0.6, 1.0]:
        a, p = orc.tree_accel(q, 4, 64, theta, 0.01, targets=tg)
        rel = np.linalg.norm(a - ad, axis=1) / np.linalg.norm(ad, axis=1)
        errs.append(np.sqrt(np.mean(rel ** 2)))
        # monopole truncation is second order in the size-to-distance ratio
        assert errs[-1] < 0.1 * theta ** 2
        assert np.sqrt(np.mean(((p - pd) / pd) ** 2)) < 0.1 * theta ** 2
    assert errs[0] < errs[1] < errs[2]
    assert errs[0] > 0.0
