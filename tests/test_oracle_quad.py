"""Pins of the oracle's quadrupole cells (the expansion of the paper's
reference [20] through l = 2, evaluated directly from the cell's traceless
quadrupole tensor).

A far probe: 64 bodies form one cell and 64 massless targets sit in a tiny
cluster at distance R along a chosen direction, so the ORB recursion puts
them in separate leaves and the targets' group accepts the cell whole. The
oracle's own tree force then evaluates the cell's expansion at those points.
Checked: the tensor against numpy; the error against the exact sum falls as
(a/R)^3; the difference from the independently written pseudo-particle
cells falls as (a/R)^4 (their only difference is the pseudo-particles'
l >= 4 residue); the force is minus the gradient of the potential (central
differences, with and without softening); theta = 0 is the direct sum; in a
Plummer tree the error matches the pseudo-particle cells' and beats the
monopole's.
"""
import math

import numpy as np
import pytest

import ics


def _orb(orc, pm, leaf):
    perm = orc.orb_order(pm, leaf)
    return np.ascontiguousarray(np.asarray(pm, dtype=np.float32)[perm])


def test_quadrupole_tensor_against_numpy(orc):
    pm, _ = ics.plummer(2000, 51)
    q = _orb(orc, pm, 4)
    x, m = q[:, :3].astype(np.float64), q[:, 3].astype(np.float64)
    nodes = orc.tree_nodes(2000, 4)
    mo = orc.tree_moments(q, 4)
    Q = orc.tree_quad(q, 4)
    for k in range(0, nodes.shape[0], 7):
        b, e = nodes[k, :2]
        r = x[b:e] - mo["com"][k]
        r2 = (r * r).sum(1)
        T = 3 * np.einsum("i,ij,ik->jk", m[b:e], r, r) - np.eye(3) * (m[b:e] * r2).sum()
        want = np.array([T[0, 0], T[1, 1], T[2, 2], T[0, 1], T[0, 2], T[1, 2]])
        scale = m[b:e].sum() * max(float(r2.max()), 1e-300)
        np.testing.assert_allclose(Q[k], want, rtol=0, atol=1e-13 * scale)
        assert abs(Q[k, 0] + Q[k, 1] + Q[k, 2]) <= 1e-13 * scale


def _probe(orc, cells, R, u, eps=0.0, shift=None, seed=61):
    """Potential and acceleration of the 64 probe targets (massless, a tiny
    cluster at R u) from the 64-body cell near the origin, through the tree
    with theta = 1 (the cell is accepted whole)."""
    rng = np.random.default_rng(seed)
    cell = np.c_[rng.uniform(-0.5, 0.5, (64, 3)) * np.array([1.0, 0.7, 0.4]), rng.uniform(0.5, 1.5, 64)]
    tg = np.c_[R * u + rng.uniform(-1, 1, (64, 3)) * 1e-3 * R, np.zeros(64)]
    if shift is not None:
        tg[:, :3] += shift
    pm = np.r_[cell, tg].astype(np.float64)
    perm = orc.orb_order(pm, 64)
    q = pm[perm]
    nodes = orc.tree_nodes(128, 64)
    assert nodes.shape[0] == 3
    L = orc.tree_lists(q, 64, 64, 1.0)
    is_target = q[:, 3] == 0
    tgt_group = 1 if is_target[nodes[1, 0]] else 2
    g = list(L["group_id"]).index(tgt_group)
    # the cell is the one far entry; the near list is the targets' own leaf
    assert L["far_cnt"][g] == 1 and L["near_cnt"][g] == 1, "the probe must accept the cell whole"
    assert L["far"][int(L["far_cnt"][:g].sum())] == 3 - tgt_group
    a, p = orc.tree_accel(q, 64, 64, 1.0, eps, cells=cells)
    ad, pd = orc.accel(q, eps)
    return a[is_target], p[is_target], ad[is_target], pd[is_target], q[is_target]


def test_far_field_orders_against_exact_and_pseudo_particles(orc):
    dirs = np.random.default_rng(62).normal(size=(24, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    eq, eqp, eqa = [], [], []
    for R in (8.0, 16.0, 32.0, 64.0):
        r_q, r_qp, r_qa = [], [], []
        for u in dirs:
            a3, p3, ad, pd, _ = _probe(orc, 3, R, u)
            a2, p2, _, _, _ = _probe(orc, 2, R, u)
            r_q.append(np.abs((p3 - pd) / pd))
            r_qp.append(np.abs((p3 - p2) / pd))
            r_qa.append(np.linalg.norm(a3 - ad, axis=1) / np.linalg.norm(ad, axis=1))
        eq.append(np.sqrt(np.mean(np.square(r_q))))
        eqp.append(np.sqrt(np.mean(np.square(r_qp))))
        eqa.append(np.sqrt(np.mean(np.square(r_qa))))
    rq = np.array(eq[:-1]) / np.array(eq[1:])
    rqp = np.array(eqp[:-1]) / np.array(eqp[1:])
    rqa = np.array(eqa[:-1]) / np.array(eqa[1:])
    print("potential error ratios", rq, "quad-vs-pseudo ratios", rqp, "force error ratios", rqa)
    assert np.all((rq > 6.5) & (rq < 9.5)), rq
    assert np.all((rqp > 13) & (rqp < 19)), rqp
    assert np.all((rqa > 6.5) & (rqa < 9.5)), rqa


@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_force_is_minus_the_potential_gradient(orc, eps):
    u = np.array([0.6, -0.48, 0.64])
    R, h = 6.0, 1e-4
    a, _, _, _, xt = _probe(orc, 3, R, u, eps)
    # the targets are massless, so each one's potential is the cell's field at
    # its own position; moving them all together keeps every decision
    grad = np.zeros_like(a)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        _, pp_, _, _, xp = _probe(orc, 3, R, u, eps, shift=e)
        _, pm_, _, _, xm = _probe(orc, 3, R, u, eps, shift=-e)
        # same targets in the same ORB order (the shift moves them rigidly)
        assert np.allclose(xp[:, :3] - xt[:, :3], e) and np.allclose(xm[:, :3] - xt[:, :3], -e)
        grad[:, k] = (pp_ - pm_) / (2 * h)
    np.testing.assert_allclose(a, -grad, rtol=2e-7, atol=2e-7 * np.abs(a).max())


def test_theta_zero_is_the_direct_sum(orc):
    pm, _ = ics.plummer(700, 63)
    q = _orb(orc, pm, 4).astype(np.float64)
    a, p = orc.tree_accel(q, 4, 64, 0.0, 0.01, cells=3)
    ra, rp = orc.accel(q, 0.01)
    np.testing.assert_allclose(a, ra, rtol=1e-12, atol=1e-12 * np.abs(ra).max())
    np.testing.assert_allclose(p, rp, rtol=1e-12)


def test_tree_error_matches_pseudo_particles_and_beats_monopole(orc):
    pm, _ = ics.plummer(4000, 43)
    q = _orb(orc, pm, 4).astype(np.float64)
    ra, _ = orc.accel(q, 0.01)
    for theta in (0.5, 0.7, 1.0):
        err = {}
        for cells in (0, 2, 3):
            a, _ = orc.tree_accel(q, 4, 64, theta, 0.01, cells=cells)
            err[cells] = np.sqrt(np.mean((np.linalg.norm(a - ra, axis=1) / np.linalg.norm(ra, axis=1)) ** 2))
        print("theta", theta, "monopole", err[0], "pseudo-particles", err[2], "quadrupole", err[3])
        assert err[3] < err[0] / 2
        assert 0.5 < err[3] / err[2] < 2.0


def test_cells_are_validated(orc):
    pm, _ = ics.plummer(100, 64)
    for bad in (1, 5, -1):
        with pytest.raises(ValueError):
            orc.tree_accel(_orb(orc, pm, 4), 4, 64, 0.5, 0.01, cells=bad)
