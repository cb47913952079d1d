"""Pins of the oracle's pseudo-particle cells (the pseudo-particle multipole
method of Makino 1999, the paper's reference [20], cited in Section VI for
the O(N) fast multipole method): each cell's
expansion to quadrupole order about its centre of mass is carried by 12
point masses on the icosahedron directions.

The checks stand apart from the oracle's formula: the directions integrate
every monomial of degree <= 5 like the unit sphere (closed-form sphere
moments), the pseudo-particles reproduce the cell's mass, dipole and
traceless quadrupole computed from the bodies with numpy, the far-field
error falls one order of a/R faster than the monopole's and agrees with the
explicit quadrupole expansion to the next order, theta = 0 is the direct
sum, and the tree force beats the monopole tree at the same theta.
"""
import itertools
import math

import numpy as np
import pytest

import ics


def _orb(orc, pm, leaf):
    perm = orc.orb_order(pm, leaf)
    return np.ascontiguousarray(np.asarray(pm, dtype=np.float32)[perm])


def _dfact(k):
    return 1 if k <= 0 else k * _dfact(k - 2)


def _sphere_mean(a, b, c):
    """Mean of x^a y^b z^c over the unit sphere."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    return _dfact(a - 1) * _dfact(b - 1) * _dfact(c - 1) / _dfact(a + b + c + 1)


def test_directions_are_a_spherical_5_design(orc):
    s = orc.pseudo_dirs()
    assert s.shape == (12, 3)
    np.testing.assert_allclose(np.linalg.norm(s, axis=1), 1.0, rtol=0, atol=1e-15)
    # 12 distinct directions, each with 5 nearest neighbours at arccos(1/sqrt 5)
    cos = s @ s.T
    assert np.all(cos[~np.eye(12, dtype=bool)] < 1 - 1e-9)
    near = np.sum(np.isclose(cos, 1 / math.sqrt(5), atol=1e-12), axis=1)
    assert np.all(near == 5)
    for a, b, c in itertools.product(range(6), repeat=3):
        if a + b + c > 5:
            continue
        mean = np.mean(s[:, 0] ** a * s[:, 1] ** b * s[:, 2] ** c)
        assert mean == pytest.approx(_sphere_mean(a, b, c), abs=1e-14), (a, b, c)
    # degree 6 is not integrated exactly (x^6 + y^6 + z^6 has sphere mean 3/7)
    assert abs(np.mean((s ** 6).sum(1)) - 3 / 7) > 1e-3


def _body_moments(x, m, com):
    r = x - com
    M = m.sum()
    D = (m[:, None] * r).sum(0)
    r2 = (r * r).sum(1)
    Q = 3 * np.einsum("i,ij,ik->jk", m, r, r) - np.eye(3) * (m * r2).sum()
    return M, D, Q


@pytest.mark.parametrize("n,leaf,seed", [(300, 8, 31), (1000, 3, 32), (64, 64, 33)])
def test_pseudo_particles_carry_the_cell_moments(orc, n, leaf, seed):
    pm, _ = ics.plummer(n, seed)
    q = _orb(orc, pm, leaf)
    x = q[:, :3].astype(np.float64)
    m = q[:, 3].astype(np.float64)
    nodes = orc.tree_nodes(n, leaf)
    mo = orc.tree_moments(q, leaf)
    pp = orc.tree_pseudo(q, leaf)
    assert pp.shape == (nodes.shape[0], 12, 4)
    s = orc.pseudo_dirs()
    for k in range(nodes.shape[0]):
        b, e = nodes[k, :2]
        com = mo["com"][k]
        a = 0.5 * math.sqrt(mo["diag2"][k])
        # positions: com + a s_j
        np.testing.assert_allclose(pp[k, :, :3], com + a * s, rtol=0, atol=1e-15)
        M, D, Q = _body_moments(x[b:e], m[b:e], com)
        qq, P = pp[k, :, 3], pp[k, :, :3]
        Mp, Dp, Qp = _body_moments(P, qq, com)
        assert Mp == pytest.approx(M, rel=1e-13)
        scale = M * max(a, 1e-300)
        if a > 0:
            np.testing.assert_allclose(Dp, D, rtol=0, atol=1e-13 * scale)
            np.testing.assert_allclose(Qp, Q, rtol=0, atol=1e-12 * M * a * a)
        else:
            np.testing.assert_allclose(qq, M / 12, rtol=1e-15)


def _pot(src, ms, pts):
    d = pts[:, None, :] - src[None, :, :]
    return -(ms[None, :] / np.sqrt((d * d).sum(-1))).sum(1)


def test_far_field_error_orders(orc):
    """One cell of 50 bodies: along 200 random directions at R = 8a .. 64a the
    monopole's relative error falls as (a/R)^2, the pseudo-particles' as
    (a/R)^3, and the pseudo-particles differ from the explicit quadrupole
    expansion -(M/R + R.Q.R / (2 R^5)) as (a/R)^4."""
    rng = np.random.default_rng(41)
    n = 50
    x = rng.uniform(-0.5, 0.5, (n, 3)) * np.array([1.0, 0.6, 0.3])
    m = rng.uniform(0.5, 1.5, n)
    pm = np.c_[x, m].astype(np.float32)
    pp = orc.tree_pseudo(pm, 64)[0]
    mo = orc.tree_moments(pm, 64)
    com, a = mo["com"][0], 0.5 * math.sqrt(mo["diag2"][0])
    xs, ms = pm[:, :3].astype(np.float64), pm[:, 3].astype(np.float64)
    M, _, Q = _body_moments(xs, ms, com)
    u = rng.normal(size=(200, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    e_mono, e_pp, e_q = [], [], []
    for R in (8 * a, 16 * a, 32 * a, 64 * a):
        pts = com + R * u
        exact = _pot(xs, ms, pts)
        mono = -M / R * np.ones(len(u))
        pseudo = _pot(pp[:, :3], pp[:, 3], pts)
        quad = -(M / R + np.einsum("ij,jk,ik->i", u, Q, u) / (2 * R ** 3))
        e_mono.append(np.sqrt(np.mean(((mono - exact) / exact) ** 2)))
        e_pp.append(np.sqrt(np.mean(((pseudo - exact) / exact) ** 2)))
        e_q.append(np.sqrt(np.mean(((pseudo - quad) / exact) ** 2)))
    r_mono = np.array(e_mono[:-1]) / np.array(e_mono[1:])
    r_pp = np.array(e_pp[:-1]) / np.array(e_pp[1:])
    r_q = np.array(e_q[:-1]) / np.array(e_q[1:])
    assert np.all((r_mono > 3.5) & (r_mono < 4.5)), r_mono
    assert np.all((r_pp > 6.5) & (r_pp < 9.5)), r_pp
    assert np.all((r_q > 13) & (r_q < 19)), r_q
    assert e_pp[0] < 0.3 * e_mono[0]


def test_theta_zero_is_the_direct_sum(orc):
    pm, _ = ics.plummer(700, 42)
    q = _orb(orc, pm, 4).astype(np.float64)
    a, p = orc.tree_accel(q, 4, 64, 0.0, 0.01, cells=2)
    ra, rp = orc.accel(q, 0.01)
    np.testing.assert_allclose(a, ra, rtol=1e-12, atol=1e-12 * np.abs(ra).max())
    np.testing.assert_allclose(p, rp, rtol=1e-12)


def test_tree_force_beats_the_monopole_tree(orc):
    """Plummer N = 4000, leaf 4: at theta 0.5, 0.7, 1.0 the pseudo-particle
    tree's rms force error is below half the monopole tree's, and the gain
    grows as theta falls (one more order of the size-to-distance ratio;
    measured 7.0x, 5.5x, 3.0x)."""
    pm, _ = ics.plummer(4000, 43)
    q = _orb(orc, pm, 4).astype(np.float64)
    ra, rp = orc.accel(q, 0.01)
    gain = []
    for theta in (0.5, 0.7, 1.0):
        err = {}
        for order in (0, 2):
            a, p = orc.tree_accel(q, 4, 64, theta, 0.01, cells=order)
            err[order] = np.sqrt(np.mean((np.linalg.norm(a - ra, axis=1) / np.linalg.norm(ra, axis=1)) ** 2))
        print("theta", theta, "rms force error monopole", err[0], "pseudo-particles", err[2])
        assert err[2] < err[0] / 2
        gain.append(err[0] / err[2])
    assert gain[0] > gain[1] > gain[2]


def test_massless_and_point_cells(orc):
    """A cell of zero mass has zero pseudo-masses; a cell whose bodies sit on
    one point (box diagonal 0) keeps M / 12 on each pseudo-particle."""
    pm = np.zeros((16, 4), dtype=np.float32)
    pm[:8, :3] = np.float32(0.25)
    pm[:8, 3] = np.arange(1, 9, dtype=np.float32)
    pm[8:, :3] = np.random.default_rng(5).uniform(-1, 1, (8, 3)).astype(np.float32) + 3
    pm[8:, 3] = 0.0
    q = _orb(orc, pm, 8)
    nodes = orc.tree_nodes(16, 8)
    pp = orc.tree_pseudo(q, 8)
    for k in range(nodes.shape[0]):
        b, e = nodes[k, :2]
        M = q[b:e, 3].astype(np.float64).sum()
        if nodes[k, 2] >= 0:
            continue
        if M == 0:
            assert np.all(pp[k, :, 3] == 0)
        else:
            np.testing.assert_allclose(pp[k, :, 3], M / 12, rtol=1e-15)
            np.testing.assert_allclose(pp[k, :, :3], 0.25, rtol=0, atol=1e-15)


def test_order_is_validated(orc):
    pm, _ = ics.plummer(100, 44)
    with pytest.raises(ValueError):
        orc.tree_accel(_orb(orc, pm, 4), 4, 64, 0.5, 0.01, cells=1)
