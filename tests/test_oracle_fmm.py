"""Pins of the oracle's multi-level fast multipole method on the ORB nodes
(the O(N) method Section VI points to): quadrupole cells, third-order local
expansions, L2L down the tree, M2P cells and P2P leaves at the leaves.

* theta = 0: no M2L or M2P entry, and the result is the direct sum.
* The dual-tree traversal counts every ordered pair of distinct bodies
  exactly once (brute force over all pairs), every M2L entry passes the
  acceptance test, every M2P entry is a leaf target for which the source
  fails it but passes the tree code's box test, and every P2P entry is a
  pair of leaves that fails both (the tests recomputed here from the node
  moments).
* A leaf of a few far-flung bodies gets a short list of M2P cells instead
  of a P2P entry with every leaf, and its bodies' forces stay within the
  quadrupole cells' error of the direct sum.
* L2L: the re-expanded cubic equals the original at every point (the
  Taylor polynomial evaluated here from its definition).
* Far-field order: for two clusters at distance D the force error of one
  M2L + L2P falls as D^-5 (relative error (b/D)^3, the quadrupole cells'
  order), which a dropped quadrupole or cubic term would turn into D^-4.
* Accuracy improves as theta shrinks, on a Plummer sphere.
"""
import numpy as np
import pytest

import ics
from nbtest import rms_rel, widen32


def _orb(orc, pm, leaf):
    pm32 = np.asarray(pm, dtype=np.float32)
    perm = orc.orb_order(pm32, leaf)
    return widen32(pm32[perm])


def test_theta_zero_is_the_direct_sum(orc):
    for n, leaf in [(1, 4), (2, 1), (777, 4), (3000, 8)]:
        pm, _ = ics.plummer(max(n, 2), 70 + n)
        q = _orb(orc, pm[:n], leaf)
        L = orc.fmm_lists(q, leaf, 0.0)
        assert L["m2l_cnt"].sum() == 0 and L["m2p_cnt"].sum() == 0
        a, p = orc.fmm_accel(q, leaf, 0.0, 0.01)
        if n == 1:
            assert np.all(a == 0) and np.all(p == 0)
            continue
        ad, pd = orc.accel(q, 0.01)
        np.testing.assert_allclose(a, ad, rtol=1e-12, atol=1e-12 * np.abs(ad).max())
        np.testing.assert_allclose(p, pd, rtol=1e-12)


@pytest.mark.parametrize("n,leaf,theta,kind", [(300, 4, 0.6, "plummer"), (256, 1, 0.9, "collide"),
                                               (400, 8, 0.4, "ball"), (333, 3, 1.2, "plummer")])
def test_every_pair_counted_once_and_lists_follow_the_tests(orc, n, leaf, theta, kind):
    gen = {"plummer": ics.plummer, "collide": ics.colliding_pair, "ball": ics.uniform_ball}[kind]
    pm, _ = gen(n, 80 + n)
    q = _orb(orc, pm, leaf)
    nodes = orc.tree_nodes(n, leaf)
    mom = orc.tree_moments(q, leaf)
    L = orc.fmm_lists(q, leaf, theta)
    cov = np.zeros((n, n), dtype=np.int64)
    th2 = theta * theta

    def overlap(a, b):
        return nodes[a, 0] < nodes[b, 1] and nodes[b, 0] < nodes[a, 1]

    def mac(a, b):
        if overlap(a, b):
            return False
        d = mom["com"][a] - mom["com"][b]
        return mom["diag2"][a] + mom["diag2"][b] < th2 * float(d @ d)

    def box_test(a, b):  # source b against the box of target a
        if overlap(a, b):
            return False
        gap = np.maximum(mom["lo"][a] - mom["com"][b], 0) + np.maximum(mom["com"][b] - mom["hi"][a], 0)
        return mom["diag2"][b] < th2 * float(gap @ gap)

    o = 0
    for a in range(nodes.shape[0]):
        for b in L["m2l"][o:o + L["m2l_cnt"][a]]:
            assert mac(a, b)
            cov[nodes[a, 0]:nodes[a, 1], nodes[b, 0]:nodes[b, 1]] += 1
        o += L["m2l_cnt"][a]
    o = 0
    for a in range(nodes.shape[0]):
        if L["m2p_cnt"][a]:
            assert nodes[a, 2] < 0
        for b in L["m2p"][o:o + L["m2p_cnt"][a]]:
            assert not mac(a, b) and box_test(a, b)
            cov[nodes[a, 0]:nodes[a, 1], nodes[b, 0]:nodes[b, 1]] += 1
        o += L["m2p_cnt"][a]
    o = 0
    for a in range(nodes.shape[0]):
        if L["p2p_cnt"][a]:
            assert nodes[a, 2] < 0
        for b in L["p2p"][o:o + L["p2p_cnt"][a]]:
            assert nodes[b, 2] < 0 and not mac(a, b) and not box_test(a, b)
            cov[nodes[a, 0]:nodes[a, 1], nodes[b, 0]:nodes[b, 1]] += 1
        o += L["p2p_cnt"][a]
    off = ~np.eye(n, dtype=bool)
    assert np.all(cov[off] == 1)
    # the diagonal is covered once, by each leaf's P2P entry with itself,
    # whose self pair the sum skips
    assert np.all(np.diag(cov) == 1)


def _taylor(c, y):
    """P0 + p.y + y.K.y/2 + T(y,y,y)/6 and its gradient, from the 20 stored
    coefficients (K: xx, yy, zz, xy, xz, yz; T: xxx, yyy, zzz, xxy, xxz, xyy,
    yyz, xzz, yzz, xyz)."""
    K = np.array([[c[4], c[7], c[8]], [c[7], c[5], c[9]], [c[8], c[9], c[6]]])
    idx = [(0, 0, 0), (1, 1, 1), (2, 2, 2), (0, 0, 1), (0, 0, 2), (0, 1, 1), (1, 1, 2), (0, 2, 2), (1, 2, 2),
           (0, 1, 2)]
    T = np.zeros((3, 3, 3))
    import itertools
    for u, t in enumerate(idx):
        for perm in itertools.permutations(t):
            T[perm] = c[10 + u]
    p = np.asarray(c[1:4])
    val = c[0] + p @ y + 0.5 * y @ K @ y + np.einsum("klm,k,l,m->", T, y, y, y) / 6.0
    grad = p + K @ y + 0.5 * np.einsum("klm,l,m->k", T, y, y)
    return val, grad


def test_l2l_reexpands_the_cubic_exactly(orc):
    g = np.random.default_rng(5)
    for _ in range(20):
        c = g.normal(size=20)
        dz = g.normal(size=3)
        s = orc.local_shift(c, dz)
        assert np.array_equal(s[10:], c[10:])
        for _ in range(5):
            y = g.normal(size=3)
            v0, g0 = _taylor(c, y + dz)
            v1, g1 = _taylor(s, y)
            assert abs(v1 - v0) <= 1e-12 * (1 + abs(v0)) * 50
            np.testing.assert_allclose(g1, g0, rtol=1e-11, atol=1e-11 * (1 + np.abs(g0).max()))
    # zero shift is the identity
    c = g.normal(size=20)
    assert np.array_equal(orc.local_shift(c, np.zeros(3)), c)


def test_far_field_order(orc):
    """Two 20-body clusters of radius 1 at distance D, each a leaf: one M2L
    each way.  Far-field force error ~ D^-5 (ratio 32 per doubling)."""
    g = np.random.default_rng(3)

    def ball(k):
        v = g.normal(size=(k, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        return v * g.uniform(size=(k, 1)) ** (1 / 3)

    A, B = ball(20), ball(20)
    m = g.uniform(0.5, 1.5, 40)
    errs = []
    for D in (8.0, 16.0, 32.0):
        x = np.vstack([A, B + [D, 0, 0]])
        q = _orb(orc, np.hstack([x, m[:, None]]), 20)
        L = orc.fmm_lists(q, 20, 0.9)
        assert L["m2l_cnt"].sum() == 2 and L["p2p_cnt"].sum() == 2 and L["m2p_cnt"].sum() == 0
        a, p = orc.fmm_accel(q, 20, 0.9, 0.0)
        ad, pd = orc.accel(q, 0.0)
        errs.append(np.sqrt(np.mean(np.sum((a - ad) ** 2, axis=1))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 24 < r1 < 42 and 24 < r2 < 42, (r1, r2)


def test_accuracy_improves_with_theta(orc):
    pm, _ = ics.plummer(6000, 91)
    q = _orb(orc, pm, 8)
    ad, _ = orc.accel(q, 0.01)
    e = [rms_rel(orc.fmm_accel(q, 8, th, 0.01)[0], ad) for th in (0.25, 0.45, 0.7)]
    assert e[0] < e[1] < e[2]
    assert e[0] < 2e-4 and e[2] < 2e-2


def test_far_flung_leaf_takes_cells_not_every_leaf(orc):
    """A dense ball of 2000 bodies and 8 bodies strung along the x axis from
    20 to 60.  ORB puts the 8 in one leaf whose box is far larger than its
    distance to the ball, so it fails the FMM's test against every node;
    through M2P it still sees the ball as cells, not leaf by leaf, and its
    bodies' forces stay within the quadrupole cells' error."""
    g = np.random.default_rng(17)
    v = g.normal(size=(2000, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    ball = v * g.uniform(size=(2000, 1)) ** (1 / 3)
    line = np.column_stack([np.linspace(20, 60, 8), g.normal(0, 0.5, (8, 2))])
    x = np.vstack([ball, line])
    pm = np.hstack([x, g.uniform(0.5, 1.5, (x.shape[0], 1))]).astype(np.float32)
    leaf = 8
    perm = orc.orb_order(pm, leaf)
    q = widen32(pm[perm])
    far = np.nonzero(np.linalg.norm(q[:, :3], axis=1) > 20)[0]
    assert far.size == 8 and far.max() - far.min() == 7  # one leaf
    nodes = orc.tree_nodes(q.shape[0], leaf)
    A = int(np.nonzero((nodes[:, 0] == far.min()) & (nodes[:, 2] < 0))[0][0])
    theta = 0.5
    L = orc.fmm_lists(q, leaf, theta)
    off = lambda c, a: int(c[:a].sum())
    m2p = L["m2p"][off(L["m2p_cnt"], A):off(L["m2p_cnt"], A) + L["m2p_cnt"][A]]
    p2p = L["p2p"][off(L["p2p_cnt"], A):off(L["p2p_cnt"], A) + L["p2p_cnt"][A]]
    assert L["m2l_cnt"][A] == 0 and len(m2p) > 0
    nleaves = int((nodes[:, 2] < 0).sum())
    assert len(p2p) + len(m2p) < nleaves / 4, (len(p2p), len(m2p), nleaves)
    # the M2P cells hold most of the ball
    ball_in_cells = int(sum(nodes[b, 1] - nodes[b, 0] for b in m2p))
    assert ball_in_cells > 1500
    a, _ = orc.fmm_accel(q, leaf, theta, 0.0, targets=far)
    ad, _ = orc.accel(q, 0.0, targets=far)
    assert rms_rel(a, ad) < 1e-3


def test_coincident_bodies_take_no_expansion(orc):
    """Every body at one point: every box has zero size and every pair of
    nodes zero distance, so no test passes and the FMM is the direct sum
    (with softening), whatever theta."""
    n, leaf = 200, 4
    pm = np.zeros((n, 4))
    pm[:, :3] = [0.25, -1.5, 3.0]
    pm[:, 3] = np.linspace(0.5, 1.5, n)
    q = _orb(orc, pm, leaf)
    for theta in (0.5, 5.0):
        L = orc.fmm_lists(q, leaf, theta)
        assert L["m2l_cnt"].sum() == 0 and L["m2p_cnt"].sum() == 0
        a, p = orc.fmm_accel(q, leaf, theta, 0.1, G=2.0)
        assert np.all(a == 0)
        # phi_i = -G (M - m_i) / eps
        np.testing.assert_allclose(p, -2.0 * (q[:, 3].sum() - q[:, 3]) / 0.1, rtol=1e-13)
