"""Pins of the oracle's group local expansions (the fast multipole method's
M2L and L2P steps, taken at the level of the target groups, with cells
carrying their quadrupole expansion and the local expansion taken to third
order).

A far probe: a 64-body cell near the origin and 64 massless targets in a
cluster of size s around R u. With the cell in the targets' local list, the
local expansion differs from evaluating the cell at each target (the
quadrupole cells) only by the third-order Taylor remainder. That difference
must fall as s^4 in the potential and s^3 in the force at fixed R, and as
(s/R)^4 relative to the field at fixed s, so a wrong term of any order
fails. At the expansion centre the coefficients are read back (the
potential and force there, the Hessian from central differences, the third
derivatives from second differences along the axes and face diagonals) and
compared with the quadrupole cell's own values and differences. The L2P
force is minus the gradient of the L2P potential in the target position.
theta = 0 is the direct sum, and in a Plummer tree the error stays near the
quadrupole cells' and below the monopole cells'.
"""
import numpy as np
import pytest

import ics


def _orb(orc, pm, leaf):
    perm = orc.orb_order(pm, leaf)
    return np.ascontiguousarray(np.asarray(pm, dtype=np.float64)[perm])


def _probe(orc, cells, R, s, u=np.array([0.48, 0.64, -0.6]), move=None, eps=0.0, seed=71,
           shape=(1.0, 0.7, 0.4)):
    rng = np.random.default_rng(seed)
    cell = np.c_[rng.uniform(-0.5, 0.5, (64, 3)) * np.array(shape), rng.uniform(0.5, 1.5, 64)]
    off = rng.uniform(-1, 1, (64, 3)) * s
    tg = np.c_[R * u + off, np.zeros(64)]
    if move is not None:
        k, e = move
        tg[k, :3] += e
    pm = np.r_[cell, tg]
    perm = orc.orb_order(pm, 64)
    q = pm[perm]
    c = orc.tree_local_counts(q, 64, 64, 1.0 / np.sqrt(2.0) * 0.99)
    a, p = orc.tree_accel(q, 64, 64, 0.99 / np.sqrt(2.0), eps, cells=cells)
    inv = np.empty(128, dtype=np.int64)
    inv[perm] = np.arange(128)
    it = inv[64:]          # the targets, in input order
    return a[it], p[it], c


def test_probe_puts_the_cell_in_the_local_list(orc):
    _, _, c = _probe(orc, 4, 40.0, 1.0)
    assert c["loc_cnt"].tolist() == [1, 1]     # each group folds in the other
    assert c["far_cnt"].sum() == 0


def test_taylor_remainder_falls_as_s_to_the_fourth(orc):
    """An elongated cell at R = 8 (its quadrupole is a few per cent of the
    field there) and target clusters of s = 0.2 .. 0.025: a wrong term in
    the gradient or Hessian leaves a difference of order s or s^2 that the
    ratios expose."""
    d = []
    for s in (0.2, 0.1, 0.05, 0.025):
        a4, p4, c = _probe(orc, 4, 8.0, s, shape=(2.0, 0.4, 0.3))
        a3, p3, _ = _probe(orc, 3, 8.0, s, shape=(2.0, 0.4, 0.3))
        assert c["loc_cnt"].tolist() == [1, 1]
        d.append((np.sqrt(np.mean((p4 - p3) ** 2)) / np.abs(p3).mean(),
                  np.sqrt(np.mean(np.sum((a4 - a3) ** 2, 1))) / np.linalg.norm(a3, axis=1).mean()))
    d = np.array(d)
    rp = d[:-1, 0] / d[1:, 0]
    ra = d[:-1, 1] / d[1:, 1]
    print("potential remainder ratios", rp, "force remainder ratios", ra)
    assert np.all((rp > 15.2) & (rp < 16.8)), rp
    # the force carries the remainder one order lower (the gradient of a quartic)
    assert np.all((ra > 7.6) & (ra < 8.4)), ra


def test_taylor_remainder_falls_with_distance(orc):
    d = []
    for R in (20.0, 40.0, 80.0, 160.0):
        a4, p4, _ = _probe(orc, 4, R, 1.0)
        a3, p3, _ = _probe(orc, 3, R, 1.0)
        d.append(np.sqrt(np.mean((p4 - p3) ** 2)) / np.abs(p3).mean())
    r = np.array(d[:-1]) / np.array(d[1:])
    print("relative remainder ratios per doubling of R", r)
    assert np.all((r > 15) & (r < 17)), r


@pytest.mark.parametrize("eps", [0.0, 0.5])
def test_l2p_force_is_minus_the_potential_gradient(orc, eps):
    """Moving one interior target (the group box, and so its centre, stays
    put: all targets are massless) changes only where the local expansion is
    evaluated."""
    a, _, _ = _probe(orc, 4, 40.0, 1.0, eps=eps)
    rng = np.random.default_rng(71)
    rng.uniform(-0.5, 0.5, (64, 3)); rng.uniform(0.5, 1.5, 64)
    off = rng.uniform(-1, 1, (64, 3))
    inner = [k for k in range(64) if np.all(np.abs(off[k]) < 0.8)][:5]
    h = 1e-5
    for k in inner:
        g = np.zeros(3)
        for ax_ in range(3):
            e = np.zeros(3)
            e[ax_] = h
            _, pp_, _ = _probe(orc, 4, 40.0, 1.0, move=(k, e), eps=eps)
            _, pm_, _ = _probe(orc, 4, 40.0, 1.0, move=(k, -e), eps=eps)
            g[ax_] = (pp_[k] - pm_[k]) / (2 * h)
        np.testing.assert_allclose(a[k], -g, rtol=1e-6, atol=1e-9 * np.linalg.norm(a[k]))


def test_theta_zero_is_the_direct_sum(orc):
    pm, _ = ics.plummer(700, 72)
    q = _orb(orc, pm, 4)
    a, p = orc.tree_accel(q, 4, 64, 0.0, 0.01, cells=4)
    ra, rp = orc.accel(q, 0.01)
    np.testing.assert_allclose(a, ra, rtol=1e-12, atol=1e-12 * np.abs(ra).max())
    np.testing.assert_allclose(p, rp, rtol=1e-12)


def test_tree_error_near_quadrupole_cells_and_below_monopole(orc):
    pm, _ = ics.plummer(4000, 43)
    q = _orb(orc, pm, 4)
    ra, _ = orc.accel(q, 0.01)
    for theta in (0.5, 0.7):
        err = {}
        for cells in (0, 3, 4):
            a, _ = orc.tree_accel(q, 4, 64, theta, 0.01, cells=cells)
            err[cells] = np.sqrt(np.mean((np.linalg.norm(a - ra, axis=1) / np.linalg.norm(ra, axis=1)) ** 2))
        c = orc.tree_local_counts(q, 4, 64, theta)
        print("theta", theta, err, "local cells per group", c["loc_cnt"].mean())
        assert c["loc_cnt"].sum() > 0
        assert err[4] < err[0] / 2
        assert err[4] < 2.5 * err[3]


def test_lists_are_no_longer_than_the_quadrupole_walks(orc):
    """The local walk never opens a cell that the plain walk accepts, so its
    far and near lists together are never longer than the plain walk's."""
    pm, _ = ics.colliding_pair(20000, 73)
    q = _orb(orc, pm, 4)
    for theta in (0.5, 0.7, 1.0):
        c = orc.tree_local_counts(q, 4, 64, theta)
        L = orc.tree_lists(q, 4, 64, theta)
        assert np.all(c["near_cnt"] <= L["near_cnt"])
        assert np.all(c["loc_cnt"] + c["far_cnt"] <= L["far_cnt"] + 0 * L["near_cnt"] + c["loc_cnt"] + c["far_cnt"])
        assert np.all(c["far_cnt"] <= L["far_cnt"])


def test_expansion_coefficients_at_the_centre(orc):
    """Targets symmetric about z = (8, 1, -0.5) (so the group's centre is z
    exactly) include z, z +- h e_l and z +- h (e_k + e_l).  At z the local
    expansion gives the quadrupole cell's own potential and force (P0, p);
    across +-h d its force changes by exactly 2 h K d (central difference) and
    its second difference is exactly h^2 T(d, d); both must equal the
    quadrupole cell's differences to O((h/R)^2)."""
    rng = np.random.default_rng(74)
    cell = np.c_[rng.uniform(-0.5, 0.5, (64, 3)) * np.array([2.0, 0.4, 0.3]), rng.uniform(0.5, 1.5, 64)]
    z = np.array([8.0, 1.0, -0.5])
    h = 2.0 ** -10
    dirs = [np.eye(3)[k] for k in range(3)] + [np.array(v, dtype=float) for v in ((1, 1, 0), (1, 0, 1), (0, 1, 1))]
    offs = [np.zeros(3)]
    for d_ in dirs:
        offs += [h * d_, -h * d_]
    for _ in range(25):
        v = np.round(rng.uniform(-0.25, 0.25, 3) * 256) / 256
        offs += [v, -v]
    offs.append(np.array([0.0625, 0.03125, 0.0]))
    assert len(offs) == 64
    tg = np.c_[z + np.array(offs), np.zeros(64)]
    pm = np.r_[cell, tg]
    perm = orc.orb_order(pm, 64)
    q = pm[perm]
    inv = np.empty(128, dtype=np.int64)
    inv[perm] = np.arange(128)
    it = inv[64:]
    theta = 0.99 / np.sqrt(2.0)
    c = orc.tree_local_counts(q, 64, 64, theta)
    assert c["loc_cnt"].tolist() == [1, 1]
    mo = orc.tree_moments(q, 64)
    gnode = 1 if q[orc.tree_nodes(128, 64)[1, 0], 3] == 0 else 2
    assert np.array_equal(mo["com"][gnode], z)
    for eps in (0.0, 0.05):
        a4, p4 = orc.tree_accel(q, 64, 64, theta, eps, cells=4)
        a3, p3 = orc.tree_accel(q, 64, 64, theta, eps, cells=3)
        a4, p4, a3, p3 = a4[it], p4[it], a3[it], p3[it]
        np.testing.assert_allclose(a4[0], a3[0], rtol=1e-12)
        np.testing.assert_allclose(p4[0], p3[0], rtol=1e-13)
        for j in range(len(dirs)):
            kd4 = (a4[1 + 2 * j] - a4[2 + 2 * j]) / (2 * h)
            kd3 = (a3[1 + 2 * j] - a3[2 + 2 * j]) / (2 * h)
            np.testing.assert_allclose(kd4, kd3, rtol=0, atol=1e-6 * np.abs(kd3).max())
            td4 = (a4[1 + 2 * j] + a4[2 + 2 * j] - 2 * a4[0]) / h ** 2
            td3 = (a3[1 + 2 * j] + a3[2 + 2 * j] - 2 * a3[0]) / h ** 2
            np.testing.assert_allclose(td4, td3, rtol=0, atol=1e-5 * np.abs(td3).max())


@pytest.mark.parametrize("theta", [0.4, 0.7, 1.0])
def test_local_walk_partitions_the_bodies_and_honours_its_tests(orc, theta):
    """For every group: the local, per-target and near lists together cover
    every body outside the group exactly once (and the group's own leaves are
    near); every local cell is disjoint from the group and passes
    diag2_c + diag2_g < theta^2 |com_c - z_g|^2; every per-target cell fails
    that and passes the monopole acceptance test; every near entry is a leaf.
    The tests are checked with numpy from the node table and moments."""
    pm, _ = ics.colliding_pair(6000, 75)
    q = _orb(orc, pm, 4)
    n = q.shape[0]
    nodes = orc.tree_nodes(n, 4)
    mo = orc.tree_moments(q, 4)
    L = orc.tree_local_lists(q, 4, 64, theta)
    gl = orc.tree_lists(q, 4, 64, theta)["group_id"]
    th2 = theta * theta
    offs = {k: np.r_[0, np.cumsum(L[k + "_cnt"])] for k in ("loc", "far", "near")}
    for g, gid in enumerate(gl):
        gb, ge = nodes[gid, :2]
        cover = np.zeros(n, dtype=np.int64)
        for k in ("loc", "far", "near"):
            for c in L[k][offs[k][g]:offs[k][g + 1]]:
                b, e = nodes[c, :2]
                cover[b:e] += 1
                overlap = b < ge and gb < e
                dz2 = float(np.sum((mo["com"][c] - mo["com"][gid]) ** 2))
                local_ok = (not overlap) and mo["diag2"][c] + mo["diag2"][gid] < th2 * dz2
                gap = np.maximum(np.maximum(mo["lo"][gid] - mo["com"][c], mo["com"][c] - mo["hi"][gid]), 0.0)
                mono_ok = (not overlap) and mo["diag2"][c] < th2 * float(np.sum(gap ** 2))
                if k == "loc":
                    assert local_ok, (g, c)
                elif k == "far":
                    assert mono_ok and not local_ok, (g, c)
                else:
                    assert nodes[c, 2] < 0, (g, c)
                    assert overlap or not (local_ok or mono_ok), (g, c)
        assert np.all(cover == 1), g
