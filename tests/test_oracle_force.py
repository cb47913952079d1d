"""Pins of the FP64 oracle's direct-sum force and potential (paper Section IV:
bodies under mutual gravitation; Section IV.A force loop with every cell
opened = the exact pairwise sum) against closed forms, invariants and
physics that do not depend on the oracle's own code."""
import math

import numpy as np
import pytest

import ics
from conftest import golden_path


def _load_two_body():
    rows = []
    for line in open(golden_path("two_body.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append([float(t) for t in line.split()])
    return rows


def test_two_body_closed_form(orc):
    p = np.array([[0.0, 0.0, 0.0, 1.0], [3.0, 4.0, 0.0, 2.0]])
    for row in _load_two_body():
        G, eps2 = row[0], row[1]
        acc, pot = orc.accel(p, math.sqrt(eps2), G=G)
        np.testing.assert_allclose(acc[0], row[2:5], rtol=1e-15, atol=1e-17)
        np.testing.assert_allclose(pot[0], row[5], rtol=1e-15)
        np.testing.assert_allclose(acc[1], row[6:9], rtol=1e-15, atol=1e-17)
        np.testing.assert_allclose(pot[1], row[9], rtol=1e-15)


def _cube(m=1.0, center=False):
    pts = [[sx, sy, sz, m] for sx in (-1.0, 1.0) for sy in (-1.0, 1.0) for sz in (-1.0, 1.0)]
    if center:
        pts.append([0.0, 0.0, 0.0, 5.0])
    return np.array(pts)


def test_cube_vertex_closed_form(orc):
    # Vertex (1,1,1) of the cube with unit masses, eps = 0: 3 edge neighbours
    # at distance 2, 3 face diagonals at 2 sqrt 2, 1 body diagonal at 2 sqrt 3.
    # a = -(1/4 + 1/(4 sqrt 2) + 1/(12 sqrt 3)) (1,1,1)
    # phi = -(3/2 + 3/(2 sqrt 2) + 1/(2 sqrt 3))
    m = 0.75
    p = _cube(m)
    acc, pot = orc.accel(p, 0.0, G=2.0)
    i = 7  # (1,1,1)
    assert np.all(p[i, :3] == 1.0)
    amag = 0.25 + 1 / (4 * math.sqrt(2)) + 1 / (12 * math.sqrt(3))
    assert abs(amag - 0.474889218) < 1e-9
    np.testing.assert_allclose(acc[i], -2.0 * m * amag * np.ones(3), rtol=1e-14)
    phi = -(1.5 + 3 / (2 * math.sqrt(2)) + 1 / (2 * math.sqrt(3)))
    np.testing.assert_allclose(pot[i], 2.0 * m * phi, rtol=1e-14)
    # every vertex points to the centre with the same magnitude
    np.testing.assert_allclose(acc, -2.0 * m * amag * p[:, :3], rtol=1e-14)


def test_cube_centre_feels_no_force(orc):
    p = _cube(1.0, center=True)
    acc, pot = orc.accel(p, 0.1)
    assert np.max(np.abs(acc[8])) < 1e-15
    np.testing.assert_allclose(pot[8], -8.0 / math.sqrt(3.0 + 0.01), rtol=1e-14)


@pytest.mark.parametrize("nring", [3, 7, 64])
def test_ring_closed_form(orc, nring):
    # N equal masses on a circle of radius R: the pair k apart is 2R sin(pi k/N)
    # away, its pull towards the centre is m sin(pi k/N)/(2R sin(pi k/N))^2, so
    # |a| = G m/(4 R^2) sum_k 1/sin(pi k/N), phi = -G m/(2R) sum_k 1/sin(pi k/N).
    R, m = 1.7, 0.3
    th = 2 * math.pi * np.arange(nring) / nring
    p = np.zeros((nring, 4))
    p[:, 0] = R * np.cos(th)
    p[:, 1] = R * np.sin(th)
    p[:, 3] = m
    acc, pot = orc.accel(p, 0.0)
    S = sum(1.0 / math.sin(math.pi * k / nring) for k in range(1, nring))
    amag = m / (4 * R * R) * S
    np.testing.assert_allclose(acc[:, :2], -amag * p[:, :2] / R, rtol=1e-12, atol=1e-14 * amag)
    assert np.max(np.abs(acc[:, 2])) == 0.0
    np.testing.assert_allclose(pot, -m / (2 * R) * S, rtol=1e-13)


@pytest.mark.parametrize("kind", ["ball", "plummer"])
def test_momentum_conservation(orc, kind):
    if kind == "ball":
        p, _ = ics.uniform_ball(777, 5)
        p[:, 3] *= np.linspace(0.5, 2.0, 777)  # unequal masses
    else:
        p, _ = ics.plummer(1000, 6)
    acc, _ = orc.accel(p, 0.01)
    mom = (p[:, 3:4] * acc).sum(axis=0)
    scale = (p[:, 3] * np.linalg.norm(acc, axis=1)).sum()
    assert np.linalg.norm(mom) / scale <= 1e-13


def test_mirror_rotation_scaling_exact(orc):
    p, _ = ics.plummer(300, 7)
    acc, pot = orc.accel(p, 0.02)
    q = p.copy()
    q[:, :3] = -q[:, :3]
    a2, p2 = orc.accel(q, 0.02)
    assert np.array_equal(a2, -acc) and np.array_equal(p2, pot)
    # 90 degree rotation about z: (x, y) -> (-y, x), exact in floating point
    q = p.copy()
    q[:, 0], q[:, 1] = -p[:, 1], p[:, 0]
    a2, p2 = orc.accel(q, 0.02)
    assert np.array_equal(a2[:, 0], -acc[:, 1]) and np.array_equal(a2[:, 1], acc[:, 0])
    assert np.array_equal(a2[:, 2], acc[:, 2]) and np.array_equal(p2, pot)
    # (x, eps) -> (2x, 2 eps): a -> a/4, phi -> phi/2 (powers of two are exact)
    q = p.copy()
    q[:, :3] *= 2.0
    a2, p2 = orc.accel(q, 0.04)
    assert np.array_equal(a2, acc / 4) and np.array_equal(p2, pot / 2)
    # m -> 2m: a and phi double; G -> 2G likewise
    q = p.copy()
    q[:, 3] *= 2.0
    a2, p2 = orc.accel(q, 0.02)
    assert np.array_equal(a2, 2 * acc) and np.array_equal(p2, 2 * pot)


def test_translation_invariance(orc):
    p, _ = ics.uniform_ball(200, 8)
    acc, pot = orc.accel(p, 0.01)
    q = p.copy()
    q[:, :3] += np.array([0.25, -0.5, 0.125])
    a2, p2 = orc.accel(q, 0.01)
    scale = np.abs(acc).max()
    assert np.abs(a2 - acc).max() <= 1e-12 * scale
    np.testing.assert_allclose(p2, pot, rtol=1e-12)


def test_targets_subset_matches_full(orc):
    p, _ = ics.plummer(500, 9)
    acc, pot = orc.accel(p, 0.01)
    t = ics.sample_targets(500, 37, 10)
    a2, p2 = orc.accel(p, 0.01, targets=t)
    assert np.array_equal(a2, acc[t]) and np.array_equal(p2, pot[t])


def test_eps_zero_coincident_bodies_are_inf_or_nan(orc):
    p = np.array([[0.0, 0, 0, 1.0], [0.0, 0, 0, 1.0], [1.0, 0, 0, 1.0]])
    acc, pot = orc.accel(p, 0.0)
    assert not np.isfinite(pot[0]) and not np.isfinite(pot[1])
    assert np.isfinite(pot[2])


def test_plummer_mean_field_and_energy(orc):
    # Physics pin for the sign and magnitude at scale: in a Plummer sphere
    # (M = a = G = 1) the mean radial acceleration at radius r is
    # -r/(r^2+1)^(3/2), the potential energy is -3 pi/32, and the sampled
    # velocities are virialised (2K + U ~ 0).  Discreteness noise at this N
    # is a few per cent.
    n = 6000
    p, v = ics.plummer(n, 11)
    acc, pot = orc.accel(p, 0.01)
    r = np.linalg.norm(p[:, :3], axis=1)
    ar = (acc * p[:, :3]).sum(axis=1) / r
    for lo, hi in [(0.3, 0.6), (0.6, 1.0), (1.0, 1.6), (1.6, 3.0)]:
        sel = (r >= lo) & (r < hi)
        model = -(r[sel] / (r[sel] ** 2 + 1.0) ** 1.5)
        assert abs(ar[sel].mean() / model.mean() - 1.0) < 0.05, (lo, hi)
    K, U = orc.energy(v, p, pot)
    assert abs(U / (-3 * math.pi / 32) - 1.0) < 0.03
    assert abs(2 * K / -U - 1.0) < 0.06
