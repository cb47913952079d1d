"""Pins of the oracle's kick-drift-kick leapfrog (paper Section IV.A last
step and the Section IV.B pseudo-code: bodies update velocity and position
from the computed forces after the force calculation) against Kepler
orbits, conservation laws and time symmetry."""
import math

import numpy as np
import pytest

import ics


def _energy(res):
    return res["energy"][:, 0] + res["energy"][:, 1]


def _circular_position(t):
    # circular Kepler pair (a = 1, total mass 1, period 2 pi): body 1 sits at
    # (cos t, sin t)/2 relative to the centre of mass.
    return np.array([0.5 * math.cos(t), 0.5 * math.sin(t)])


def test_circular_orbit_second_order(orc):
    p, v = ics.kepler_pair(0.0)
    errs = []
    for nstep in (200, 400, 800):
        dt = 2 * math.pi / nstep
        res = orc.leapfrog(p, v, 0.0, dt, nstep)
        errs.append(np.linalg.norm(res["x"][1, :2] - _circular_position(2 * math.pi)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, errs


@pytest.mark.parametrize("e", [0.0, 0.5])
def test_kepler_energy_bounded_no_drift(orc, e):
    p, v = ics.kepler_pair(e)
    nper = 200
    res = orc.leapfrog(p, v, 0.0, 2 * math.pi / nper, 10 * nper)
    E = _energy(res)
    rel = np.abs(E / E[0] - 1.0)
    first = rel[: nper + 1].max()
    last = rel[9 * nper:].max()
    assert rel.max() < (5e-3 if e else 1e-3)
    assert last <= 1.5 * first + 1e-15  # bounded oscillation, no secular growth
    # halving dt cuts the energy error about four-fold (second order)
    res2 = orc.leapfrog(p, v, 0.0, 2 * math.pi / (2 * nper), 2 * nper)
    rel2 = np.abs(_energy(res2) / E[0] - 1.0).max()
    if e:
        assert 3.5 < first / rel2 < 4.5


def test_angular_momentum_conserved(orc):
    p, v = ics.plummer(64, 21)
    res = orc.leapfrog(p, v, 0.05, 1e-2, 50)
    L0 = (p[:, 3:4] * np.cross(p[:, :3], v[:, :3])).sum(axis=0)
    L1 = (p[:, 3:4] * np.cross(res["x"], res["v"])).sum(axis=0)
    scale = (p[:, 3] * np.linalg.norm(np.cross(p[:, :3], v[:, :3]), axis=1)).sum()
    assert np.linalg.norm(L1 - L0) <= 1e-13 * scale


def test_time_reversal(orc):
    # KDK is time-symmetric: reverse the velocities and integrate again to
    # land back on the initial positions, up to rounding.
    p, v = ics.plummer(48, 22)
    res = orc.leapfrog(p, v, 0.05, 1e-2, 30)
    q = p.copy()
    q[:, :3] = res["x"]
    w = np.zeros_like(v)
    w[:, :3] = -res["v"]
    back = orc.leapfrog(q, w, 0.05, 1e-2, 30)
    assert np.abs(back["x"] - p[:, :3]).max() < 1e-12
    assert np.abs(back["v"] + v[:, :3]).max() < 1e-12


def test_free_particles_move_straight(orc):
    # G = 0: no force, x(T) = x0 + T v0 exactly up to one rounding per step
    p, v = ics.plummer(10, 23)
    res = orc.leapfrog(p, v, 0.01, 0.125, 8, G=0.0)
    np.testing.assert_allclose(res["x"], p[:, :3] + 1.0 * v[:, :3], rtol=0, atol=1e-14)
    assert np.array_equal(res["v"], v[:, :3])


def test_energy_at_rest_is_potential_only(orc):
    p, v = ics.uniform_ball(256, 24)
    res = orc.leapfrog(p, v, 0.01, 1e-3, 0)
    assert res["energy"][0, 0] == 0.0
    _, pot = orc.accel(p, 0.01)
    np.testing.assert_allclose(res["energy"][0, 1], 0.5 * (p[:, 3] * pot).sum(), rtol=1e-14)
