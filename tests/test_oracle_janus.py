"""Pins of the oracle's bit-reversible fixed-point kick-drift-kick (the
integer-state reading of the leapfrog used for exact reverse reconstruction
in the adjoint): exact reversal, agreement with the plain FP64 leapfrog to
the fixed-point resolution, and the integer closed form of force-free
motion."""
import numpy as np
import pytest

import ics


@pytest.mark.parametrize("n,steps,sx,sv", [(1, 5, 40, 40), (64, 30, 40, 40), (300, 25, 36, 44), (2, 100, 50, 30)])
def test_exact_reversal(orc, n, steps, sx, sv):
    pm, v = ics.plummer(max(n, 2), 500 + n)
    pm, v = pm[:n], v[:n]
    st0 = orc.janus_encode(pm, v, sx, sv)
    st1 = orc.janus_run(st0, pm[:, 3], 0.05, 2e-3, steps, sx, sv)
    assert not np.array_equal(st0, st1) or n == 1
    st2 = orc.janus_run(st1, pm[:, 3], 0.05, 2e-3, steps, sx, sv, direction=-1)
    assert np.array_equal(st0, st2)


def test_tracks_the_leapfrog(orc):
    """Each kick and drift rounds to 2^-40, so after 40 steps the state is the
    FP64 leapfrog's to about steps x 2^-40."""
    pm, v = ics.plummer(400, 510)
    x0 = np.ldexp(np.rint(np.ldexp(pm[:, :3], 40)), -40)
    v0 = np.ldexp(np.rint(np.ldexp(v[:, :3], 40)), -40)
    pm2 = pm.copy(); pm2[:, :3] = x0
    st = orc.janus_run(orc.janus_encode(pm2, v0), pm[:, 3], 0.05, 1e-3, 40)
    r = orc.leapfrog(pm2, v0, 0.05, 1e-3, 40)
    assert np.abs(np.ldexp(st[:, :3].astype(np.float64), -40) - r["x"]).max() < 40 * 2.0 ** -40 * 4
    assert np.abs(np.ldexp(st[:, 4:7].astype(np.float64), -40) - r["v"]).max() < 1e-9


def test_force_free_closed_form(orc):
    """G = 0: no kick changes V, every drift adds round(V dt 2^(sx-sv))."""
    pm, v = ics.uniform_ball(50, 520)
    v = ics.rng(521).standard_normal((50, 3))
    st0 = orc.janus_encode(pm, v, 40, 40)
    st = orc.janus_run(st0, pm[:, 3], 0.05, 1e-3, 17, 40, 40, G=0.0)
    inc = np.rint(st0[:, 4:7].astype(np.float64) * 1e-3).astype(np.int64)
    assert np.array_equal(st[:, :3], st0[:, :3] + 17 * inc)
    assert np.array_equal(st[:, 4:7], st0[:, 4:7])
