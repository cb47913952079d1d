"""Parity of the leapfrog driver (nbody_leapfrog_kdk: Move_bodies after the
force calculation, Section IV.B, as kick-drift-kick) and of its HIP-graph
capture with the oracle and with eager launches."""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu


def test_ball4096_f64_ten_steps(orc):
    """One force evaluation then 10 KDK steps, dt = 1e-3, FP64: <= 1e-12."""
    torch, nb = gpu()
    w = ics.WORKLOADS["ball4096_f64"]
    pm, v = ics.uniform_ball(w["n"], w["seed"])
    p = to_dev(torch, pm, torch.float64)
    vv = to_dev(torch, v, torch.float64)
    a = torch.empty_like(p)
    en = nb.leapfrog_kdk(p, vv, a, w["eps"], w["dt"], w["steps"], energy=True)
    torch.cuda.synchronize()
    ref = orc.leapfrog(pm, v, w["eps"], w["dt"], w["steps"])
    assert rms_rel(host(p)[:, :3], ref["x"]) <= 1e-12
    assert rms_rel(host(vv)[:, :3], ref["v"]) <= 1e-12
    assert rms_rel(host(a)[:, :3], ref["acc"]) <= 1e-12
    assert rms_rel(host(a)[:, 3], ref["pot"]) <= 1e-12
    e = en.cpu().numpy()
    assert e[0, 0] == 0.0
    np.testing.assert_allclose(e[:, 1], ref["energy"][:, 1], rtol=1e-12)
    np.testing.assert_allclose(e[1:, 0], ref["energy"][1:, 0], rtol=1e-10)


@pytest.mark.parametrize("mode", ["F32_KAHAN", "F32_F64ACC", "F32"])
def test_f32_modes_few_steps(orc, mode):
    torch, nb = gpu()
    pm, v = ics.plummer(8192, 50)
    p = to_dev(torch, pm, torch.float32)
    vv = to_dev(torch, v, torch.float32)
    a = torch.empty_like(p)
    en = nb.leapfrog_kdk(p, vv, a, 0.01, 1e-3, 5, prec=getattr(nb, mode), energy=True)
    torch.cuda.synchronize()
    ref = orc.leapfrog(widen32(pm), widen32(v), 0.01, 1e-3, 5)
    assert rms_rel(host(p)[:, :3], ref["x"]) <= 1e-6
    # force at the GPU's own final state
    acc, pot = orc.accel(host(p), 0.01, targets=np.arange(0, 8192, 8))
    assert rms_rel(host(a)[::8, :3], acc) <= (1e-4 if mode == "F32" else 1e-5)
    e = en.cpu().numpy().sum(axis=1)
    assert abs(e[-1] / e[0] - 1) < 1e-5


def test_kepler_orbit_on_gpu():
    """Circular Kepler pair (period 2 pi), FP64: back at the start after one
    period to O(dt^2)."""
    torch, nb = gpu()
    pm, v = ics.kepler_pair(0.0)
    for nstep, tol in [(400, 2e-3), (800, 5e-4)]:
        p = to_dev(torch, pm, torch.float64)
        vv = to_dev(torch, v, torch.float64)
        a = torch.empty_like(p)
        nb.leapfrog_kdk(p, vv, a, 0.0, 2 * np.pi / nstep, nstep)
        torch.cuda.synchronize()
        assert np.abs(host(p)[:, :3] - pm[:, :3]).max() < tol


@pytest.mark.parametrize("mode", ["F32_KAHAN", "F64"])
def test_graph_replays_match_eager(mode):
    """Captured step loop == eager launches, bitwise, on every replay, with
    eager work and synchronisation between replays."""
    torch, nb = gpu()
    dtype = torch.float64 if mode == "F64" else torch.float32
    prec = getattr(nb, mode)
    pm, v = ics.plummer(3000, 51)
    pg, vg = to_dev(torch, pm, dtype), to_dev(torch, v, dtype)
    pe, ve = pg.clone(), vg.clone()
    ag, ae = torch.empty_like(pg), torch.empty_like(pe)
    eg = torch.empty((8, 2), dtype=torch.float64, device="cuda")
    ee = torch.empty_like(eg)
    for rep in range(4):
        nb.leapfrog_kdk(pg, vg, ag, 0.01, 1e-3, 7, prec=prec, graph=True, energy=True, energy_out=eg)
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()  # unrelated eager work
        nb.leapfrog_kdk(pe, ve, ae, 0.01, 1e-3, 7, prec=prec, graph=False, energy=True, energy_out=ee)
        torch.cuda.synchronize()
        assert torch.equal(pg, pe) and torch.equal(vg, ve) and torch.equal(ag, ae), rep
        assert torch.equal(eg, ee), rep
        del junk


def test_acc_valid_flag_skips_first_evaluation():
    torch, nb = gpu()
    pm, v = ics.plummer(2000, 52)
    p1, v1 = to_dev(torch, pm, torch.float32), to_dev(torch, v, torch.float32)
    p2, v2 = p1.clone(), v1.clone()
    a1, a2 = torch.empty_like(p1), torch.empty_like(p1)
    nb.leapfrog_kdk(p1, v1, a1, 0.01, 1e-3, 6)
    nb.leapfrog_kdk(p2, v2, a2, 0.01, 1e-3, 3)
    nb.leapfrog_kdk(p2, v2, a2, 0.01, 1e-3, 3, acc_valid=True)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(v1, v2) and torch.equal(a1, a2)
