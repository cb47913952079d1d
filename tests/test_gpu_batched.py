"""Ragged batches (nbody_batched_accel: many independent systems in one
persistent launch) against standalone evaluations and the oracle."""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu


def _batch(sizes, seed):
    ps, vs = [], []
    for k, s in enumerate(sizes):
        p, v = ics.plummer(max(int(s), 2), seed + k)
        ps.append(p[:s])
        vs.append(v[:s])
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return np.concatenate(ps), np.concatenate(vs), off


SIZES = [1, 64, 65, 300, 2, 3000, 777, 128, 1, 5000, 129, 256]


@pytest.mark.parametrize("mode", ["F32_KAHAN", "F32", "F32_F64ACC", "F64"])
@pytest.mark.parametrize("tpl", [1, 2])
def test_batched_equals_standalone_bitwise(orc, mode, tpl):
    torch, nb = gpu()
    prec = getattr(nb, mode)
    dtype = torch.float64 if mode == "F64" else torch.float32
    pm, _, off = _batch(SIZES, 70)
    nb.set_tuning(0, prec, tpl, 1, 256)
    nb.set_tuning(1, prec, tpl, 1, 256)
    try:
        p = to_dev(torch, pm, dtype)
        out = nb.batched_accel(p, off, 0.01, prec=prec)
        out2 = nb.batched_accel(p, off, 0.01, prec=prec)  # counters reset by the kernel itself
        torch.cuda.synchronize()
        assert torch.equal(out, out2)
        for s in range(len(SIZES)):
            a, b = off[s], off[s + 1]
            ref = nb.accel(p[a:b].contiguous(), 0.01, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(out[a:b], ref), s
    finally:
        nb.set_tuning(0, prec)
        nb.set_tuning(1, prec)
    o = host(out)
    src = pm if mode == "F64" else widen32(pm)
    for s in [1, 3, 5, 9]:
        a, b = off[s], off[s + 1]
        acc, pot = orc.accel(src[a:b], 0.01)
        bar = 1e-12 if mode == "F64" else (1e-4 if mode == "F32" else 2e-6)
        assert rms_rel(o[a:b, :3], acc) <= bar


def test_batched_eps_per_system(orc):
    torch, nb = gpu()
    pm, _, off = _batch([100, 2000, 513], 71)
    eps = np.array([0.01, 0.05, 0.001], dtype=np.float32)
    p = to_dev(torch, pm, torch.float32)
    out = host(nb.batched_accel(p, off, 0.5, eps_per_sys=torch.as_tensor(eps).cuda()))
    for s in range(3):
        a, b = off[s], off[s + 1]
        acc, pot = orc.accel(widen32(pm[a:b]), float(eps[s]))
        assert rms_rel(out[a:b, :3], acc) <= 2e-6


def test_ragged_512_systems_sampled(orc):
    """512 Plummer systems, N_s log-uniform in [256, 32768], FP32 + Kahan:
    sampled (system, target) pairs against the oracle."""
    torch, nb = gpu()
    w = ics.WORKLOADS["batch512"]
    pm, v, off = ics.ragged_batch(w["nsys"], w["seed"])
    p = to_dev(torch, pm, torch.float32)
    out = host(nb.batched_accel(p, off, w["eps"]))
    g = ics.rng(w["seed"] + 1)
    errs = []
    for s in g.choice(w["nsys"], 16, replace=False):
        a, b = off[s], off[s + 1]
        tg = ics.sample_targets(b - a, 64, int(s))
        acc, _ = orc.accel(widen32(pm[a:b]), w["eps"], targets=tg)
        errs.append(rms_rel(out[a + tg, :3], acc))
    assert max(errs) <= 1e-5


def test_batched_leapfrog_graph_matches_eager():
    torch, nb = gpu()
    pm, v, off = _batch([300, 1000, 64, 2500], 72)
    prec = nb.F32_KAHAN
    pg, vg = to_dev(torch, pm, torch.float32), to_dev(torch, v, torch.float32)
    pe, ve = pg.clone(), vg.clone()
    ag, ae = torch.empty_like(pg), torch.empty_like(pe)
    for rep in range(3):
        nb.leapfrog_kdk(pg, vg, ag, 0.01, 1e-3, 5, offsets=off, graph=True)
        torch.cuda.synchronize()
        nb.leapfrog_kdk(pe, ve, ae, 0.01, 1e-3, 5, offsets=off, graph=False)
        torch.cuda.synchronize()
        assert torch.equal(pg, pe) and torch.equal(vg, ve) and torch.equal(ag, ae), rep
    # systems do not feel each other: equals per-system leapfrogs
    nb.set_tuning(0, prec, *nb.get_tuning(1, prec, pm.shape[0]))
    try:
        p0, v0 = to_dev(torch, pm, torch.float32), to_dev(torch, v, torch.float32)
        a0 = torch.empty_like(p0)
        nb.leapfrog_kdk(p0, v0, a0, 0.01, 1e-3, 15, offsets=off)
        for s in range(4):
            a, b = off[s], off[s + 1]
            ps, vs = p0.new_tensor(pm[a:b]), v0.new_tensor(v[a:b])
            acs = torch.empty_like(ps)
            nb.leapfrog_kdk(ps, vs, acs, 0.01, 1e-3, 15)
            torch.cuda.synchronize()
            assert torch.equal(ps, p0[a:b]) and torch.equal(vs, v0[a:b]), s
    finally:
        nb.set_tuning(0, prec)


@pytest.mark.parametrize("mode", ["F32_KAHAN", "F64"])
def test_batched_with_empty_systems(orc, mode):
    """Systems of zero bodies (first, last and in between) take no work and
    leave the other systems' results as their standalone evaluations; the
    batched leapfrog steps over them too."""
    torch, nb = gpu()
    prec = getattr(nb, mode)
    dtype = torch.float64 if mode == "F64" else torch.float32
    sizes = [0, 5, 0, 0, 70, 1, 0]
    pm, vel, off = _batch(sizes, 90)
    p = to_dev(torch, pm, dtype)
    # the standalone kernel in the batched kernel's shape (one source range)
    nb.set_tuning(0, prec, *nb.get_tuning(1, prec, pm.shape[0]))
    try:
        out = nb.batched_accel(p, off, 0.01, prec=prec)
        torch.cuda.synchronize()
        for s in range(len(sizes)):
            a, b = off[s], off[s + 1]
            if b > a:
                ref = nb.accel(p[a:b].contiguous(), 0.01, prec=prec)
                torch.cuda.synchronize()
                assert torch.equal(out[a:b], ref), s
        v = to_dev(torch, vel, dtype)
        pb, vb, ab = p.clone(), v.clone(), torch.empty_like(p)
        nb.leapfrog_kdk(pb, vb, ab, 0.01, 1e-3, 3, prec=prec, offsets=off)
        singles = {}
        for s in (1, 4):
            a, b = off[s], off[s + 1]
            ps, vs, as_ = p[a:b].clone(), v[a:b].clone(), torch.empty_like(p[a:b])
            nb.leapfrog_kdk(ps, vs, as_, 0.01, 1e-3, 3, prec=prec)
            singles[s] = (ps, vs)
        torch.cuda.synchronize()
    finally:
        nb.set_tuning(0, prec)
    src = pm if mode == "F64" else widen32(pm)
    acc, _ = orc.accel(src[off[4]:off[5]], 0.01)
    assert rms_rel(host(out)[off[4]:off[5], :3], acc) <= (1e-12 if mode == "F64" else 2e-6)
    # the batched leapfrog: each non-empty system as if alone
    for s, (ps, vs) in singles.items():
        a, b = off[s], off[s + 1]
        assert torch.equal(pb[a:b], ps), s
        assert torch.equal(vb[a:b], vs), s


def test_empty_target_range():
    """target_count = 0 is a valid call that writes nothing."""
    torch, nb = gpu()
    p = to_dev(torch, ics.plummer(100, 91)[0], torch.float32)
    out = nb.accel(p, 0.01, target_begin=40, target_count=0)
    torch.cuda.synchronize()
    assert out.shape == (0, 4)
    sentinel = torch.full((5, 4), 7.0, device="cuda")
    nb.accel(p, 0.01, target_begin=100, target_count=0, out=sentinel[:0])
    torch.cuda.synchronize()
    assert torch.all(sentinel == 7.0)
