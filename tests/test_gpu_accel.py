"""Parity of the HIP force/potential kernels (nbody_accel) with the FP64
oracle: the exact softened pair sum of the paper's force calculation
(Section IV.B, Calculate_forces with every body on the interaction list)."""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, max_rel, normwise, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu

MODES32 = ["F32", "F32_KAHAN", "F32_F64ACC"]


def _run(nb, torch, pm_np, eps, prec, dtype, **kw):
    pm = to_dev(torch, pm_np, dtype)
    out = nb.accel(pm, eps, prec=getattr(nb, prec), **kw)
    torch.cuda.synchronize()
    return host(out)


def test_f64_plain_method_ball4096(orc):
    """Uniform ball N = 4096, FP64, eps = 0.01: <= 1e-12 RMS relative."""
    torch, nb = gpu()
    w = ics.WORKLOADS["ball4096_f64"]
    pm, _ = ics.uniform_ball(w["n"], w["seed"])
    out = _run(nb, torch, pm, w["eps"], "F64", torch.float64)
    acc, pot = orc.accel(pm, w["eps"])
    assert rms_rel(out[:, :3], acc) <= 1e-12
    assert rms_rel(out[:, 3], pot) <= 1e-12
    mom = (pm[:, 3:4] * out[:, :3]).sum(axis=0)
    assert np.linalg.norm(mom) / (pm[:, 3] * np.linalg.norm(out[:, :3], axis=1)).sum() <= 1e-13


@pytest.mark.parametrize("mode", MODES32)
def test_f32_modes_plummer65536_sampled(orc, mode):
    """Plummer N = 65536, eps = 0.01, 1024 sampled targets: compensated modes
    <= 1e-5 RMS relative, pure FP32 reported with a looser bar."""
    torch, nb = gpu()
    w = ics.WORKLOADS["plummer65536"]
    pm, _ = ics.plummer(w["n"], w["seed"])
    pm32 = widen32(pm)
    tg = ics.sample_targets(w["n"], 1024, w["seed"] + 1)
    out = _run(nb, torch, pm32, w["eps"], mode, torch.float32)
    acc, pot = orc.accel(pm32, w["eps"], targets=tg)
    e_a = rms_rel(out[tg, :3], acc)
    e_p = rms_rel(out[tg, 3], pot)
    print(f"{mode}: force rms rel {e_a:.3e} max {max_rel(out[tg, :3], acc):.3e}; pot rms rel {e_p:.3e}")
    bar = 1e-4 if mode == "F32" else 1e-5
    assert e_a <= bar and e_p <= bar


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 257, 1000, 4097])
@pytest.mark.parametrize("mode", ["F64"] + MODES32)
def test_ragged_sizes(orc, n, mode):
    torch, nb = gpu()
    pm, _ = ics.plummer(max(n, 2), 100 + n)
    pm = pm[:n].copy()
    pm[:, 3] *= np.linspace(0.5, 1.5, n)
    dtype = torch.float64 if mode == "F64" else torch.float32
    src = pm if mode == "F64" else widen32(pm)
    out = _run(nb, torch, src, 0.02, mode, dtype)
    acc, pot = orc.accel(src, 0.02)
    if n == 1:
        assert np.all(out == 0.0)
        return
    bar = 1e-12 if mode == "F64" else 2e-6
    assert rms_rel(out[:, :3], acc) <= bar
    assert rms_rel(out[:, 3], pot) <= bar


@pytest.mark.parametrize("tpl,js,jt", [(1, 1, 8), (2, 3, 64), (4, 5, 256), (1, 32, 2048), (2, 8, 16), (1, 24, 64)])
@pytest.mark.parametrize("mode", ["F64", "F32_KAHAN", "F32"])
def test_kernel_shapes(orc, tpl, js, jt, mode):
    """Every tuning shape gives the same answer (to rounding) as the oracle.
    (The sources fit in one XCD's L2 here, so every shape keeps the plain
    workgroup order; test_xcd_order_shapes covers the XCD order.)"""
    torch, nb = gpu()
    if mode == "F64" and tpl == 4:
        pytest.skip("FP64 kernel has tpl 1 and 2")
    n = 3001
    pm, _ = ics.uniform_ball(n, 7)
    prec = getattr(nb, mode)
    nb.set_tuning(0, prec, tpl, js, jt)
    try:
        dtype = torch.float64 if mode == "F64" else torch.float32
        src = pm if mode == "F64" else widen32(pm)
        out = _run(nb, torch, src, 0.01, mode, dtype)
    finally:
        nb.set_tuning(0, prec)
    acc, pot = orc.accel(src, 0.01)
    bar = 1e-12 if mode == "F64" else 2e-6
    assert rms_rel(out[:, :3], acc) <= bar and rms_rel(out[:, 3], pot) <= bar


@pytest.mark.parametrize("mode,n,tpl,js,jt", [("F32_F64ACC", 300001, 1, 8, 512), ("F32_KAHAN", 300001, 2, 24, 256),
                                             ("F32", 300001, 1, 32, 512), ("F64", 150001, 1, 8, 512),
                                             ("F64", 150001, 2, 16, 64)])
def test_xcd_order_shapes(orc, mode, n, tpl, js, jt):
    """Split counts that are multiples of 8, over sources larger than one
    XCD's 4 MiB L2, take the XCD workgroup order (XCD x runs splits x J/8 to
    (x + 1) J/8 - 1): 8, 16, 24 and 32 splits (one to four per XCD), ragged
    target counts, FP32 and FP64 records.  Every output record is written
    and sampled targets match the oracle."""
    torch, nb = gpu()
    pm, _ = ics.plummer(n, 11 + js)
    dtype = torch.float64 if mode == "F64" else torch.float32
    src = pm if mode == "F64" else widen32(pm)
    prec = getattr(nb, mode)
    nb.set_tuning(0, prec, tpl, js, jt)
    try:
        p = to_dev(torch, src, dtype)
        out = torch.full_like(p, float("nan"))
        nb.accel(p, 0.01, prec=prec, out=out)
        torch.cuda.synchronize()
    finally:
        nb.set_tuning(0, prec)
    got = host(out)
    assert np.isfinite(got).all()
    tg = ics.sample_targets(n, 256, 5 + js)
    acc, pot = orc.accel(src, 0.01, targets=tg)
    bar = 1e-12 if mode == "F64" else (1e-5 if mode == "F32" else 2e-6)
    assert rms_rel(got[tg, :3], acc) <= bar and rms_rel(got[tg, 3], pot) <= bar


def test_xcd_order_target_subset(orc):
    """A target range (one GPU's share) over sources larger than an XCD's L2,
    split 8 ways in the XCD order: the records of exactly the requested
    targets are written and match the oracle."""
    torch, nb = gpu()
    n, tb, tc = 300001, 1000, 200001
    pm, _ = ics.plummer(n, 23)
    src = widen32(pm)
    nb.set_tuning(0, nb.F32_F64ACC, 1, 8, 512)
    try:
        p = to_dev(torch, src, torch.float32)
        out = torch.full((tc, 4), float("nan"), dtype=torch.float32, device=p.device)
        nb.accel(p, 0.01, prec=nb.F32_F64ACC, target_begin=tb, target_count=tc, out=out)
        torch.cuda.synchronize()
    finally:
        nb.set_tuning(0, nb.F32_F64ACC)
    got = host(out)
    assert np.isfinite(got).all()
    k = ics.sample_targets(tc, 256, 29)
    acc, pot = orc.accel(src, 0.01, targets=tb + k)
    assert rms_rel(got[k, :3], acc) <= 2e-6 and rms_rel(got[k, 3], pot) <= 2e-6


@pytest.mark.parametrize("mode", ["F64", "F32_KAHAN"])
def test_target_subsets(orc, mode):
    torch, nb = gpu()
    n = 2000
    pm, _ = ics.plummer(n, 8)
    dtype = torch.float64 if mode == "F64" else torch.float32
    src = pm if mode == "F64" else widen32(pm)
    full = _run(nb, torch, src, 0.01, mode, dtype)
    for tb, tc in [(0, 1), (5, 300), (1999, 1), (700, 1300), (123, 0)]:
        part = _run(nb, torch, src, 0.01, mode, dtype, target_begin=tb, target_count=tc)
        assert part.shape[0] == tc
        # the same wave shape covers different target ranges; only rounding
        # order at tile edges can differ from the full evaluation
        if tc:
            acc, pot = orc.accel(src, 0.01, targets=np.arange(tb, tb + tc))
            bar = 1e-12 if mode == "F64" else 2e-6
            assert rms_rel(part[:, :3], acc) <= bar


def test_deterministic_and_mirror_exact():
    torch, nb = gpu()
    pm, _ = ics.plummer(5000, 9)
    for mode in ["F64", "F32", "F32_KAHAN", "F32_F64ACC"]:
        dtype = torch.float64 if mode == "F64" else torch.float32
        a = _run(nb, torch, pm, 0.01, mode, dtype)
        b = _run(nb, torch, pm, 0.01, mode, dtype)
        assert np.array_equal(a, b), mode
        q = pm.copy()
        q[:, :3] = -q[:, :3]
        c = _run(nb, torch, q, 0.01, mode, dtype)
        assert np.array_equal(c[:, :3], -a[:, :3]) and np.array_equal(c[:, 3], a[:, 3]), mode


@pytest.mark.parametrize("mode", ["F64", "F32", "F32_KAHAN", "F32_F64ACC"])
def test_power_of_two_scaling_exact(mode):
    """Mass enters each pair term linearly: doubling every mass doubles a and
    phi bit for bit.  Doubling positions and eps scales every pair distance by
    2, so a becomes a / 4 and phi becomes phi / 2, exactly as long as the
    hardware reciprocal square root commutes with powers of four."""
    torch, nb = gpu()
    pm, _ = ics.plummer(3000, 19)
    dtype = torch.float64 if mode == "F64" else torch.float32
    src = pm if mode == "F64" else widen32(pm)
    a = _run(nb, torch, src, 0.01, mode, dtype)
    heavy = src.copy()
    heavy[:, 3] *= 2.0
    b = _run(nb, torch, heavy, 0.01, mode, dtype)
    assert np.array_equal(b, 2.0 * a)
    wide = src.copy()
    wide[:, :3] *= 2.0
    c = _run(nb, torch, wide, 0.02, mode, dtype)
    assert np.array_equal(c[:, :3], a[:, :3] / 4.0)
    assert np.array_equal(c[:, 3], a[:, 3] / 2.0)


def test_closed_forms_on_gpu():
    """Cube vertices (eps = 0): a = -(1/4 + 1/(4 sqrt2) + 1/(12 sqrt3)) G m x."""
    torch, nb = gpu()
    pts = np.array([[sx, sy, sz, 0.5] for sx in (-1.0, 1.0) for sy in (-1.0, 1.0) for sz in (-1.0, 1.0)])
    amag = 0.25 + 1 / (4 * np.sqrt(2)) + 1 / (12 * np.sqrt(3))
    out = _run(nb, torch, pts, 0.0, "F64", torch.float64)
    np.testing.assert_allclose(out[:, :3], -0.5 * amag * pts[:, :3], rtol=1e-14)
    out = _run(nb, torch, pts, 0.0, "F32_KAHAN", torch.float32)
    np.testing.assert_allclose(out[:, :3], -0.5 * amag * pts[:, :3], rtol=1e-6)


def test_eps_zero_and_coincident():
    torch, nb = gpu()
    pm = np.array([[0.0, 0, 0, 1.0], [0.0, 0, 0, 1.0], [1.0, 0, 0, 1.0]])
    out = _run(nb, torch, pm, 0.0, "F32_KAHAN", torch.float32)
    assert not np.isfinite(out[0, 3]) and not np.isfinite(out[1, 3])
    pm[1, 0] = 2.0
    out = _run(nb, torch, pm, 0.0, "F32_KAHAN", torch.float32)
    assert np.all(np.isfinite(out))
    np.testing.assert_allclose(out[0, 3], -1.5, rtol=1e-6)


def test_energy_entry_point(orc):
    torch, nb = gpu()
    pm, v = ics.plummer(3000, 12)
    for mode, dtype in [("F64", torch.float64), ("F32_KAHAN", torch.float32)]:
        p = to_dev(torch, pm, dtype)
        vv = to_dev(torch, v, dtype)
        a = nb.accel(p, 0.01, prec=getattr(nb, mode))
        e = nb.energy(p, vv, a).cpu().numpy()
        K, U = orc.energy(host(vv), host(p), host(a)[:, 3])
        np.testing.assert_allclose(e, [K, U], rtol=1e-12)


def test_full_size_collide1m_sampled(orc):
    """Two colliding Plummer spheres, N = 2^20, eps = 0.005, FP32 with FP64
    cross-tile sums, the launch shape the benchmark uses: sampled targets."""
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    pm, _ = ics.colliding_pair(w["n"], w["seed"])
    pm32 = widen32(pm)
    tg = ics.sample_targets(w["n"], 256, w["seed"] + 1)
    acc, pot = orc.accel(pm32, w["eps"], targets=tg)
    for mode in ["F32_F64ACC", "F32_KAHAN", "F32"]:
        out = _run(nb, torch, pm32, w["eps"], mode, torch.float32)
        e = rms_rel(out[tg, :3], acc)
        print(f"collide1m {mode}: force rms rel {e:.3e}, pot rms rel {rms_rel(out[tg, 3], pot):.3e}")
        # every FP32 mode sums per-tile partials, pure FP32 too: all meet 1e-5
        assert e <= 1e-5
        assert rms_rel(out[tg, 3], pot) <= 1e-5


@pytest.mark.parametrize("mode", ["F32", "F32_KAHAN", "F32_F64ACC"])
@pytest.mark.parametrize("tpl,js,jt", [(1, 1, 256), (2, 3, 512), (4, 1, 1024), (1, 7, 256), (2, 16, 256)])
def test_lds_variant_equals_scalar_variant(orc, mode, tpl, js, jt):
    """Sources staged in LDS give bit for bit the result of the scalar-load
    sweep (same arithmetic, same order), including ragged tails, the masked
    self range and inactive waves of the last workgroup."""
    torch, nb = gpu()
    prec = getattr(nb, mode)
    for n in (1, 255, 257, 5003):
        pm, _ = ics.plummer(max(n, 2), 300 + n)
        p = to_dev(torch, widen32(pm[:n]), torch.float32)
        try:
            nb.set_tuning(0, prec, tpl, js, jt, 0)
            a = nb.accel(p, 0.01, prec=prec)
            b0 = nb.accel(p, 0.01, prec=prec, target_begin=n // 3, target_count=n - n // 3)
            nb.set_tuning(0, prec, tpl, js, jt, 1)
            b = nb.accel(p, 0.01, prec=prec)
            b1 = nb.accel(p, 0.01, prec=prec, target_begin=n // 3, target_count=n - n // 3)
            torch.cuda.synchronize()
        finally:
            nb.set_tuning(0, prec)
        assert torch.equal(a, b), n
        assert torch.equal(b0, b1), n
        if n > 1:
            acc, pot = orc.accel(widen32(pm[:n]), 0.01)
            bar = 1e-4 if mode == "F32" else 2e-6
            assert rms_rel(host(b)[:, :3], acc) <= bar


def test_caller_outputs_must_fit():
    """A caller-supplied `out` of the wrong row count or dtype is refused in
    the binding before any kernel is launched."""
    torch, nb = gpu()
    p = torch.rand(300, 4, device="cuda")
    perm = torch.arange(300, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        nb.accel(p, 0.01, out=torch.empty(299, 4, device="cuda"))
    with pytest.raises(ValueError):
        nb.accel(p, 0.01, target_begin=100, target_count=50, out=torch.empty(60, 4, device="cuda"))
    with pytest.raises(TypeError):
        nb.accel(p, 0.01, out=torch.empty(300, 4, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        nb.permute(p, perm, out=torch.empty(200, 4, device="cuda"))
    with pytest.raises(ValueError):
        nb.batched_accel(p, [0, 100, 300], 0.01, out=torch.empty(100, 4, device="cuda"))
    with pytest.raises(ValueError):
        nb.tree_accel(p, 0.01, 0.5, out=torch.empty(30, 4, device="cuda"))
    out = torch.empty(50, 4, device="cuda")
    assert nb.accel(p, 0.01, target_begin=100, target_count=50, out=out) is out


def test_scratch_growth_does_not_wait():
    """A call that needs a larger split buffer than any earlier one gets a
    new buffer without waiting for the work that may still use the old one:
    it returns while a 2^19-body force launch is still running, and that
    launch's result equals a later evaluation bit for bit."""
    import time
    torch, nb = gpu()
    mode = nb.F32_F64ACC
    nb.release()  # no library scratch yet
    nb.set_tuning(0, mode, tpl=1, jsplit=8, jtile=512)
    try:
        pm1, _ = ics.plummer(1 << 19, 750)
        pm2, _ = ics.plummer(1 << 20, 751)
        q1 = to_dev(torch, pm1, torch.float32)
        q2 = to_dev(torch, pm2, torch.float32)
        out2 = torch.empty((q2.shape[0], 4), dtype=torch.float32, device=q2.device)
        torch.cuda.synchronize()
        out1 = nb.accel(q1, 0.01, prec=mode)  # about 75 ms on the device
        t0 = time.perf_counter()
        nb.accel(q2, 0.01, prec=mode, out=out2)  # twice the split scratch of the call before
        waited = time.perf_counter() - t0
        torch.cuda.synchronize()
        again = nb.accel(q1, 0.01, prec=mode)
        torch.cuda.synchronize()
        assert torch.equal(out1, again)
        assert torch.isfinite(out2).all()
        assert waited < 0.03, f"the growing call took {waited * 1e3:.1f} ms on the host"
    finally:
        nb.set_tuning(0, mode)
        nb.release()
