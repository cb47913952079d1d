"""nbody_accel_noalloc, the force entry point that allocates nothing, called
through the C ABI and checked against nbody_accel on the same inputs: two
calls in a row (the second smaller), each equal to nbody_accel bit for bit
while the split partials fit the static device array; a shape whose
partials would not fit runs with fewer splits and stays within the force
bar of the FP64 oracle."""
import ctypes

import numpy as np
import pytest

import ics
from nbtest import gpu, host, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu


def _c(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(torch, nb, p, prec, eps, tb, tc):
    L = nb.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ref = torch.full((tc, 4), float("nan"), dtype=p.dtype, device=p.device)
    got = torch.full((tc, 4), float("nan"), dtype=p.dtype, device=p.device)
    n = p.shape[0]
    assert L.nbody_accel(_c(p), n, prec, 1.0, eps, _c(ref), tb, tc, st) == 0
    assert L.nbody_accel_noalloc(_c(p), n, prec, 1.0, eps, _c(got), tb, tc, st) == 0
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("mode", ["F32_KAHAN", "F32_F64ACC", "F32", "F64"])
def test_noalloc_equals_accel_two_calls(orc, mode):
    torch, nb = gpu()
    prec = getattr(nb, mode)
    dt = torch.float64 if mode == "F64" else torch.float32
    eps = 0.01
    for n, tb, tc in [(40001, 0, 40001), (5003, 1000, 3000)]:
        print(f"noalloc {mode} n={n} targets [{tb}, {tb + tc})", flush=True)
        pm, _ = ics.plummer(n, 900 + n)
        pm = pm if mode == "F64" else widen32(pm)
        p = to_dev(torch, pm, dt)
        assert nb.get_tuning(0, prec, n)[1] > 1  # the split path, so the static array is used
        ref, got = _both(torch, nb, p, prec, eps, tb, tc)
        assert torch.equal(ref, got)
        tg = ics.sample_targets(tc, min(tc, 512), n)
        acc, pot = orc.accel(pm, eps, targets=tb + tg)
        bar = 1e-12 if mode == "F64" else 1e-5
        assert rms_rel(host(got)[tg, :3], acc) <= bar
        assert rms_rel(host(got)[tg, 3], pot) <= bar


def test_noalloc_fewer_splits_when_partials_do_not_fit(orc):
    """2^17 + 64 targets: the default shape's 32 splits need 134 MB of
    partials; the call runs with fewer splits (grouping differs, so equality
    is to the force bar, not bitwise)."""
    torch, nb = gpu()
    n = (1 << 17) + 64
    eps = 0.01
    pm, _ = ics.plummer(n, 4242)
    pm = widen32(pm)
    p = to_dev(torch, pm, torch.float32)
    js = nb.get_tuning(0, nb.F32_KAHAN, n)[1]
    assert js * n * 32 > (64 << 20)
    print(f"noalloc clamp n={n} default jsplit {js}", flush=True)
    ref, got = _both(torch, nb, p, nb.F32_KAHAN, eps, 0, n)
    assert not torch.isnan(got).any()
    assert rms_rel(host(got)[:, :3], host(ref)[:, :3]) <= 1e-6
    tg = ics.sample_targets(n, 256, 4243)
    acc, pot = orc.accel(pm, eps, targets=tg)
    assert rms_rel(host(got)[tg, :3], acc) <= 1e-5
    assert rms_rel(host(got)[tg, 3], pot) <= 1e-5
