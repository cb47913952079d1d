"""Force kernel at the largest body count the library accepts,
n = 2^31 - 4096 (its target and source indices are 32-bit).

No oracle sums 2^62 pairs, so the input is built so that a small case decides
the answer: every body is massless except a few spread over the whole index
range (the first and last records, split and tile boundaries, the target
window itself).  With softening every pair term is finite, so a massless
source adds exactly zero to each partial sum, and the exact force on a
target is the sum over the massive bodies alone (the paper's pair law,
Section IV), which the oracle computes.

The shapes include a source tile of 10^7 records with 32 source splits: the
last tile of the last split then starts within 10^7 of 2^31, where forming
its end as start + tile would leave the int range."""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, max_rel, normwise

pytestmark = pytest.mark.gpu

N_MAX = (1 << 31) - 4096
EPS = 0.01
BIG_TILE = 10_000_000


def _massive(n, window):
    per = -(-n // 32)
    idx = {0, 1, 777, per - 1, per, 1 << 30, 31 * per - 1, 31 * per, 31 * per + 6 * BIG_TILE - 1,
           31 * per + 6 * BIG_TILE, n - 4097, n - 300, n - 2, n - 1,
           int(window[0]), int(window[0]) + 63, int(window[0]) + 64, int(window[-1])}
    return np.array(sorted(i for i in idx if 0 <= i < n), dtype=np.int64)


CASES = [
    # (mode, first target, target count, pinned (tpl, jsplit, jtile) or None)
    ("F32_F64ACC", N_MAX - 256, 256, None),
    ("F32_F64ACC", 0, 256, (1, 32, BIG_TILE)),
    ("F32_KAHAN", N_MAX - 200, 200, (1, 32, BIG_TILE)),
    ("F32", N_MAX - 100, 100, (2, 32, 512)),
    ("F64", N_MAX - 64, 64, (1, 32, BIG_TILE)),
]


@pytest.mark.parametrize("mode,tbeg,tcount,shape", CASES)
def test_accel_at_maximum_n(orc, mode, tbeg, tcount, shape):
    torch, nb = gpu()
    f64 = mode == "F64"
    dtype = torch.float64 if f64 else torch.float32
    need = N_MAX * (32 if f64 else 16)
    free, _ = torch.cuda.mem_get_info()
    if free < need + (4 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    prec = getattr(nb, mode)
    window = np.arange(tbeg, tbeg + tcount, dtype=np.int64)
    heavy = _massive(N_MAX, window)
    keep = np.union1d(heavy, window)

    # the small case: the window's targets (massless unless listed) and the
    # massive bodies, as the exact values the kernel reads
    rec = np.zeros((keep.size, 4))
    tpos, _ = ics.uniform_ball(tcount, 2100 + tcount)
    rec[np.searchsorted(keep, window), :3] = tpos[:, :3]
    hpos, _ = ics.uniform_ball(heavy.size, 2200 + heavy.size)
    rec[np.searchsorted(keep, heavy)] = hpos
    if not f64:
        rec = rec.astype(np.float32).astype(np.float64)
    acc_ref, pot_ref = orc.accel(rec, EPS, targets=np.searchsorted(keep, window))

    pm = torch.zeros((N_MAX, 4), dtype=dtype, device="cuda")
    try:
        pm[torch.as_tensor(keep, device="cuda")] = torch.as_tensor(rec, dtype=dtype, device="cuda")
        if shape is not None:
            nb.set_tuning(0, prec, *shape)
        out = nb.accel(pm, EPS, prec=prec, target_begin=tbeg, target_count=tcount)
        torch.cuda.synchronize()
        got = host(out)
    finally:
        nb.set_tuning(0, prec)
        del pm
        torch.cuda.empty_cache()
    bar = 1e-12 if f64 else 1e-5
    assert normwise(got[:, :3], acc_ref) < bar
    assert normwise(got[:, 3], pot_ref) < bar
    assert max_rel(got[:, :3], acc_ref) < 100 * bar
    assert max_rel(got[:, 3], pot_ref) < 100 * bar
