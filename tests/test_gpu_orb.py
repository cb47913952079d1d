"""ORB order on the device (nbody_orb_order: the paper's Orthogonal
Recursive Bisection of Section IV.B used as a body ordering) must equal the
oracle's order bit for bit."""
import numpy as np
import pytest

import ics
from nbtest import gpu, to_dev

pytestmark = pytest.mark.gpu


def _gpu_perm(torch, nb, pos4, leaf, dtype):
    p = to_dev(torch, pos4, dtype)
    perm = nb.orb_order(p, leaf)
    torch.cuda.synchronize()
    return perm.cpu().numpy()


@pytest.mark.parametrize("n,leaf", [(1, 1), (2, 1), (7, 2), (100, 1), (100, 7), (2049, 16), (4097, 64),
                                    (10000, 1), (10000, 256), (20000, 4096), (65536, 128), (70001, 3),
                                    (3000, 2500), (9000, 2100), (131073, 2), (300007, 5)])
def test_orb_bitexact_plummer(orc, n, leaf):
    torch, nb = gpu()
    pm, _ = ics.plummer(max(n, 2), 200 + n)
    pm = pm[:n].copy()
    want = orc.orb_order(pm, leaf)
    got = _gpu_perm(torch, nb, pm.astype(np.float32), leaf, torch.float32)
    assert np.array_equal(got, want)


def test_orb_f64_input_rounds_to_f32(orc):
    torch, nb = gpu()
    pm, _ = ics.uniform_ball(9000, 210)
    want = orc.orb_order(pm, 32)  # oracle rounds coordinates to FP32
    got = _gpu_perm(torch, nb, pm, 32, torch.float64)
    assert np.array_equal(got, want)


def test_orb_ties_and_signed_zeros(orc):
    torch, nb = gpu()
    g = ics.rng(211)
    for n, leaf in [(5000, 4), (3000, 1), (12000, 64)]:
        pos = np.zeros((n, 4), dtype=np.float32)
        pos[:, :3] = g.integers(-3, 4, size=(n, 3))
        xyz = pos[:, :3]
        xyz[g.random((n, 3)) < 0.3] = 0.0
        neg = g.random((n, 3)) < 0.2
        xyz[neg & (xyz == 0)] = -0.0
        pos[:, :3] = xyz
        assert np.signbit(pos[:, :3][pos[:, :3] == 0]).any()
        want = orc.orb_order(pos, leaf)
        got = _gpu_perm(torch, nb, pos, leaf, torch.float32)
        assert np.array_equal(got, want), (n, leaf)


def test_orb_coincident_bodies(orc):
    """Every body at one point, then at two: every split is decided by the
    index alone, so the tie pass selects over whole segments."""
    torch, nb = gpu()
    g = ics.rng(212)
    for n, leaf, npts in [(6000, 4, 1), (6000, 1000, 1), (9000, 8, 2), (2500, 1, 2)]:
        pos = np.zeros((n, 4), dtype=np.float32)
        pts = g.standard_normal((npts, 3)).astype(np.float32)
        pos[:, :3] = pts[g.integers(0, npts, size=n)]
        pos[:, 3] = 1.0
        want = orc.orb_order(pos, leaf)
        got = _gpu_perm(torch, nb, pos, leaf, torch.float32)
        assert np.array_equal(got, want), (n, leaf, npts)


def test_orb_full_size_collide1m(orc):
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    pm, _ = ics.colliding_pair(w["n"], w["seed"])
    pm32 = pm.astype(np.float32)
    want = orc.orb_order(pm32, 256)
    got = _gpu_perm(torch, nb, pm32, 256, torch.float32)
    assert np.array_equal(got, want)


def test_orb_repeat_and_permute_roundtrip():
    torch, nb = gpu()
    pm, v = ics.plummer(30000, 212)
    p = to_dev(torch, pm, torch.float32)
    a = nb.orb_order(p, 64)
    b = nb.orb_order(p, 64)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    q = nb.permute(p, a)
    back = nb.permute(q, a, inverse=True)
    torch.cuda.synchronize()
    assert torch.equal(back, p)
    assert torch.equal(q, p[a.long()])
    # the force is a function of the set: evaluating in ORB order and scattering
    # back agrees with the unordered evaluation to rounding
    f0 = nb.accel(p, 0.01)
    f1 = nb.permute(nb.accel(q, 0.01), a, inverse=True)
    torch.cuda.synchronize()
    rel = ((f1 - f0).norm(dim=1) / f0.norm(dim=1)).max().item()
    assert rel < 1e-5


def test_orb_rejects_large_leaf():
    torch, nb = gpu()
    p = to_dev(torch, ics.plummer(100, 213)[0], torch.float32)
    with pytest.raises(nb.NBodyError):
        nb.orb_order(p, 5000)


@pytest.mark.parametrize("inverse", [False, True])
@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_permute_skips_entries_outside_range(inverse, dtype_name):
    """An index outside [0, n) in perm is skipped by the gather and the
    scatter: no record is read or written for it, the others are moved."""
    torch, nb = gpu()
    dtype = getattr(torch, dtype_name)
    n = 1000
    src = torch.arange(4 * n, dtype=dtype, device="cuda").reshape(n, 4)
    perm = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")
    bad = [3, 500, 999]
    perm[bad[0]] = -1
    perm[bad[1]] = n
    perm[bad[2]] = 2 ** 31 - 1
    out = torch.full((n, 4), -7.0, dtype=dtype, device="cuda")
    nb.permute(src, perm, inverse=inverse, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = np.full((n, 4), -7.0)
    s = src.cpu().numpy()
    for p in range(n):
        if p in bad:
            continue
        q = n - 1 - p
        if inverse:
            want[q] = s[p]
        else:
            want[p] = s[q]
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_orb_input_check(monkeypatch, dtype_name):
    """With NBODY_CHECK_INPUTS set, non-finite records are refused before any
    ordering work (naming the first one); clean input orders as before."""
    torch, nb = gpu()
    dtype = getattr(torch, dtype_name)
    pm, _ = ics.plummer(5000, 31)
    p = to_dev(torch, pm, dtype)
    ref = nb.orb_order(p, 16)
    monkeypatch.setenv("NBODY_CHECK_INPUTS", "1")
    assert torch.equal(nb.orb_order(p, 16), ref)
    bad = p.clone()
    bad[3000, 3] = float("inf")
    bad[777, 1] = float("nan")
    with pytest.raises(nb.NBodyError, match="record 777 "):
        nb.orb_order(bad, 16)
    bad[777, 1] = 0.0
    with pytest.raises(nb.NBodyError, match="record 3000 "):
        nb.orb_order(bad, 16)
    monkeypatch.setenv("NBODY_CHECK_INPUTS", "0")
    assert torch.equal(nb.orb_order(p, 16), ref)
