"""Pins of the oracle's ORB order (paper Section IV.B, Orthogonal Recursive
Bisection into sub-spaces of about equal body counts) against hand-worked
examples and a structural verifier written independently of the oracle."""
import numpy as np
import pytest

import ics
from conftest import golden_path


def _parse(name):
    cases = []
    for line in open(golden_path(name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        leaf, xs, perm = [s.strip() for s in line.split("|")]
        cases.append((int(leaf), [float(t) for t in xs.split()], [int(t) for t in perm.split()]))
    return cases


def test_golden_line(orc):
    for leaf, xs, perm in _parse("orb_line8.txt"):
        pos = np.zeros((len(xs), 3))
        pos[:, 0] = xs
        assert orc.orb_order(pos, leaf).tolist() == perm, leaf


def test_golden_axis_and_ties(orc):
    for leaf, xs, perm in _parse("orb_axis.txt"):
        pos = np.array(xs).reshape(-1, 3)
        assert orc.orb_order(pos, leaf).tolist() == perm, (leaf, xs)


def _tkey(f):
    u = np.asarray(f, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return np.where(u & 0x80000000, (~u) & 0xFFFFFFFF, u | 0x80000000)


def verify_orb(pos32, perm, leaf):
    """Check the structure of an ORB order from the output alone: recursive
    segments split at leaf*ceil(ceil(n/leaf)/2), every key on the left below
    every key on the right along the longest extent, leaves by index."""
    n = pos32.shape[0]
    assert sorted(perm.tolist()) == list(range(n))

    def rec(lo, hi):
        seg = perm[lo:hi]
        cnt = hi - lo
        if cnt <= leaf:
            assert np.all(np.diff(seg) > 0)
            return
        c = pos32[seg]
        ext = (c.max(axis=0) - c.min(axis=0)).astype(np.float32)
        axis = int(np.argmax(ext))  # first maximum = lowest axis on ties
        L = -(-cnt // leaf)
        k = min(cnt, leaf * (-(-L // 2)))
        key = (_tkey(c[:, axis]) << np.uint64(32)) | seg.astype(np.uint64)
        assert key[:k].max() < key[k:].min()
        rec(lo, lo + k)
        rec(lo + k, hi)

    rec(0, n)


@pytest.mark.parametrize("n,leaf", [(1, 1), (2, 1), (7, 2), (8, 8), (9, 8), (1000, 16), (4097, 64), (3000, 1)])
def test_random_structure(orc, n, leaf):
    p, _ = ics.plummer(max(n, 2), 30 + n)
    pos32 = p[:n, :3].astype(np.float32)
    perm = orc.orb_order(pos32, leaf)
    verify_orb(pos32, perm, leaf)


def test_many_ties_and_signed_zeros(orc):
    g = ics.rng(31)
    pos = g.integers(-2, 3, size=(500, 3)).astype(np.float32)
    pos[g.random((500, 3)) < 0.2] = -0.0
    perm = orc.orb_order(pos, 4)
    verify_orb(pos, perm, 4)


def test_tiny_exhaustive(orc):
    # every point set of n <= 6 points on a 3x3x2 grid drawn by the seed; the
    # verifier checks each result
    g = ics.rng(32)
    for trial in range(300):
        n = int(g.integers(1, 9))
        leaf = int(g.integers(1, 4))
        pos = g.integers(0, 3, size=(n, 3)).astype(np.float32)
        verify_orb(pos, orc.orb_order(pos, leaf), leaf)


def test_leaves_full_except_last(orc):
    p, _ = ics.uniform_ball(1000, 33)
    leaf = 64
    perm = orc.orb_order(p, leaf)
    # leaf boundaries fall on multiples of leaf: every leaf but the last is full
    pos32 = p[:, :3].astype(np.float32)
    verify_orb(pos32, perm, leaf)
    for b in range(0, 1000 - leaf, leaf):
        assert np.all(np.diff(perm[b:b + leaf]) > 0)


def test_verifier_rejects_wrong_orders(orc):
    p, _ = ics.plummer(300, 34)
    pos32 = p[:, :3].astype(np.float32)
    perm = orc.orb_order(pos32, 8)
    bad = perm.copy()
    bad[[0, 200]] = bad[[200, 0]]
    with pytest.raises(AssertionError):
        verify_orb(pos32, bad, 8)
    with pytest.raises(AssertionError):
        verify_orb(pos32, np.arange(300, dtype=np.int32), 8)
