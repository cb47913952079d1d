"""The C ABI: the library loads, exports every entry point the header
declares, and rejects bad arguments before enqueueing anything (these calls
return on the host without touching a GPU)."""
import ctypes

import numpy as np
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1211_2292_amd as nb
    if not os.path.exists(nb.LIB_PATH):
        pytest.skip("libnbody.so not built")
    return nb, nb.lib()


def _declared():
    src = open(os.path.join(ROOT, "include", "nbody.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    nb, L = _lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
        assert name in nb._SIGS, name


def test_version_and_status_strings():
    nb, L = _lib()
    assert L.nbody_version() == 100
    for rc in (0, -1, -2, -3, -4, -5):
        assert L.nbody_status_string(rc)


P = ctypes.c_void_p


@pytest.mark.parametrize("args,rc", [
    ((None, 10, 1, 1.0, 0.01, P(64), 0, 10, None), -1),            # NULL input
    ((P(64), 0, 1, 1.0, 0.01, P(128), 0, 0, None), -1),             # n = 0
    ((P(64), 1 << 31, 1, 1.0, 0.01, P(128), 0, 1, None), -1),       # n too large
    ((P(64), 10, 7, 1.0, 0.01, P(128), 0, 10, None), -1),           # bad precision
    ((P(64), 10, 1, 1.0, -0.5, P(1024), 0, 10, None), -1),          # eps < 0
    ((P(64), 10, 1, float("nan"), 0.5, P(1024), 0, 10, None), -1),  # G not finite
    ((P(72), 10, 1, 1.0, 0.01, P(1024), 0, 10, None), -2),          # misaligned float4
    ((P(80), 10, 0, 1.0, 0.01, P(2048), 0, 10, None), -2),          # double4 needs 32 B
    ((P(64), 10, 1, 1.0, 0.01, P(1024), 5, 6, None), -1),           # targets beyond n
    ((P(64), 10, 1, 1.0, 0.01, P(96), 0, 10, None), -1),            # output overlaps input
])
def test_accel_validation(args, rc):
    nb, L = _lib()
    assert L.nbody_accel(*args) == rc
    assert L.nbody_last_error()
    assert L.nbody_accel_noalloc(*args) == rc
    assert L.nbody_last_error()


def test_noalloc_refuses_pinned_split_beyond_static_scratch():
    """A pinned shape whose split partials exceed the static buffer is
    refused on the host, before any device call: 32 splits x 2^17 targets x
    32-byte records = 128 MiB > 64 MiB."""
    nb, L = _lib()
    n = 1 << 17
    assert L.nbody_set_tuning(0, 2, 1, 32, 512, 0) == 0
    try:
        assert L.nbody_accel_noalloc(P(1 << 12), n, 2, 1.0, 0.01, P(1 << 40), 0, n, None) == -1
        msg = L.nbody_last_error()
        msg = msg.decode() if isinstance(msg, bytes) else msg
        assert "static buffer" in msg and str(64 << 20) in msg
    finally:
        assert L.nbody_set_tuning(0, 2, -1, -1, -1, 0) == 0


def test_other_entry_points_validate():
    nb, L = _lib()
    off = (ctypes.c_int64 * 3)(0, 5, 4)  # decreasing
    assert L.nbody_batched_accel(P(64), off, 2, 1, 1.0, None, 0.01, P(1024), None) == -1
    off = (ctypes.c_int64 * 3)(1, 5, 9)  # does not start at 0
    assert L.nbody_batched_accel(P(64), off, 2, 1, 1.0, None, 0.01, P(1024), None) == -1
    assert L.nbody_leapfrog_kdk(P(64), P(1024), P(4096), 10, None, 0, 1, 1.0, 0.01, 1e-3, -1, 0, None, None) == -1
    assert L.nbody_leapfrog_kdk(P(64), P(1024), P(4096), 10, None, 0, 1, 1.0, 0.01, 1e-3, 1, 0x100, None, None) == -1
    assert L.nbody_leapfrog_kdk(P(64), P(1024), P(4096), 10, None, 0, 1, 1.0, 0.01, 1e-3, 1, 0x4, None, None) == -1
    assert L.nbody_leapfrog_kdk(P(64), P(64), P(4096), 10, None, 0, 1, 1.0, 0.01, 1e-3, 1, 0, None, None) == -1
    assert L.nbody_accel_vjp(P(64), P(1024), 10, 1, 1.0, 0.01, P(4096), None, None, None) == -1
    assert L.nbody_orb_order(P(64), 1, 10, 0, P(1024), None) == -1
    assert L.nbody_permute(P(64), P(1024), P(4096), 10, 24, 0, None) == -1
    assert L.nbody_trajectory_forward(P(64), P(1024), 10, 1, 1.0, 0.01, 1e-3, 30, 20, P(4096), None) == -1
    assert L.nbody_set_tuning(0, 1, 3, 1, 512, 0) == -1
    assert L.nbody_set_tuning(0, 1, 2, 1, 100, 0) == -1
    assert L.nbody_set_tuning(1, 1, 2, 4, 512, 0) == -1
    assert L.nbody_set_tuning(0, 1, 2, 1, 320, 1) == -1   # LDS variant needs jtile % 256 == 0
    assert L.nbody_set_tuning(0, 0, 1, 1, 512, 1) == -1   # no LDS variant in FP64
    assert L.nbody_set_tuning(2, 1, 1, 1, 512, 1) == -1   # nor for the VJP
    assert L.nbody_set_tuning(0, 1, 1, 1, 512, 2) == -1   # variants 0 and 1 only
    assert L.nbody_energy(P(64), P(1024), P(4096), 10, 1, None, None) == -1
    # tree code: leaf range, precision, theta, list arguments
    assert L.nbody_tree_shape(100, 0, None, None, None) == -1
    assert L.nbody_tree_shape(100, 65, None, None, None) == -1
    assert L.nbody_tree_accel(P(64), 100, 1, 1.0, 0.01, 0.5, 0, P(4096), None) == -1
    assert L.nbody_tree_accel(P(64), 100, 0, 1.0, 0.01, 0.5, 8, P(4096), None) == -5   # FP64 unsupported
    assert L.nbody_tree_accel(P(64), 100, 1, 1.0, 0.01, -0.1, 8, P(4096), None) == -1
    assert L.nbody_tree_accel(P(64), 100, 1, 1.0, 0.01, float("inf"), 8, P(4096), None) == -1
    assert L.nbody_tree_accel(P(72), 100, 1, 1.0, 0.01, 0.5, 8, P(4096), None) == -2
    assert L.nbody_tree_lists(P(64), 100, 8, 0.5, 4, 4, None, P(256), None, None, None) == -1
    assert L.nbody_tree_lists(P(64), 100, 8, 0.5, 0, 4, P(256), P(512), P(1024), None, None) == -1
    assert L.nbody_tree_moments(P(64), 100, 8, P(12), None, None) == -2
    # cell models 0, 2, 3, 4 only; record exports need float4 alignment
    ao = lambda *a: L.nbody_tree_accel_cells(*a)
    assert ao(P(64), 100, 1, 1.0, 0.01, 0.5, 4, 1, P(4096), None) == -1
    assert ao(P(64), 100, 1, 1.0, 0.01, 0.5, 4, -1, P(4096), None) == -1
    assert L.nbody_tree_quad(P(64), 100, 4, P(4104), None) == -2
    assert L.nbody_tree_quad(P(64), 0, 4, P(4096), None) == -1
    assert ao(P(64), 100, 1, 1.0, 0.01, 0.5, 4, 5, P(4096), None) == -1
    assert L.nbody_tree_local_counts(P(64), 100, 4, 0.5, None, P(256), P(512), None) == -1
    assert L.nbody_tree_local_counts(P(64), 100, 4, -0.5, P(128), P(256), P(512), None) == -1
    assert L.nbody_tree_local_counts(P(64), 100, 4, 0.5, P(130), P(256), P(512), None) == -1
    assert ao(P(64), 100, 0, 1.0, 0.01, 0.5, 4, 2, P(4096), None) == -5   # FP64 unsupported
    assert ao(P(64), 100, 1, 1.0, 0.01, 0.5, 0, 2, P(4096), None) == -1
    assert L.nbody_tree_pseudo(P(64), 100, 4, P(4100), None) == -2
    assert L.nbody_tree_pseudo(None, 100, 4, P(4096), None) == -1
    assert L.nbody_tree_pseudo(P(64), 100, 65, P(4096), None) == -1
    # tree leapfrog: precision, flags, order map, energy output
    lf = lambda *a: L.nbody_tree_leapfrog(*a)
    assert lf(P(64), P(1024), P(4096), None, 100, 0, 1.0, 0.01, 0.5, 8, 1e-3, 4, 0, 0, None, None) == -5
    assert lf(P(64), P(1024), P(4096), None, 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, 4, 0, 0x2, None, None) == -1
    assert lf(P(64), P(1024), P(4096), None, 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, 4, 0, 0x8 | 0x2, None, None) == -1
    assert lf(P(64), P(1024), P(4096), None, 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, 4, 0, 0x8 | 0x20, None, None) == -1
    assert lf(P(64), P(1024), P(4096), None, 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, 4, 0, 0x40 | 0x20, None, None) == -1
    assert lf(P(64), P(1024), P(4096), None, 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, 4, 2, 0, None, None) == -1
    assert lf(P(64), P(1024), P(4096), None, 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, 4, 0, 0x4, None, None) == -1
    assert lf(P(64), P(1024), P(4096), None, 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, -1, 0, 0, None, None) == -1
    assert lf(P(64), P(1024), P(4096), None, 100, 1, 1.0, 0.01, 0.5, 0, 1e-3, 4, 0, 0, None, None) == -1
    # adjoint: an unknown scheme stays invalid with the potential flag set
    assert L.nbody_trajectory_adjoint(P(64), 10, 1, 1.0, 0.01, 1e-3, 20, 20, P(1024), P(2048), P(4096),
                                      P(8192), P(16384), 0x10 | 5, None) == -1
    # fixed-point leapfrog: step count, shifts, state pointer and alignment
    jf = lambda *a: L.nbody_janus_forward(*a)
    assert jf(P(64), P(1024), 10, 1.0, 0.01, 1e-3, -1, 40, 40, P(4096), P(8192), None, None) == -1
    assert jf(P(64), P(1024), 10, 1.0, 0.01, 1e-3, 4, 61, 40, P(4096), P(8192), None, None) == -1
    assert jf(P(64), P(1024), 10, 1.0, 0.01, 1e-3, 4, 40, -1, P(4096), P(8192), None, None) == -1
    assert jf(P(64), P(1024), 10, 1.0, 0.01, 1e-3, 4, 40, 40, None, P(8192), None, None) == -2
    assert jf(P(64), P(1024), 10, 1.0, 0.01, 1e-3, 4, 40, 40, P(4112), P(8192), None, None) == -2
    assert jf(P(64), P(1024), 10, 1.0, 0.01, float("nan"), 4, 40, 40, P(4096), P(8192), None, None) == -1
    ja = lambda *a: L.nbody_janus_adjoint(*a)
    assert ja(P(4096), P(64), 10, 1.0, 0.01, 1e-3, -2, 40, 40, P(1024), P(2048), P(8192), P(16384), P(32768),
              None) == -1
    assert ja(P(4112), P(64), 10, 1.0, 0.01, 1e-3, 2, 40, 40, P(1024), P(2048), P(8192), P(16384), P(32768),
              None) == -2
    assert ja(P(4096), P(64), 10, 1.0, 0.01, 1e-3, 2, 40, 40, P(1024), P(2048), P(8192), P(16384), None,
              None) == -2



def test_overlapping_buffers_rejected():
    """Outputs that share memory with an input or with each other are refused
    before anything is enqueued (addresses only: nothing is dereferenced)."""
    nb, L = _lib()
    A, B, C, D = 0x100000, 0x200000, 0x300000, 0x400000
    # tree force: 100 float4 records = 1600 bytes from A
    assert L.nbody_tree_accel_cells(P(A), 100, 1, 1.0, 0.01, 0.5, 4, 3, P(A + 1024), None) == -1
    assert L.nbody_tree_accel(P(A), 100, 1, 1.0, 0.01, 0.5, 4, P(A + 1024), None) == -1
    # pseudo-particle and quadrupole exports run past the end of pos_mass
    assert L.nbody_tree_pseudo(P(A), 100, 4, P(A + 1024), None) == -1
    assert L.nbody_tree_quad(P(A), 100, 4, P(A + 1024), None) == -1
    # list counts must be int32-aligned
    assert L.nbody_tree_lists(P(A), 100, 8, 0.5, 0, 0, P(B + 2), P(C), None, None, None) == -2
    assert L.nbody_tree_lists(P(A), 100, 8, 0.5, 4, 0, P(B), P(C), P(D + 1), None, None) == -2
    # tree leapfrog: state buffers and the order map are disjoint
    lf = lambda *a: L.nbody_tree_leapfrog(*a)
    assert lf(P(A), P(A + 1024), P(C), None, 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, 4, 0, 0, None, None) == -1
    assert lf(P(A), P(B), P(B + 1584), None, 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, 4, 0, 0, None, None) == -1
    assert lf(P(A), P(B), P(C), P(B + 64), 100, 1, 1.0, 0.01, 0.5, 8, 1e-3, 4, 1, 0, None, None) == -1
    # fixed-point leapfrog: the state (64 bytes per body) is disjoint from the rest
    jf = lambda *a: L.nbody_janus_forward(*a)
    assert jf(P(A), P(B), 10, 1.0, 0.01, 1e-3, 4, 40, 40, P(C), P(C + 256), None, None) == -1
    assert jf(P(A), P(B), 10, 1.0, 0.01, 1e-3, 4, 40, 40, P(C), P(A + 64), None, None) == -1
    assert jf(P(A), P(B), 10, 1.0, 0.01, 1e-3, 4, 40, 40, P(C), P(D), P(D + 128), None) == -1
    ja = lambda *a: L.nbody_janus_adjoint(*a)
    assert ja(P(C), P(A), 10, 1.0, 0.01, 1e-3, 2, 40, 40, P(B), P(B + 256), P(D), P(D + 64), P(D + 1024),
              None) == -1
    assert ja(P(C), P(A), 10, 1.0, 0.01, 1e-3, 2, 40, 40, P(B), P(B + 256), P(C + 512), P(D), P(D + 1024),
              None) == -1
    assert ja(P(C), P(A), 10, 1.0, 0.01, 1e-3, 2, 40, 40, P(B), P(B + 256), P(D), P(D + 512), P(B + 8),
              None) == -1
    # energies, ORB order, tree inspection and the checkpointed trajectory
    assert L.nbody_energy(P(A), P(B), P(C), 100, 1, P(C + 1600 - 8), None) == -1
    assert L.nbody_orb_order(P(A), 1, 100, 8, P(A + 1596), None) == -1
    assert L.nbody_tree_moments(P(A), 100, 8, P(B), P(B + 64), None) == -1
    assert L.nbody_tree_moments(P(A), 100, 8, P(A + 8), None, None) == -1
    assert L.nbody_tree_lists(P(A), 100, 8, 0.5, 0, 0, P(B), P(B + 4), None, None, None) == -1
    assert L.nbody_tree_lists(P(A), 100, 8, 0.5, 4, 0, P(B), P(C), P(C + 4), None, None) == -1
    assert L.nbody_tree_local_counts(P(A), 100, 4, 0.5, P(B), P(C), P(B + 4), None) == -1
    assert L.nbody_trajectory_forward(P(A), P(A + 800), 100, 1, 1.0, 0.01, 1e-3, 20, 20, P(D), None) == -1
    assert L.nbody_trajectory_forward(P(A), P(B), 100, 1, 1.0, 0.01, 1e-3, 20, 20, P(B + 1024), None) == -1
    assert L.nbody_trajectory_adjoint(P(A), 100, 1, 1.0, 0.01, 1e-3, 20, 20, P(B), P(C), P(A + 4800),
                                      P(D), P(D + 4096), 1, None) == -1
    assert L.nbody_trajectory_adjoint(P(A), 100, 1, 1.0, 0.01, 1e-3, 20, 20, P(B), P(C), P(D),
                                      P(D + 1024), P(D + 8192), 1, None) == -1
    assert L.nbody_last_error()


@pytest.mark.parametrize("n,leaf", [(1, 1), (9, 8), (100, 8), (1000, 3), (4096, 16), (70001, 8), (777, 64)])
def test_tree_node_table_matches_oracle(orc, n, leaf):
    """The library's tree plan (host code) numbers and splits the nodes
    exactly as the oracle's ORB recursion."""
    nb, L = _lib()
    nn, ng, tab = nb.tree_shape(n, leaf, nodes=True)
    want = orc.tree_nodes(n, leaf)
    assert np.array_equal(tab.astype(np.int64), want)
    assert ng == orc._load().oracle_tree_num_groups(n, leaf, nb.TREE_GROUP)
    # the counts-only call (no table) takes a shortcut and must agree
    assert nb.tree_shape(n, leaf) == (nn, ng) == (want.shape[0], ng)


@pytest.mark.parametrize("n,leaf", [(1 << 20, 4), (10_000_019, 8), (3_000_001, 1), ((1 << 31) - 4096, 64)])
def test_tree_counts_shortcut_at_large_n(orc, n, leaf):
    """Node and group counts without building the plan, against the oracle's
    recursion."""
    nb, L = _lib()
    nn, ng = nb.tree_shape(n, leaf)
    lib = orc._load()
    assert nn == lib.oracle_tree_nodes(n, leaf, None)
    assert ng == lib.oracle_tree_num_groups(n, leaf, nb.TREE_GROUP)


def test_tuning_pin_roundtrip():
    nb, L = _lib()
    assert L.nbody_set_tuning(0, 2, 4, 8, 1024, 1) == 0
    assert nb.get_tuning(0, 2, 1 << 20) == (4, 8, 1024, 1)
    assert L.nbody_set_tuning(0, 2, -1, -1, -1, 0) == 0
    t = nb.get_tuning(0, 2, 1 << 20)
    assert t[0] in (1, 2, 4) and t[2] % 8 == 0 and t[3] in (0, 1)


def test_default_splits_take_the_xcd_mapping():
    """Without a pin or a tuned entry, the force kernel splits 2^20 sources
    in 8 (a multiple of the 8 XCDs, 2 MiB per split); small n keep splits of
    at least 256 sources."""
    import os
    if os.environ.get("NBODY_TUNE_CACHE"):
        pytest.skip("a tuning cache may hold a measured shape")
    nb, L = _lib()
    assert nb.get_tuning(0, 2, 1 << 20)[1] == 8
    assert nb.get_tuning(0, 2, 1 << 22)[1] == 8
    assert nb.get_tuning(0, 2, 1 << 17)[1] == 32
    assert nb.get_tuning(0, 2, 1024)[1] == 4
    assert nb.get_tuning(0, 2, 1023)[1] == 2


def test_missing_library_fails_loudly(tmp_path):
    """Without the built library the binding raises instead of computing
    anything elsewhere."""
    import subprocess, sys
    code = r"""
import sys
sys.path.insert(0, %r)
import paper_1211_2292_amd as nb
nb.LIB_PATH = %r
try:
    nb.lib()
except nb.NBodyError as e:
    print("raised:", e)
    sys.exit(0)
sys.exit(3)
""" % (ROOT, str(tmp_path / "missing.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "not built" in r.stdout


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with a message saying so,
    before touching torch or the library."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
