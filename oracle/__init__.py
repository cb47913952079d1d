"""Plain FP64 CPU oracle for the direct-sum n-body hot path (test
infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library and its Python
binding never import it; the two sides share no code, only the seeded
inputs from ``ics``.

The arithmetic lives in ``nbody_oracle.c`` (plain C, FP64, OpenMP over
targets, built with ``-O2 -ffp-contract=off``); this module builds it with
gcc and wraps it with numpy.  Each wrapper names the passage of the paper it
follows; the C file states the formulas.

Array conventions: ``pos_mass`` (N, 4) = (x, y, z, m); ``vel`` (N, 3) or
(N, 4) (w ignored); FP32 inputs are widened exactly to FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_f = ctypes.POINTER(ctypes.c_float)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile nbody_oracle.c into liboracle.so next to it (gcc, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        # NBODY_ORACLE_LIB: a prebuilt variant of this library (the tests
        # that plant mistakes in the oracle point it at their mutants)
        alt = os.environ.get("NBODY_ORACLE_LIB")
        if not alt:
            build(force=False)
        lib = ctypes.CDLL(alt or _LIB_PATH)
        lib.oracle_accel.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int64, _i64, _d, _d]
        lib.oracle_accel.restype = None
        lib.oracle_energy.argtypes = [ctypes.c_int64, _d, _d, _d, _d]
        lib.oracle_energy.restype = None
        lib.oracle_leapfrog.argtypes = [ctypes.c_int64, _d, _d, _d, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int32, _d, _d, _d]
        lib.oracle_leapfrog.restype = None
        lib.oracle_orb_order.argtypes = [ctypes.c_int64, _f, ctypes.c_int32, _i32]
        lib.oracle_orb_order.restype = ctypes.c_int
        lib.oracle_vjp.argtypes = [ctypes.c_int64, _d, _d, ctypes.c_double, ctypes.c_double, _d, _d, _d, _d]
        lib.oracle_vjp.restype = None
        lib.oracle_traj_grad.argtypes = [ctypes.c_int64, _d, _d, _d, _d, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int32, _d, _d, _d]
        lib.oracle_traj_grad.restype = ctypes.c_double
        lib.oracle_traj_grad_cot.argtypes = [ctypes.c_int64, _d, _d, _d, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int32, _d, _d, _d, _d, _d, _d]
        lib.oracle_traj_grad_cot.restype = ctypes.c_int
        lib.oracle_janus_run.argtypes = [ctypes.c_int64, _i64, _d, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32]
        lib.oracle_janus_run.restype = ctypes.c_int
        lib.oracle_tree_nodes.argtypes = [ctypes.c_int64, ctypes.c_int32, _i64]
        lib.oracle_tree_nodes.restype = ctypes.c_int64
        lib.oracle_tree_moments.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d, _d, _d, _d, _d]
        lib.oracle_tree_moments.restype = ctypes.c_int
        lib.oracle_tree_num_groups.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
        lib.oracle_tree_num_groups.restype = ctypes.c_int64
        lib.oracle_tree_lists.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d, ctypes.c_double,
                                          _i64, _i64, _i64, _i32, ctypes.c_int64, _i32, ctypes.c_int64]
        lib.oracle_tree_lists.restype = ctypes.c_int
        lib.oracle_tree_accel.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int64, _i64, _d, _d]
        lib.oracle_tree_accel.restype = ctypes.c_int
        lib.oracle_tree_accel_cells.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_int32, ctypes.c_int64, _i64, _d, _d]
        lib.oracle_tree_accel_cells.restype = ctypes.c_int
        lib.oracle_tree_quad.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d]
        lib.oracle_tree_quad.restype = ctypes.c_int
        lib.oracle_tree_local_counts.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d,
                                                 ctypes.c_double, _i64, _i64, _i64]
        lib.oracle_tree_local_counts.restype = ctypes.c_int
        lib.oracle_tree_local_lists.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d,
                                                ctypes.c_double, _i64, _i64, _i64, _i32, ctypes.c_int64, _i32,
                                                ctypes.c_int64, _i32, ctypes.c_int64]
        lib.oracle_tree_local_lists.restype = ctypes.c_int
        lib.oracle_tree_pseudo.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d]
        lib.oracle_tree_pseudo.restype = ctypes.c_int
        lib.oracle_pseudo_dirs.argtypes = [_d]
        lib.oracle_pseudo_dirs.restype = None
        lib.oracle_fmm_lists.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, ctypes.c_double, _i64, _i64, _i64,
                                         _i32, ctypes.c_int64, _i32, ctypes.c_int64, _i32, ctypes.c_int64]
        lib.oracle_fmm_lists.restype = ctypes.c_int
        lib.oracle_fmm_accel.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_int64, _i64, _d, _d]
        lib.oracle_fmm_accel.restype = ctypes.c_int
        lib.oracle_local_shift.argtypes = [_d, _d, _d]
        lib.oracle_local_shift.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
        return lib


def _c64(a, shape_last=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _split(pos_mass):
    pm = np.asarray(pos_mass)
    x = np.ascontiguousarray(pm[:, :3], dtype=np.float64)
    m = np.ascontiguousarray(pm[:, 3], dtype=np.float64)
    return x, m


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def accel(pos_mass, eps: float, G: float = 1.0, targets=None):
    """Exact softened direct sum (Section IV; force loop of Section IV.A with
    every cell opened).  Returns (acc (T, 3), pot (T,)) for the targets
    (all bodies when ``targets`` is None)."""
    lib = _load()
    x, m = _split(pos_mass)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        t = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        if t.size and (t.min() < 0 or t.max() >= n):
            raise IndexError("target index out of range")
        nt, tp = t.shape[0], t
    acc = np.empty((nt, 3))
    pot = np.empty(nt)
    lib.oracle_accel(n, _ptr(x, _d), _ptr(m, _d), float(G), float(eps), nt,
                     None if tp is None else _ptr(tp, _i64), _ptr(acc, _d), _ptr(pot, _d))
    return acc, pot


def energy(vel, pos_mass, pot):
    """(K, U) = (1/2 sum m |v|^2, 1/2 sum m phi)."""
    lib = _load()
    _, m = _split(pos_mass)
    v = np.ascontiguousarray(np.asarray(vel)[:, :3], dtype=np.float64)
    p = np.ascontiguousarray(pot, dtype=np.float64)
    out = np.empty(2)
    lib.oracle_energy(m.shape[0], _ptr(v, _d), _ptr(m, _d), _ptr(p, _d), _ptr(out, _d))
    return float(out[0]), float(out[1])


def leapfrog(pos_mass, vel, eps: float, dt: float, nsteps: int, G: float = 1.0):
    """Kick-drift-kick leapfrog (Move_bodies after Calculate_forces, Section
    IV.B pseudo-code).  Returns dict with x, v (N, 3), acc (N, 3), pot (N,)
    at the final state and energy ((nsteps+1), 2)."""
    lib = _load()
    x, m = _split(pos_mass)
    v = np.ascontiguousarray(np.asarray(vel)[:, :3], dtype=np.float64).copy()
    x = x.copy()
    n = x.shape[0]
    acc = np.empty((n, 3))
    pot = np.empty(n)
    en = np.empty((nsteps + 1, 2))
    lib.oracle_leapfrog(n, _ptr(x, _d), _ptr(v, _d), _ptr(m, _d), float(G), float(eps), float(dt),
                        int(nsteps), _ptr(acc, _d), _ptr(pot, _d), _ptr(en, _d))
    return dict(x=x, v=v, acc=acc, pot=pot, energy=en)


def orb_order(pos, leaf: int) -> np.ndarray:
    """Orthogonal Recursive Bisection order (Section IV.B) on the FP32
    coordinates of ``pos`` (N, >=3); perm[p] = original index at position p."""
    lib = _load()
    xf = np.ascontiguousarray(np.asarray(pos)[:, :3], dtype=np.float32)
    n = xf.shape[0]
    perm = np.empty(n, dtype=np.int32)
    rc = lib.oracle_orb_order(n, _ptr(xf, _f), int(leaf), _ptr(perm, _i32))
    if rc != 0:
        raise ValueError("oracle_orb_order: bad arguments")
    return perm


def vjp(pos_mass, eps: float, acc_cot, pot_cot=None, G: float = 1.0):
    """Vector-Jacobian product of the direct sum with respect to positions and
    masses.  Returns (x_cot (N, 3), m_cot (N,))."""
    lib = _load()
    x, m = _split(pos_mass)
    n = x.shape[0]
    ab = np.ascontiguousarray(np.asarray(acc_cot)[:, :3], dtype=np.float64)
    pb = None if pot_cot is None else np.ascontiguousarray(pot_cot, dtype=np.float64)
    xb = np.empty((n, 3))
    mb = np.empty(n)
    lib.oracle_vjp(n, _ptr(x, _d), _ptr(m, _d), float(G), float(eps), _ptr(ab, _d),
                   None if pb is None else _ptr(pb, _d), _ptr(xb, _d), _ptr(mb, _d))
    return xb, mb


def traj_grad(pos_mass, vel, y, eps: float, dt: float, nsteps: int, G: float = 1.0):
    """Loss L = sum |x(T) - y|^2 through ``nsteps`` leapfrog steps and its
    gradient (dL/dx0 (N,3), dL/dv0 (N,3), dL/dm (N,))."""
    lib = _load()
    x, m = _split(pos_mass)
    n = x.shape[0]
    v = np.ascontiguousarray(np.asarray(vel)[:, :3], dtype=np.float64)
    yy = np.ascontiguousarray(np.asarray(y)[:, :3], dtype=np.float64)
    gx = np.empty((n, 3))
    gv = np.empty((n, 3))
    gm = np.empty(n)
    L = lib.oracle_traj_grad(n, _ptr(x, _d), _ptr(v, _d), _ptr(m, _d), _ptr(yy, _d), float(G), float(eps),
                             float(dt), int(nsteps), _ptr(gx, _d), _ptr(gv, _d), _ptr(gm, _d))
    return float(L), gx, gv, gm


def traj_grad_cot(pos_mass, vel, eps: float, dt: float, nsteps: int, xbar_T, vbar_T, phibar_T=None,
                  G: float = 1.0):
    """Reverse mode through the leapfrog for cotangents of the final state
    (xbar_T, vbar_T (N, 3), phibar_T (N,) on the final potential, optional).
    Returns (dL/dx0 (N, 3), dL/dv0 (N, 3), dL/dm (N,)) through the
    trajectory."""
    lib = _load()
    x, m = _split(pos_mass)
    n = x.shape[0]
    v = np.ascontiguousarray(np.asarray(vel)[:, :3], dtype=np.float64)
    xb = np.ascontiguousarray(np.asarray(xbar_T)[:, :3], dtype=np.float64)
    vb = np.ascontiguousarray(np.asarray(vbar_T)[:, :3], dtype=np.float64)
    pb = None if phibar_T is None else np.ascontiguousarray(phibar_T, dtype=np.float64)
    gx = np.empty((n, 3))
    gv = np.empty((n, 3))
    gm = np.empty(n)
    rc = lib.oracle_traj_grad_cot(n, _ptr(x, _d), _ptr(v, _d), _ptr(m, _d), float(G), float(eps), float(dt),
                                  int(nsteps), _ptr(xb, _d), _ptr(vb, _d), None if pb is None else _ptr(pb, _d),
                                  _ptr(gx, _d), _ptr(gv, _d), _ptr(gm, _d))
    if rc != 0:
        raise MemoryError("oracle_traj_grad_cot failed")
    return gx, gv, gm


def janus_encode(pos, vel, sx: int = 40, sv: int = 40) -> np.ndarray:
    """Fixed-point state int64 (N, 8) = (X, Y, Z, 0, VX, VY, VZ, 0) from
    positions and velocities (rounded to nearest, half to even)."""
    n = np.asarray(pos).shape[0]
    st = np.zeros((n, 8), dtype=np.int64)
    st[:, :3] = np.rint(np.ldexp(np.asarray(pos, dtype=np.float64)[:, :3], sx)).astype(np.int64)
    st[:, 4:7] = np.rint(np.ldexp(np.asarray(vel, dtype=np.float64)[:, :3], sv)).astype(np.int64)
    return st


def janus_run(state, masses, eps: float, dt: float, nsteps: int, sx: int = 40, sv: int = 40, G: float = 1.0,
              direction: int = 1) -> np.ndarray:
    """Bit-reversible fixed-point kick-drift-kick (FP64 forces): nsteps
    forward (direction 1) or backward (-1) from ``state``; returns the new
    state."""
    lib = _load()
    st = np.ascontiguousarray(np.array(state, dtype=np.int64))
    m = np.ascontiguousarray(masses, dtype=np.float64)
    rc = lib.oracle_janus_run(st.shape[0], _ptr(st, _i64), _ptr(m, _d), float(G), float(eps), float(dt),
                              int(nsteps), int(sx), int(sv), int(direction))
    if rc != 0:
        raise ValueError("oracle_janus_run: bad arguments")
    return st


# ---- tree code on the ORB cells (Section IV.A walk, Section IV.B cells) ----
# All tree functions take bodies already in ORB order (``orb_order`` with the
# same leaf, then a gather).  Groups are the maximal nodes of at most
# ``group`` bodies, in ORB order.

def tree_nodes(n: int, leaf: int) -> np.ndarray:
    """Node table (nn, 4) = (begin, end, left, right) of the ORB recursion in
    preorder; left = right = -1 for a leaf."""
    lib = _load()
    nn = int(lib.oracle_tree_nodes(int(n), int(leaf), None))
    if nn < 1:
        raise ValueError("oracle_tree_nodes: bad arguments")
    nodes = np.empty((nn, 4), dtype=np.int64)
    lib.oracle_tree_nodes(int(n), int(leaf), _ptr(nodes, _i64))
    return nodes


def tree_moments(pos_mass_orb, leaf: int):
    """Monopole moments of every node: dict(mass (nn,), com (nn, 3), lo, hi
    (nn, 3), diag2 (nn,)), FP64 in the fixed summation order of the C file."""
    lib = _load()
    x, m = _split(pos_mass_orb)
    n = x.shape[0]
    nn = tree_nodes(n, leaf).shape[0]
    out = dict(mass=np.empty(nn), com=np.empty((nn, 3)), lo=np.empty((nn, 3)), hi=np.empty((nn, 3)),
               diag2=np.empty(nn))
    rc = lib.oracle_tree_moments(n, int(leaf), _ptr(x, _d), _ptr(m, _d), _ptr(out["mass"], _d),
                                 _ptr(out["com"], _d), _ptr(out["lo"], _d), _ptr(out["hi"], _d),
                                 _ptr(out["diag2"], _d))
    if rc != 0:
        raise ValueError("oracle_tree_moments failed")
    return out


def tree_lists(pos_mass_orb, leaf: int, group: int, theta: float):
    """Interaction lists of every group (Section IV.A walk): dict(group_id,
    far_cnt, near_cnt (ngroups,), far, near (concatenated node ids in walk
    order))."""
    lib = _load()
    x, m = _split(pos_mass_orb)
    n = x.shape[0]
    ng = int(lib.oracle_tree_num_groups(n, int(leaf), int(group)))
    if ng < 1:
        raise ValueError("oracle_tree_num_groups: bad arguments")
    gid = np.empty(ng, dtype=np.int64)
    fc = np.empty(ng, dtype=np.int64)
    nc = np.empty(ng, dtype=np.int64)
    rc = lib.oracle_tree_lists(n, int(leaf), int(group), _ptr(x, _d), _ptr(m, _d), float(theta), _ptr(gid, _i64),
                               _ptr(fc, _i64), _ptr(nc, _i64), None, 0, None, 0)
    if rc != 0:
        raise ValueError("oracle_tree_lists: bad arguments")
    far = np.empty(max(int(fc.sum()), 1), dtype=np.int32)
    near = np.empty(max(int(nc.sum()), 1), dtype=np.int32)
    rc = lib.oracle_tree_lists(n, int(leaf), int(group), _ptr(x, _d), _ptr(m, _d), float(theta), _ptr(gid, _i64),
                               _ptr(fc, _i64), _ptr(nc, _i64), _ptr(far, _i32), far.shape[0], _ptr(near, _i32),
                               near.shape[0])
    if rc != 0:
        raise ValueError("oracle_tree_lists failed")
    return dict(group_id=gid, far_cnt=fc, near_cnt=nc, far=far[:int(fc.sum())], near=near[:int(nc.sum())])


def tree_accel(pos_mass_orb, leaf: int, group: int, theta: float, eps: float, G: float = 1.0, targets=None,
               cells: int = 0):
    """Tree-code force and potential (Section IV.A) on the ORB cells: far
    cells as monopoles (cells 0), as their 12 pseudo-particles (2, the
    pseudo-particle multipole method of the paper's reference [20]) or through
    their quadrupole expansion (3); near leaves body by body.  Returns
    (acc (T, 3), pot (T,)) for ORB positions ``targets`` (all when None)."""
    lib = _load()
    x, m = _split(pos_mass_orb)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        tp = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        if tp.size and (tp.min() < 0 or tp.max() >= n):
            raise IndexError("target index out of range")
        nt = tp.shape[0]
    acc = np.empty((nt, 3))
    pot = np.empty(nt)
    rc = lib.oracle_tree_accel_cells(n, int(leaf), int(group), _ptr(x, _d), _ptr(m, _d), float(G), float(eps),
                                     float(theta), int(cells), nt, None if tp is None else _ptr(tp, _i64),
                                     _ptr(acc, _d), _ptr(pot, _d))
    if rc != 0:
        raise ValueError("oracle_tree_accel_cells failed")
    return acc, pot


def pseudo_dirs() -> np.ndarray:
    """The 12 unit directions (icosahedron vertices) of the pseudo-particles."""
    out = np.empty((12, 3))
    _load().oracle_pseudo_dirs(_ptr(out, _d))
    return out


def tree_pseudo(pos_mass_orb, leaf: int) -> np.ndarray:
    """Pseudo-particles (x, y, z, q) of every node, (nn, 12, 4): the order-2
    expansion of each cell about its centre of mass carried by 12 point
    masses on a sphere of half the box diagonal (Makino's formula, summed
    over the cell's bodies)."""
    lib = _load()
    x, m = _split(pos_mass_orb)
    n = x.shape[0]
    nn = tree_nodes(n, leaf).shape[0]
    out = np.empty((nn, 12, 4))
    if lib.oracle_tree_pseudo(n, int(leaf), _ptr(x, _d), _ptr(m, _d), _ptr(out, _d)) != 0:
        raise ValueError("oracle_tree_pseudo: bad arguments")
    return out


def tree_quad(pos_mass_orb, leaf: int) -> np.ndarray:
    """Traceless quadrupole (Qxx, Qyy, Qzz, Qxy, Qxz, Qyz) of every node about
    its centre of mass, (nn, 6), summed over the cell's bodies."""
    lib = _load()
    x, m = _split(pos_mass_orb)
    n = x.shape[0]
    nn = tree_nodes(n, leaf).shape[0]
    out = np.empty((nn, 6))
    if lib.oracle_tree_quad(n, int(leaf), _ptr(x, _d), _ptr(m, _d), _ptr(out, _d)) != 0:
        raise ValueError("oracle_tree_quad: bad arguments")
    return out


def tree_local_counts(pos_mass_orb, leaf: int, group: int, theta: float):
    """Per-group sizes of the local-expansion walk: dict(loc_cnt, far_cnt,
    near_cnt), each (ngroups,) int64, groups in ORB order."""
    lib = _load()
    x, m = _split(pos_mass_orb)
    n = x.shape[0]
    ng = int(lib.oracle_tree_num_groups(n, int(leaf), int(group)))
    if ng < 1:
        raise ValueError("oracle_tree_num_groups: bad arguments")
    out = dict(loc_cnt=np.empty(ng, dtype=np.int64), far_cnt=np.empty(ng, dtype=np.int64),
               near_cnt=np.empty(ng, dtype=np.int64))
    rc = lib.oracle_tree_local_counts(n, int(leaf), int(group), _ptr(x, _d), _ptr(m, _d), float(theta),
                                      _ptr(out["loc_cnt"], _i64), _ptr(out["far_cnt"], _i64),
                                      _ptr(out["near_cnt"], _i64))
    if rc != 0:
        raise ValueError("oracle_tree_local_counts failed")
    return out


def tree_local_lists(pos_mass_orb, leaf: int, group: int, theta: float):
    """Lists of the local-expansion walk: dict(loc_cnt, far_cnt, near_cnt
    (ngroups,), loc, far, near (concatenated node ids in walk order))."""
    lib = _load()
    x, m = _split(pos_mass_orb)
    n = x.shape[0]
    c = tree_local_counts(pos_mass_orb, leaf, group, theta)
    ng = c["loc_cnt"].shape[0]
    out = {k: np.empty(ng, dtype=np.int64) for k in ("loc_cnt", "far_cnt", "near_cnt")}
    caps = {k: max(int(c[k + "_cnt"].sum()), 1) for k in ("loc", "far", "near")}
    lists = {k: np.empty(caps[k], dtype=np.int32) for k in caps}
    rc = lib.oracle_tree_local_lists(n, int(leaf), int(group), _ptr(x, _d), _ptr(m, _d), float(theta),
                                     _ptr(out["loc_cnt"], _i64), _ptr(out["far_cnt"], _i64),
                                     _ptr(out["near_cnt"], _i64), _ptr(lists["loc"], _i32), caps["loc"],
                                     _ptr(lists["far"], _i32), caps["far"], _ptr(lists["near"], _i32), caps["near"])
    if rc != 0:
        raise ValueError("oracle_tree_local_lists failed")
    for k in ("loc", "far", "near"):
        out[k] = lists[k][:int(out[k + "_cnt"].sum())]
    return out


def fmm_lists(pos_mass_orb, leaf: int, theta: float):
    """Interaction lists of the multi-level FMM's dual-tree traversal on the
    ORB nodes (Section VI's O(N) method): dict(m2l_cnt, m2p_cnt, p2p_cnt
    (nn,) per target node, m2l, m2p, p2p (source node ids, targets in node
    order, each target's sources in traversal order))."""
    lib = _load()
    x, m = _split(pos_mass_orb)
    n = x.shape[0]
    nn = tree_nodes(n, leaf).shape[0]
    cnt = [np.empty(nn, dtype=np.int64) for _ in range(3)]
    if lib.oracle_fmm_lists(n, int(leaf), _ptr(x, _d), _ptr(m, _d), float(theta), *(_ptr(c, _i64) for c in cnt),
                            None, 0, None, 0, None, 0) != 0:
        raise ValueError("oracle_fmm_lists: bad arguments")
    ids = [np.empty(max(int(c.sum()), 1), dtype=np.int32) for c in cnt]
    args = []
    for a in ids:
        args += [_ptr(a, _i32), a.shape[0]]
    if lib.oracle_fmm_lists(n, int(leaf), _ptr(x, _d), _ptr(m, _d), float(theta), *(_ptr(c, _i64) for c in cnt),
                            *args) != 0:
        raise ValueError("oracle_fmm_lists failed")
    out = {}
    for name, c, a in zip(("m2l", "m2p", "p2p"), cnt, ids):
        out[name + "_cnt"] = c
        out[name] = a[:int(c.sum())]
    return out


def fmm_accel(pos_mass_orb, leaf: int, theta: float, eps: float, G: float = 1.0, targets=None):
    """Force and potential by the multi-level FMM on the ORB nodes
    (quadrupole cells, third-order local expansions, L2L down the tree, M2P
    cells and P2P leaves at the leaves).  Returns (acc (T, 3), pot (T,)) for ORB positions
    ``targets`` (all when None)."""
    lib = _load()
    x, m = _split(pos_mass_orb)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        tp = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        if tp.size and (tp.min() < 0 or tp.max() >= n):
            raise IndexError("target index out of range")
        nt = tp.shape[0]
    acc = np.empty((nt, 3))
    pot = np.empty(nt)
    rc = lib.oracle_fmm_accel(n, int(leaf), _ptr(x, _d), _ptr(m, _d), float(G), float(eps), float(theta), nt,
                              None if tp is None else _ptr(tp, _i64), _ptr(acc, _d), _ptr(pot, _d))
    if rc != 0:
        raise ValueError("oracle_fmm_accel failed")
    return acc, pot


def local_shift(coeffs, dz) -> np.ndarray:
    """Re-expansion (L2L) of a cubic local expansion (20 coefficients: P0,
    p (3), K (xx, yy, zz, xy, xz, yz), T (xxx, yyy, zzz, xxy, xxz, xyy, yyz,
    xzz, yzz, xyz)) about its centre + dz."""
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    d = np.ascontiguousarray(np.asarray(dz, dtype=np.float64))
    out = np.empty(20)
    _load().oracle_local_shift(_ptr(c, _d), _ptr(d, _d), _ptr(out, _d))
    return out
