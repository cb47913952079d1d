"""Python binding of the gfx950 direct-sum n-body library (include/nbody.h).

Argument marshalling only: every entry point checks dtypes, devices, shapes
and contiguity, then calls the C ABI of ``libnbody.so`` with raw device
pointers and torch's current HIP stream.  All arithmetic runs in the HIP
kernels of the library; there is no fallback.  If the library has not been
built (``python -m paper_1211_2292_amd.build``), the first call raises.

Records are (N, 4) tensors on the GPU: pos_mass = (x, y, z, m),
vel = (vx, vy, vz, unused), acc_pot = (ax, ay, az, phi).  float64 tensors use
the FP64 path; float32 tensors use one of the FP32 modes (default
NBODY_F32_KAHAN).
"""
from __future__ import annotations

import ctypes
import functools
import os
import threading

import torch

__all__ = [
    "F64", "F32", "F32_KAHAN", "F32_F64ACC", "ACC_VALID", "GRAPH", "ENERGY", "ADJ_RECOMPUTE",
    "ADJ_REVERSE", "ADJ_PHI",
    "lib", "accel", "accel_vjp", "leapfrog_kdk", "kick_drift", "batched_accel", "energy", "orb_order",
    "permute", "trajectory_forward", "trajectory_adjoint", "NBodyTrajectory", "autotune",
    "set_tuning", "get_tuning", "release", "NBodyError", "TREE_GROUP", "tree_shape", "tree_accel",
    "tree_moments", "tree_lists", "tree_leapfrog", "tree_pseudo", "tree_quad", "TREE_PSEUDO",
    "CELLS_MONOPOLE", "CELLS_PSEUDO", "CELLS_QUADRUPOLE", "CELLS_LOCAL", "tree_local_counts",
    "janus_forward", "janus_adjoint", "ReversibleTrajectory",
]

F64, F32, F32_KAHAN, F32_F64ACC = 0, 1, 2, 3
ADJ_RECOMPUTE, ADJ_REVERSE, ADJ_PHI = 0, 1, 0x10
ACC_VALID, GRAPH, ENERGY = 0x1, 0x2, 0x4
KERNEL_ACCEL, KERNEL_BATCHED, KERNEL_VJP = 0, 1, 2
TREE_GROUP = 64
TREE_PSEUDO = 12      # pseudo-particles per cell (CELLS_PSEUDO)
CELLS_MONOPOLE, CELLS_PSEUDO, CELLS_QUADRUPOLE, CELLS_LOCAL = 0, 2, 3, 4   # tree cell models
_TREE_CELL_FLAGS = {CELLS_MONOPOLE: 0, CELLS_PSEUDO: 0x8, CELLS_QUADRUPOLE: 0x20, CELLS_LOCAL: 0x40}

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbody.so")
_lock = threading.Lock()
_lib = None

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double

_SIGS = {
    "nbody_orb_order": [_vp, _i32, _i64, _i32, _vp, _vp],
    "nbody_permute": [_vp, _vp, _vp, _i64, _i32, _i32, _vp],
    "nbody_accel": [_vp, _i64, _i32, _dbl, _dbl, _vp, _i64, _i64, _vp],
    "nbody_accel_noalloc": [_vp, _i64, _i32, _dbl, _dbl, _vp, _i64, _i64, _vp],
    "nbody_accel_vjp": [_vp, _vp, _i64, _i32, _dbl, _dbl, _vp, _vp, _vp, _vp],
    "nbody_leapfrog_kdk": [_vp, _vp, _vp, _i64, _vp, _i32, _i32, _dbl, _dbl, _dbl, _i32,
                           ctypes.c_uint32, _vp, _vp],
    "nbody_kick_drift": [_vp, _vp, _vp, _i64, _i32, _dbl, _dbl, _i32, _i32, _vp],
    "nbody_batched_accel": [_vp, _vp, _i32, _i32, _dbl, _vp, _dbl, _vp, _vp],
    "nbody_energy": [_vp, _vp, _vp, _i64, _i32, _vp, _vp],
    "nbody_trajectory_forward": [_vp, _vp, _i64, _i32, _dbl, _dbl, _dbl, _i32, _i32, _vp, _vp],
    "nbody_trajectory_adjoint": [_vp, _i64, _i32, _dbl, _dbl, _dbl, _i32, _i32, _vp, _vp, _vp,
                                 _vp, _vp, _i32, _vp],
    "nbody_tree_shape": [_i64, _i32, _vp, _vp, _vp],
    "nbody_tree_accel": [_vp, _i64, _i32, _dbl, _dbl, _dbl, _i32, _vp, _vp],
    "nbody_fmm_accel": [_vp, _i64, _i32, _dbl, _dbl, _dbl, _i32, _vp, _vp],
    "nbody_fmm_lists": [_vp, _i64, _i32, _dbl, _vp, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp],
    "nbody_tree_accel_cells": [_vp, _i64, _i32, _dbl, _dbl, _dbl, _i32, _i32, _vp, _vp],
    "nbody_tree_pseudo": [_vp, _i64, _i32, _vp, _vp],
    "nbody_tree_quad": [_vp, _i64, _i32, _vp, _vp],
    "nbody_tree_local_counts": [_vp, _i64, _i32, _dbl, _vp, _vp, _vp, _vp],
    "nbody_tree_moments": [_vp, _i64, _i32, _vp, _vp, _vp],
    "nbody_tree_lists": [_vp, _i64, _i32, _dbl, _i32, _i32, _vp, _vp, _vp, _vp, _vp],
    "nbody_tree_leapfrog": [_vp, _vp, _vp, _vp, _i64, _i32, _dbl, _dbl, _dbl, _i32, _dbl, _i32, _i32,
                            ctypes.c_uint32, _vp, _vp],
    "nbody_janus_forward": [_vp, _vp, _i64, _dbl, _dbl, _dbl, _i32, _i32, _i32, _vp, _vp, _vp, _vp],
    "nbody_janus_adjoint": [_vp, _vp, _i64, _dbl, _dbl, _dbl, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp],
    "nbody_autotune": [_i32, _i32, _i64, _vp, _i32, _vp],
    "nbody_set_tuning": [_i32, _i32, _i32, _i32, _i32, _i32],
    "nbody_get_tuning": [_i32, _i32, _i64, _vp, _vp, _vp, _vp],
    "nbody_status_string": [ctypes.c_int],
    "nbody_last_error": [],
    "nbody_release": [],
    "nbody_version": [],
}


class NBodyError(RuntimeError):
    pass


def lib():
    """Load libnbody.so (in-tree build) and declare its signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise NBodyError(f"{LIB_PATH} is not built; run `python -m paper_1211_2292_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.nbody_status_string.restype = ctypes.c_char_p
        L.nbody_last_error.restype = ctypes.c_char_p
        L.nbody_release.restype = None
        _lib = L
        return L


def _check(rc: int):
    if rc != 0:
        L = lib()
        raise NBodyError(f"{L.nbody_status_string(rc).decode()} ({rc}): {L.nbody_last_error().decode()}")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _rec(t: torch.Tensor, name: str, dtype=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dim() != 2 or t.shape[1] != 4:
        raise ValueError(f"{name} must have shape (N, 4), got {tuple(t.shape)}")
    if t.dtype not in (torch.float32, torch.float64):
        raise TypeError(f"{name} must be float32 or float64")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _out(t: torch.Tensor, rows: int, like: torch.Tensor) -> torch.Tensor:
    """A caller-supplied output: (rows, 4) records of like's dtype on like's
    device, contiguous (the kernels write exactly that many records)."""
    _rec(t, "out", like.dtype)
    if t.shape[0] != rows or t.device != like.device:
        raise ValueError(f"out must have shape ({rows}, 4) on {like.device}, got {tuple(t.shape)} on {t.device}")
    return t


def _prec(t: torch.Tensor, prec):
    if t.dtype == torch.float64:
        if prec not in (None, F64):
            raise ValueError("float64 tensors use prec=F64")
        return F64
    if prec is None:
        return F32_KAHAN
    if prec not in (F32, F32_KAHAN, F32_F64ACC):
        raise ValueError("float32 tensors use prec F32, F32_KAHAN or F32_F64ACC")
    return prec


def _on_device(fn):
    """Runs fn with the device of its GPU tensor arguments current: the
    library launches on, and keeps its scratch for, the current HIP device.
    Every GPU tensor argument must be on that one device."""
    @functools.wraps(fn)
    def wrapper(*args, **kw):
        gpu = [a for a in (*args, *kw.values()) if isinstance(a, torch.Tensor) and a.device.type == "cuda"]
        if not gpu:
            return fn(*args, **kw)
        dev = gpu[0].device
        for t in gpu[1:]:
            if t.device != dev:
                raise ValueError(f"GPU tensors of one call must share a device, got {dev} and {t.device}")
        with torch.cuda.device(dev):
            return fn(*args, **kw)
    return wrapper


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@_on_device
def accel(pos_mass, eps, G=1.0, prec=None, target_begin=0, target_count=None, out=None):
    """Force and potential records for targets [target_begin, +target_count)."""
    pm = _rec(pos_mass, "pos_mass")
    p = _prec(pm, prec)
    n = pm.shape[0]
    tc = n - target_begin if target_count is None else target_count
    if out is None:
        out = torch.empty((tc, 4), dtype=pm.dtype, device=pm.device)
    else:
        _out(out, tc, pm)
    _check(lib().nbody_accel(_ptr(pm), n, p, float(G), float(eps), _ptr(out), int(target_begin), int(tc),
                             _stream()))
    return out


@_on_device
def accel_noalloc(pos_mass, out, eps, G=1.0, prec=None, target_begin=0):
    """nbody_accel_noalloc: the force of targets [target_begin, +len(out))
    into the caller's ``out``, with no device allocation by the library."""
    pm = _rec(pos_mass, "pos_mass")
    p = _prec(pm, prec)
    tc = _rec(out, "out", pm.dtype).shape[0]
    _out(out, tc, pm)
    _check(lib().nbody_accel_noalloc(_ptr(pm), pm.shape[0], p, float(G), float(eps), _ptr(out),
                                     int(target_begin), int(tc), _stream()))
    return out


@_on_device
def accel_vjp(pos_mass, acc_pot_cot, eps, G=1.0, prec=None, forward=True):
    """(pos_cot (N,4), mass_cot (N,), acc_pot (N,4) or None) at one configuration."""
    pm = _rec(pos_mass, "pos_mass")
    cot = _rec(acc_pot_cot, "acc_pot_cot", pm.dtype)
    p = _prec(pm, prec)
    n = pm.shape[0]
    pc = torch.empty_like(pm)
    mc = torch.empty(n, dtype=pm.dtype, device=pm.device)
    ap = torch.empty_like(pm) if forward else None
    _check(lib().nbody_accel_vjp(_ptr(pm), _ptr(cot), n, p, float(G), float(eps), _ptr(pc), _ptr(mc),
                                 _ptr(ap), _stream()))
    return pc, mc, ap


def _offsets(offsets):
    if offsets is None:
        return None, 0, None
    o = torch.as_tensor(offsets, dtype=torch.int64).cpu().contiguous()
    return o, int(o.numel() - 1), ctypes.c_void_p(o.data_ptr())


@_on_device
def leapfrog_kdk(pos_mass, vel, acc_pot, eps, dt, nsteps, G=1.0, prec=None, offsets=None,
                 acc_valid=False, graph=False, energy=False, energy_out=None):
    """nsteps of KDK leapfrog in place; returns the (nsteps+1, 2) FP64 energy
    tensor when energy=True (``energy_out`` if given), else None."""
    pm = _rec(pos_mass, "pos_mass")
    v = _rec(vel, "vel", pm.dtype)
    a = _rec(acc_pot, "acc_pot", pm.dtype)
    p = _prec(pm, prec)
    o, nsys, optr = _offsets(offsets)
    flags = (ACC_VALID if acc_valid else 0) | (GRAPH if graph else 0) | (ENERGY if energy else 0)
    en = None
    if energy:
        en = energy_out
        if en is None:
            en = torch.empty((nsteps + 1, 2), dtype=torch.float64, device=pm.device)
        elif en.dtype != torch.float64 or not en.is_contiguous() or en.numel() < 2 * (nsteps + 1):
            raise ValueError("energy_out must be a contiguous float64 tensor of (nsteps+1)*2 entries")
    _check(lib().nbody_leapfrog_kdk(_ptr(pm), _ptr(v), _ptr(a), pm.shape[0], optr, nsys, p, float(G),
                                    float(eps), float(dt), int(nsteps), flags, _ptr(en), _stream()))
    return en


@_on_device
def kick_drift(pos_mass, vel, acc_pot, h, dt, close, open, prec=None):
    """Elementwise leapfrog half-step in place (see nbody.h)."""
    pm = _rec(pos_mass, "pos_mass")
    v = _rec(vel, "vel", pm.dtype)
    a = _rec(acc_pot, "acc_pot", pm.dtype)
    p = _prec(pm, prec)
    _check(lib().nbody_kick_drift(_ptr(pm), _ptr(v), _ptr(a), pm.shape[0], p, float(h), float(dt),
                                  1 if close else 0, 1 if open else 0, _stream()))


@_on_device
def batched_accel(pos_mass, offsets, eps, G=1.0, prec=None, eps_per_sys=None, out=None):
    pm = _rec(pos_mass, "pos_mass")
    p = _prec(pm, prec)
    o, nsys, optr = _offsets(offsets)
    if o is None:
        raise ValueError("offsets required")
    if out is None:
        out = torch.empty_like(pm)
    else:
        _out(out, pm.shape[0], pm)
    eptr = None
    if eps_per_sys is not None:
        if eps_per_sys.dtype != torch.float32 or eps_per_sys.device.type != "cuda" or \
                not eps_per_sys.is_contiguous() or eps_per_sys.numel() != nsys:
            raise ValueError("eps_per_sys must be a contiguous float32 GPU tensor of nsys entries")
        eptr = _ptr(eps_per_sys)
    _check(lib().nbody_batched_accel(_ptr(pm), optr, nsys, p, float(G), eptr, float(eps), _ptr(out),
                                     _stream()))
    return out


@_on_device
def energy(pos_mass, vel, acc_pot, prec=None):
    """FP64 (K, U) of one system as a 2-element float64 GPU tensor."""
    pm = _rec(pos_mass, "pos_mass")
    v = _rec(vel, "vel", pm.dtype)
    a = _rec(acc_pot, "acc_pot", pm.dtype)
    p = _prec(pm, prec)
    out = torch.empty(2, dtype=torch.float64, device=pm.device)
    _check(lib().nbody_energy(_ptr(pm), _ptr(v), _ptr(a), pm.shape[0], p, _ptr(out), _stream()))
    return out


@_on_device
def orb_order(pos_mass, leaf):
    """int32 permutation, perm[p] = original index at position p."""
    pm = _rec(pos_mass, "pos_mass")
    p = F64 if pm.dtype == torch.float64 else F32
    perm = torch.empty(pm.shape[0], dtype=torch.int32, device=pm.device)
    _check(lib().nbody_orb_order(_ptr(pm), p, pm.shape[0], int(leaf), _ptr(perm), _stream()))
    return perm


@_on_device
def permute(src, perm, inverse=False, out=None):
    s = _rec(src, "src")
    if perm.dtype != torch.int32 or perm.device != s.device or not perm.is_contiguous() or \
            perm.numel() != s.shape[0]:
        raise ValueError("perm must be a contiguous int32 GPU tensor of N entries")
    if out is None:
        out = torch.empty_like(s)
    else:
        _out(out, s.shape[0], s)
    _check(lib().nbody_permute(_ptr(s), _ptr(out), _ptr(perm), s.shape[0], s.element_size() * 4,
                               1 if inverse else 0, _stream()))
    return out


# ---- tree code on the ORB cells ------------------------------------------------
# Inputs are float32 (N, 4) records already in ORB order for the same leaf
# (orb_order, then permute); results are in that order too.  The default leaf
# of 4 bodies measured fastest at 2^20 (leaf 2, 4, 8, 16: 2.44, 2.38, 2.50,
# 3.81 ms at theta 0.7) with the same accuracy as 8.

def tree_shape(n, leaf, nodes=False):
    """(num_nodes, num_groups[, nodes int32 (num_nodes, 4) = begin, end,
    left, right]) of the ORB tree for n bodies and this leaf size."""
    nn, ng = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().nbody_tree_shape(int(n), int(leaf), ctypes.byref(nn), ctypes.byref(ng), None))
    if not nodes:
        return nn.value, ng.value
    import numpy as np
    tab = np.empty((nn.value, 4), dtype=np.int32)
    _check(lib().nbody_tree_shape(int(n), int(leaf), ctypes.byref(nn), ctypes.byref(ng),
                                  tab.ctypes.data_as(ctypes.c_void_p)))
    return nn.value, ng.value, tab


@_on_device
def tree_accel(pos_mass, eps, theta, leaf=4, G=1.0, prec=None, out=None, cells=CELLS_MONOPOLE):
    """Tree-code force and potential (ax, ay, az, phi) per body, ORB order.
    cells: CELLS_MONOPOLE (accepted cells as one body), CELLS_PSEUDO (as their
    12 pseudo-particles), CELLS_QUADRUPOLE (their quadrupole expansion) or
    CELLS_LOCAL (quadrupole cells, those far from the whole group through the
    group's local expansion)."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    p = _prec(pm, prec)
    if out is None:
        out = torch.empty_like(pm)
    else:
        _out(out, pm.shape[0], pm)
    _check(lib().nbody_tree_accel_cells(_ptr(pm), pm.shape[0], p, float(G), float(eps), float(theta),
                                        int(leaf), int(cells), _ptr(out), _stream()))
    return out


@_on_device
def fmm_accel(pos_mass, eps, theta, leaf=8, G=1.0, prec=None, out=None):
    """Force and potential (ax, ay, az, phi) per body, ORB order, by the
    multi-level fast multipole method on the ORB nodes (quadrupole cells,
    third-order local expansions)."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    p = _prec(pm, prec)
    if out is None:
        out = torch.empty_like(pm)
    else:
        _out(out, pm.shape[0], pm)
    _check(lib().nbody_fmm_accel(_ptr(pm), pm.shape[0], p, float(G), float(eps), float(theta), int(leaf),
                                 _ptr(out), _stream()))
    return out


@_on_device
def fmm_lists(pos_mass, theta, leaf=8):
    """The FMM's lists: (m2l_count, m2p_count, p2p_count) int32 (num_nodes,)
    and the concatenated source node ids (m2l, m2p, p2p), target nodes in id
    order, each target's sources in the device walk's fixed order."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    nn, _ = tree_shape(pm.shape[0], leaf)
    cnt = [torch.empty(nn, dtype=torch.int32, device=pm.device) for _ in range(3)]
    _check(lib().nbody_fmm_lists(_ptr(pm), pm.shape[0], int(leaf), float(theta), *(_ptr(c) for c in cnt),
                                 None, 0, None, 0, None, 0, _stream()))
    tot = [int(c.sum()) for c in cnt]
    ids = [torch.empty(max(t, 1), dtype=torch.int32, device=pm.device) for t in tot]
    args = []
    for a in ids:
        args += [_ptr(a), a.shape[0]]
    _check(lib().nbody_fmm_lists(_ptr(pm), pm.shape[0], int(leaf), float(theta), *(_ptr(c) for c in cnt), *args,
                                 _stream()))
    return (*cnt, *(a[:t] for a, t in zip(ids, tot)))


@_on_device
def tree_pseudo(pos_mass, leaf=4):
    """Pseudo-particles of every node, (num_nodes, 12, 4) float32 =
    (x, y, z, q), for ORB-ordered records."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    nn, _ = tree_shape(pm.shape[0], leaf)
    out = torch.empty((nn, TREE_PSEUDO, 4), dtype=torch.float32, device=pm.device)
    _check(lib().nbody_tree_pseudo(_ptr(pm), pm.shape[0], int(leaf), _ptr(out), _stream()))
    return out


@_on_device
def tree_local_counts(pos_mass, theta, leaf=4):
    """Per-group list sizes of the local-expansion walk: (loc, far, near)
    int32 (groups,)."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    _, ng = tree_shape(pm.shape[0], leaf)
    cnt = [torch.empty(ng, dtype=torch.int32, device=pm.device) for _ in range(3)]
    _check(lib().nbody_tree_local_counts(_ptr(pm), pm.shape[0], int(leaf), float(theta), _ptr(cnt[0]),
                                         _ptr(cnt[1]), _ptr(cnt[2]), _stream()))
    return tuple(cnt)


@_on_device
def tree_quad(pos_mass, leaf=4):
    """Quadrupole records of every node, (num_nodes, 3, 4) float32 =
    (com, M), (Qxx, Qyy, Qzz, Qxy), (Qxz, Qyz, 0, 0), for ORB-ordered records."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    nn, _ = tree_shape(pm.shape[0], leaf)
    out = torch.empty((nn, 3, 4), dtype=torch.float32, device=pm.device)
    _check(lib().nbody_tree_quad(_ptr(pm), pm.shape[0], int(leaf), _ptr(out), _stream()))
    return out


@_on_device
def tree_moments(pos_mass, leaf=4):
    """Node moments (num_nodes, 5) float64 = (M, com_x, com_y, com_z, diag2)
    and boxes (num_nodes, 6) float32 = (lo, hi)."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    nn, _ = tree_shape(pm.shape[0], leaf)
    mom = torch.empty((nn, 5), dtype=torch.float64, device=pm.device)
    box = torch.empty((nn, 6), dtype=torch.float32, device=pm.device)
    _check(lib().nbody_tree_moments(_ptr(pm), pm.shape[0], int(leaf), _ptr(mom), _ptr(box), _stream()))
    return mom, box


@_on_device
def tree_lists(pos_mass, theta, leaf=4, max_far=None, max_near=None):
    """Per-group interaction lists: (far_count, near_count) int32 (groups,)
    and, when the maxima are given, far_ids (groups, max_far) and near_ids
    (groups, max_near) node ids in walk order (entries past the counts are
    undefined)."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    _, ng = tree_shape(pm.shape[0], leaf)
    fc = torch.empty(ng, dtype=torch.int32, device=pm.device)
    nc = torch.empty(ng, dtype=torch.int32, device=pm.device)
    fi = None if not max_far else torch.empty((ng, int(max_far)), dtype=torch.int32, device=pm.device)
    ni = None if not max_near else torch.empty((ng, int(max_near)), dtype=torch.int32, device=pm.device)
    _check(lib().nbody_tree_lists(_ptr(pm), pm.shape[0], int(leaf), float(theta), int(max_far or 0),
                                  int(max_near or 0), _ptr(fc), _ptr(nc), None if fi is None else _ptr(fi),
                                  None if ni is None else _ptr(ni), _stream()))
    return fc, nc, fi, ni


@_on_device
def tree_leapfrog(pos_mass, vel, acc, eps, theta, dt, nsteps, leaf=4, reorder_every=0, order=None,
                  acc_valid=False, energy=False, G=1.0, prec=None, cells=CELLS_MONOPOLE):
    """Kick-drift-kick steps with tree forces, in place on ORB-ordered
    float32 records.  reorder_every = K > 0 re-orders the state by ORB at
    entry and every K steps and composes ``order`` (int32 (N,), created as
    the identity when None); cells as for tree_accel; returns (order,
    energies (nsteps+1, 2) or None)."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    v = _rec(vel, "vel", torch.float32)
    a = _rec(acc, "acc", torch.float32)
    p = _prec(pm, prec)
    n = pm.shape[0]
    if reorder_every and order is None:
        order = torch.arange(n, dtype=torch.int32, device=pm.device)
    if order is not None and (order.dtype != torch.int32 or order.numel() != n or not order.is_contiguous()):
        raise ValueError("order must be a contiguous int32 tensor of N entries")
    en = torch.empty((nsteps + 1, 2), dtype=torch.float64, device=pm.device) if energy else None
    if cells not in _TREE_CELL_FLAGS:
        raise ValueError("cells must be CELLS_MONOPOLE, CELLS_PSEUDO, CELLS_QUADRUPOLE or CELLS_LOCAL")
    flags = (ACC_VALID if acc_valid else 0) | (ENERGY if energy else 0) | _TREE_CELL_FLAGS[cells]
    _check(lib().nbody_tree_leapfrog(_ptr(pm), _ptr(v), _ptr(a), None if order is None else _ptr(order), n, p,
                                     float(G), float(eps), float(theta), int(leaf), float(dt), int(nsteps),
                                     int(reorder_every), flags, None if en is None else _ptr(en), _stream()))
    return order, en


@_on_device
def trajectory_forward(pos_mass, vel, eps, dt, nsteps, ckpt_every, G=1.0, prec=None):
    """Runs the leapfrog in place and returns the checkpoint tensor
    (nsteps/ckpt_every + 1, 2, N, 4)."""
    pm = _rec(pos_mass, "pos_mass")
    v = _rec(vel, "vel", pm.dtype)
    p = _prec(pm, prec)
    n = pm.shape[0]
    ck = torch.empty((nsteps // ckpt_every + 1, 2, n, 4), dtype=pm.dtype, device=pm.device)
    _check(lib().nbody_trajectory_forward(_ptr(pm), _ptr(v), n, p, float(G), float(eps), float(dt),
                                          int(nsteps), int(ckpt_every), _ptr(ck), _stream()))
    return ck


@_on_device
def trajectory_adjoint(ckpt, eps, dt, nsteps, ckpt_every, xbar_T, vbar_T, G=1.0, prec=None,
                       scheme=ADJ_REVERSE, phibar_T=None):
    """(pos_cot (N,4), vel_cot (N,4), mass_cot (N,)) = gradients at the
    initial state for final-state cotangents (xbar_T, vbar_T) and, if given,
    phibar_T (N,) on the final potential phi(x_T).  scheme: ADJ_RECOMPUTE
    (segments re-run from checkpoints) or ADJ_REVERSE (time reversal from each
    checkpoint, no extra force evaluations)."""
    xb = _rec(xbar_T, "xbar_T")
    vb = _rec(vbar_T, "vbar_T", xb.dtype)
    if phibar_T is not None:
        xb = xb.clone()
        xb[:, 3] = phibar_T.to(xb.dtype)
        scheme = int(scheme) | ADJ_PHI
    else:
        scheme = int(scheme) & ~ADJ_PHI
    if ckpt.dtype != xb.dtype or not ckpt.is_contiguous() or ckpt.device != xb.device:
        raise ValueError("ckpt must be a contiguous tensor of the same dtype and device")
    p = _prec(xb, prec)
    n = xb.shape[0]
    pc = torch.empty_like(xb)
    vc = torch.empty_like(xb)
    mc = torch.empty(n, dtype=xb.dtype, device=xb.device)
    _check(lib().nbody_trajectory_adjoint(_ptr(ckpt), n, p, float(G), float(eps), float(dt), int(nsteps),
                                          int(ckpt_every), _ptr(xb), _ptr(vb), _ptr(pc), _ptr(vc),
                                          _ptr(mc), int(scheme), _stream()))
    return pc, vc, mc


@_on_device
def janus_forward(pos_mass, vel, eps, dt, nsteps, shift_x=40, shift_v=40, G=1.0):
    """Bit-reversible fixed-point kick-drift-kick from float32 records.
    Returns (state int64 (2N, 4), final positions with masses (N, 4),
    final velocities (N, 4))."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    v = _rec(vel, "vel", torch.float32)
    n = pm.shape[0]
    state = torch.empty((2 * n, 4), dtype=torch.int64, device=pm.device)
    pm_out = torch.empty_like(pm)
    v_out = torch.empty_like(pm)
    _check(lib().nbody_janus_forward(_ptr(pm), _ptr(v), n, float(G), float(eps), float(dt), int(nsteps),
                                     int(shift_x), int(shift_v), _ptr(state), _ptr(pm_out), _ptr(v_out),
                                     _stream()))
    return state, pm_out, v_out


@_on_device
def janus_adjoint(state, pos_mass, eps, dt, nsteps, xbar_T, vbar_T, shift_x=40, shift_v=40, G=1.0):
    """Gradients (pos_cot, vel_cot (N, 4), mass_cot (N,)) for cotangents of the
    final state, rebuilding the trajectory backwards from ``state`` alone;
    ``state`` is rewound in place to the initial state (bit-exact)."""
    pm = _rec(pos_mass, "pos_mass", torch.float32)
    xb = _rec(xbar_T, "xbar_T", torch.float32)
    vb = _rec(vbar_T, "vbar_T", torch.float32)
    n = pm.shape[0]
    if state.dtype != torch.int64 or tuple(state.shape) != (2 * n, 4) or not state.is_contiguous():
        raise ValueError("state must be a contiguous int64 tensor of shape (2N, 4)")
    pc = torch.empty_like(xb)
    vc = torch.empty_like(xb)
    mc = torch.empty(n, dtype=torch.float32, device=pm.device)
    _check(lib().nbody_janus_adjoint(_ptr(state), _ptr(pm), n, float(G), float(eps), float(dt), int(nsteps),
                                     int(shift_x), int(shift_v), _ptr(xb), _ptr(vb), _ptr(pc), _ptr(vc), _ptr(mc),
                                     _stream()))
    return pc, vc, mc


class NBodyTrajectory(torch.autograd.Function):
    """x_T = leapfrog^nsteps(x0, v0; m), differentiable in (x0, v0, m).

    forward: checkpointed trajectory (nbody_trajectory_forward); backward:
    checkpointed adjoint (nbody_trajectory_adjoint).  x0, v0: (N, 3); m: (N,).
    Returns (x_T (N, 3), v_T (N, 3)), and with with_potential=True also the
    final potential phi(x_T) (N,), whose gradient takes the potential path of
    the adjoint (losses on the final energy)."""

    @staticmethod
    def forward(ctx, x0, v0, m, eps, dt, nsteps, ckpt_every=20, G=1.0, prec=None,
                scheme=ADJ_REVERSE, with_potential=False):
        n = x0.shape[0]
        pm = torch.empty((n, 4), dtype=x0.dtype, device=x0.device)
        pm[:, :3] = x0.detach()
        pm[:, 3] = m.detach()
        vel = torch.zeros((n, 4), dtype=x0.dtype, device=x0.device)
        vel[:, :3] = v0.detach()
        ck = trajectory_forward(pm, vel, eps, dt, nsteps, ckpt_every, G, prec)
        ctx.save_for_backward(ck)
        ctx.args = (eps, dt, nsteps, ckpt_every, G, prec, scheme, with_potential)
        if not with_potential:
            return pm[:, :3].clone(), vel[:, :3].clone()
        phi = accel(pm, eps, G, prec)[:, 3].clone()
        return pm[:, :3].clone(), vel[:, :3].clone(), phi

    @staticmethod
    def backward(ctx, gx, gv, gphi=None):
        (ck,) = ctx.saved_tensors
        eps, dt, nsteps, ckpt_every, G, prec, scheme, with_potential = ctx.args
        n = ck.shape[2]
        xb = torch.zeros((n, 4), dtype=ck.dtype, device=ck.device)
        vb = torch.zeros((n, 4), dtype=ck.dtype, device=ck.device)
        if gx is not None:
            xb[:, :3] = gx
        if gv is not None:
            vb[:, :3] = gv
        pc, vc, mc = trajectory_adjoint(ck, eps, dt, nsteps, ckpt_every, xb, vb, G, prec, scheme,
                                        phibar_T=gphi if with_potential else None)
        return pc[:, :3], vc[:, :3], mc, None, None, None, None, None, None, None, None


class ReversibleTrajectory(torch.autograd.Function):
    """x_T = leapfrog^nsteps(x0, v0; m) on the bit-reversible fixed-point
    state (janus_forward), differentiable in (x0, v0, m) through the
    checkpoint-free adjoint (janus_adjoint): the only memory kept is the final
    int64 state (64 bytes per body), whatever nsteps is.  x0, v0: (N, 3);
    m: (N,) positive; float32.  Returns (x_T (N, 3), v_T (N, 3)).  Rounding
    to the fixed-point grid is treated as the identity in the derivative."""

    @staticmethod
    def forward(ctx, x0, v0, m, eps, dt, nsteps, G=1.0, shift_x=40, shift_v=40):
        n = x0.shape[0]
        pm = torch.empty((n, 4), dtype=torch.float32, device=x0.device)
        pm[:, :3] = x0.detach()
        pm[:, 3] = m.detach()
        vel = torch.zeros((n, 4), dtype=torch.float32, device=x0.device)
        vel[:, :3] = v0.detach()
        st, pT, vT = janus_forward(pm, vel, eps, dt, nsteps, shift_x, shift_v, G)
        ctx.save_for_backward(st, pm)
        ctx.args = (eps, dt, nsteps, G, shift_x, shift_v)
        return pT[:, :3].clone(), vT[:, :3].clone()

    @staticmethod
    def backward(ctx, gx, gv):
        st, pm = ctx.saved_tensors
        eps, dt, nsteps, G, shift_x, shift_v = ctx.args
        st = st.clone()  # the adjoint rewinds the state in place
        n = pm.shape[0]
        xb = torch.zeros((n, 4), dtype=torch.float32, device=pm.device)
        vb = torch.zeros((n, 4), dtype=torch.float32, device=pm.device)
        if gx is not None:
            xb[:, :3] = gx
        if gv is not None:
            vb[:, :3] = gv
        pc, vc, mc = janus_adjoint(st, pm, eps, dt, nsteps, xb, vb, shift_x, shift_v, G)
        return pc[:, :3], vc[:, :3], mc, None, None, None, None, None, None


def autotune(kernel, prec, n, offsets=None):
    o, nsys, optr = _offsets(offsets)
    _check(lib().nbody_autotune(int(kernel), int(prec), int(n), optr, nsys, _stream()))


def set_tuning(kernel, prec, tpl=-1, jsplit=-1, jtile=-1, variant=0):
    """Pin (tpl, jsplit, jtile, variant) for a kernel and precision; no
    shape arguments clears the pin."""
    _check(lib().nbody_set_tuning(int(kernel), int(prec), int(tpl), int(jsplit), int(jtile), int(variant)))


def get_tuning(kernel, prec, n):
    """(tpl, jsplit, jtile, variant) the library would use for size n."""
    a, b, c, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().nbody_get_tuning(int(kernel), int(prec), int(n), ctypes.byref(a), ctypes.byref(b),
                                  ctypes.byref(c), ctypes.byref(d)))
    return a.value, b.value, c.value, d.value


def release():
    lib().nbody_release()
