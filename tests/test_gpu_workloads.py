"""End-to-end checks of the measured workloads against the FP64 oracle:
the Plummer and colliding-pair integrations (force error on sampled targets
at the start and on the GPU's own final state), the trajectory gradient,
the ragged batch in one captured graph, and the autotuner."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import ics
from nbtest import gpu, host, normwise, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_plummer65536_orb_ordered_100_steps(orc):
    """Plummer N = 65536, FP32 + Kahan, ORB order, eps 0.01, 100 KDK steps
    dt = 1e-3: force error <= 1e-5 on 1024 sampled targets at step 0 and at
    step 100 (oracle on the GPU's own state); FP64 energy drift reported."""
    torch, nb = gpu()
    w = ics.WORKLOADS["plummer65536"]
    pm, v = ics.plummer(w["n"], w["seed"])
    p = to_dev(torch, widen32(pm), torch.float32)
    vv = to_dev(torch, widen32(v), torch.float32)
    perm = nb.orb_order(p, 128)
    p, vv = nb.permute(p, perm), nb.permute(vv, perm)
    a = torch.empty_like(p)
    tg = ics.sample_targets(w["n"], 1024, w["seed"] + 1)
    en = nb.leapfrog_kdk(p, vv, a, w["eps"], w["dt"], 0, prec=nb.F32_KAHAN, energy=True)
    torch.cuda.synchronize()
    ph = host(p)
    acc, pot = orc.accel(ph, w["eps"], targets=tg)
    assert rms_rel(host(a)[tg, :3], acc) <= 1e-5
    en = nb.leapfrog_kdk(p, vv, a, w["eps"], w["dt"], w["steps"], prec=nb.F32_KAHAN, acc_valid=True, energy=True)
    torch.cuda.synchronize()
    ph = host(p)
    acc, pot = orc.accel(ph, w["eps"], targets=tg)
    e = rms_rel(host(a)[tg, :3], acc)
    ep = rms_rel(host(a)[tg, 3], pot)
    E = en.cpu().numpy().sum(axis=1)
    print(f"plummer65536 step 100: force rms rel {e:.2e}, pot {ep:.2e}, energy drift {E[-1] / E[0] - 1:.2e}")
    assert e <= 1e-5 and ep <= 1e-5
    assert abs(E[-1] / E[0] - 1) < 1e-4


@pytest.mark.parametrize("mode", ["F32_F64ACC", "F32_KAHAN", "F32"])
def test_collide1m_20_steps(orc, mode):
    """Colliding pair N = 2^20, eps 0.005, 20 steps dt = 5e-4: force error on
    sampled targets at step 0 and at step 20 on the GPU's own state."""
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    pm, v = ics.colliding_pair(w["n"], w["seed"])
    p = to_dev(torch, widen32(pm), torch.float32)
    vv = to_dev(torch, widen32(v), torch.float32)
    a = torch.empty_like(p)
    prec = getattr(nb, mode)
    tg = ics.sample_targets(w["n"], 128, w["seed"] + 1)
    nb.leapfrog_kdk(p, vv, a, w["eps"], w["dt"], 0, prec=prec)
    torch.cuda.synchronize()
    acc0, _ = orc.accel(host(p), w["eps"], targets=tg)
    e0 = rms_rel(host(a)[tg, :3], acc0)
    nb.leapfrog_kdk(p, vv, a, w["eps"], w["dt"], w["steps"], prec=prec, acc_valid=True)
    torch.cuda.synchronize()
    acc1, _ = orc.accel(host(p), w["eps"], targets=tg)
    e1 = rms_rel(host(a)[tg, :3], acc1)
    print(f"collide1m {mode}: step 0 {e0:.2e}, step 20 {e1:.2e}")
    assert e0 <= 1e-5 and e1 <= 1e-5


def test_gradient_plummer_200_steps(orc):
    """Differentiation workload at reduced N (the oracle's full-size gradient
    takes minutes): Plummer N = 2048, FP32 + Kahan, 200 steps dt = 1e-3,
    checkpoints every 20, gradient of sum |x_T - y|^2 against the FP64
    oracle.  No closed form pins this through 200 chaotic steps; the bar is
    the FP32 rounding propagated through the integration."""
    torch, nb = gpu()
    n, eps, dt, steps, C = 2048, 0.01, 1e-3, 200, 20
    pm, v = ics.plummer(n, 1003)
    y = ics.perturbed_snapshot(pm, 1005)
    pm32, v32 = widen32(pm), widen32(v)
    L, gx, gv, gm = orc.traj_grad(pm32, v32, y, eps, dt, steps)
    for scheme in (nb.ADJ_REVERSE, nb.ADJ_RECOMPUTE):
        p, vv = to_dev(torch, pm32, torch.float32), to_dev(torch, v32, torch.float32)
        ck = nb.trajectory_forward(p, vv, eps, dt, steps, C, prec=nb.F32_KAHAN)
        xb = torch.zeros_like(p)
        xb[:, :3] = 2 * (p[:, :3] - to_dev(torch, y, torch.float32))
        pc, vc, mc = nb.trajectory_adjoint(ck, eps, dt, steps, C, xb, torch.zeros_like(p),
                                           prec=nb.F32_KAHAN, scheme=scheme)
        torch.cuda.synchronize()
        ex, ev, em = normwise(host(pc)[:, :3], gx), normwise(host(vc)[:, :3], gv), normwise(host(mc), gm)
        print(f"gradient scheme {scheme}: x {ex:.2e} v {ev:.2e} m {em:.2e}")
        assert max(ex, ev, em) <= 1e-4


def test_gradient_plummer16384_200_steps_full_size():
    """The differentiation workload at its own size: Plummer N = 16384, FP32
    + Kahan, 200 steps dt = 1e-3, checkpoints every 20, both adjoint schemes,
    against the FP64 oracle's reverse-mode gradient (stored on 1024 sampled
    bodies by tests/golden/make_traj_grad_plummer16384.py, which calls only
    the oracle).  Bar: 1e-4 normwise on each of dL/dx0, dL/dv0, dL/dm."""
    torch, nb = gpu()
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_traj_grad_plummer16384 as mk
    ref = np.load(mk.OUT)
    w, pm, v, y = mk.inputs()
    assert str(ref["inputs_sha256"]) == mk.digest(pm, v, y), "fixture made from other inputs"
    idx = ref["idx"]
    n, eps, dt, steps, C = w["n"], w["eps"], w["dt"], w["steps"], w["ckpt"]
    yd = to_dev(torch, y, torch.float32)
    for scheme in (nb.ADJ_REVERSE, nb.ADJ_RECOMPUTE):
        p, vv = to_dev(torch, pm, torch.float32), to_dev(torch, v, torch.float32)
        ck = nb.trajectory_forward(p, vv, eps, dt, steps, C, prec=nb.F32_KAHAN)
        xb = torch.zeros_like(p)
        xb[:, :3] = 2 * (p[:, :3] - yd)
        loss = float(((p[:, :3].double() - yd.double()) ** 2).sum())
        pc, vc, mc = nb.trajectory_adjoint(ck, eps, dt, steps, C, xb, torch.zeros_like(p),
                                           prec=nb.F32_KAHAN, scheme=scheme)
        torch.cuda.synchronize()
        ex = normwise(host(pc)[idx, :3], ref["gx"])
        ev = normwise(host(vc)[idx, :3], ref["gv"])
        em = normwise(host(mc)[idx], ref["gm"])
        el = abs(loss / float(ref["L"]) - 1)
        print(f"N=16384 gradient scheme {scheme}: x {ex:.2e} v {ev:.2e} m {em:.2e}, loss {el:.2e}")
        assert max(ex, ev, em) <= 1e-4
        assert el <= 1e-5


def test_batch512_graph_50_steps_matches_eager_and_oracle(orc):
    """512 ragged Plummer systems, 50 steps in one captured graph: equal to
    eager launches bit for bit; sampled forces of the final state against the
    oracle."""
    torch, nb = gpu()
    w = ics.WORKLOADS["batch512"]
    pm, v, off = ics.ragged_batch(w["nsys"], w["seed"])
    pg, vg = to_dev(torch, pm, torch.float32), to_dev(torch, v, torch.float32)
    pe, ve = pg.clone(), vg.clone()
    ag, ae = torch.empty_like(pg), torch.empty_like(pe)
    nb.leapfrog_kdk(pg, vg, ag, w["eps"], w["dt"], w["steps"], offsets=off, graph=True)
    torch.cuda.synchronize()
    nb.leapfrog_kdk(pe, ve, ae, w["eps"], w["dt"], w["steps"], offsets=off)
    torch.cuda.synchronize()
    assert torch.equal(pg, pe) and torch.equal(vg, ve) and torch.equal(ag, ae)
    ph, ah = host(pg), host(ag)
    g = ics.rng(w["seed"] + 2)
    for s in g.choice(w["nsys"], 8, replace=False):
        a0, a1 = off[s], off[s + 1]
        tg = ics.sample_targets(a1 - a0, 32, int(s))
        acc, _ = orc.accel(ph[a0:a1], w["eps"], targets=tg)
        assert rms_rel(ah[a0 + tg, :3], acc) <= 1e-5


def test_autotune_and_cache(tmp_path):
    """nbody_autotune picks a valid shape per kernel, results stay correct,
    and the JSON cache round-trips (fresh processes)."""
    cache = tmp_path / "tune.json"
    code = r'''
import sys, json
sys.path.insert(0, %r)
import numpy as np, torch, ics
import paper_1211_2292_amd as nb
n = 6000
nb.autotune(0, nb.F32_KAHAN, n)
nb.autotune(2, nb.F32_KAHAN, 4000)
off = np.array([0, 300, 2000, 2600], dtype=np.int64)
nb.autotune(1, nb.F32_KAHAN, 2600, offsets=off)
print(json.dumps([nb.get_tuning(0, nb.F32_KAHAN, n), nb.get_tuning(2, nb.F32_KAHAN, 4000), nb.get_tuning(1, nb.F32_KAHAN, 2600)]))
''' % ROOT
    env = dict(os.environ, NBODY_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    shapes = json.loads(r.stdout.strip().splitlines()[-1])
    assert cache.exists()
    text = cache.read_text()
    assert text.count("[") >= 3
    code2 = r'''
import sys, json
sys.path.insert(0, %r)
import paper_1211_2292_amd as nb
print(json.dumps([nb.get_tuning(0, nb.F32_KAHAN, 6000), nb.get_tuning(2, nb.F32_KAHAN, 4000), nb.get_tuning(1, nb.F32_KAHAN, 2600)]))
''' % ROOT
    r2 = subprocess.run([sys.executable, "-c", code2], env=env, capture_output=True, text=True, timeout=120)
    assert r2.returncode == 0, r2.stderr[-2000:]
    assert json.loads(r2.stdout.strip().splitlines()[-1]) == shapes


def test_autotuned_accuracy_unordered(tmp_path):
    """After nbody_autotune has chosen the force kernel's shape for sizes
    4096 ... 65536, unordered Plummer input (no ORB) still meets the 1e-5 RMS
    force bar of the compensated modes against the FP64 oracle: the tuner
    only moves tile and split boundaries.  Runs in a fresh process so the
    tuned table does not leak into other tests."""
    code = r'''
import sys, json
sys.path.insert(0, %r)
import numpy as np, torch, ics, oracle
import paper_1211_2292_amd as nb
out = []
for mode in ("F32_KAHAN", "F32_F64ACC"):
    prec = getattr(nb, mode)
    for n in (4096, 8192, 16384, 65536):
        nb.autotune(0, prec, n)
        shape = nb.get_tuning(0, prec, n)
        pm, _ = ics.plummer(n, 2100 + n)
        pm32 = pm.astype(np.float32)
        a = nb.accel(torch.as_tensor(pm32, device="cuda"), 0.01, prec=prec).cpu().numpy()
        tg = ics.sample_targets(n, min(n, 2048), 2101 + n)
        acc, pot = oracle.accel(pm32.astype(np.float64), 0.01, targets=tg)
        e = float(np.sqrt(np.mean((np.linalg.norm(a[tg, :3] - acc, axis=1) / np.linalg.norm(acc, axis=1)) ** 2)))
        ep = float(np.sqrt(np.mean(((a[tg, 3] - pot) / pot) ** 2)))
        out.append([mode, n, list(shape), e, ep])
print(json.dumps(out))
''' % ROOT
    env = dict(os.environ, NBODY_TUNE_CACHE=str(tmp_path / "tune.json"))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    for mode, n, shape, e, ep in json.loads(r.stdout.strip().splitlines()[-1]):
        print(f"tuned {mode} n={n} shape={shape}: force {e:.2e}, potential {ep:.2e}")
        assert shape[3] == 0
        assert e <= 1e-5 and ep <= 1e-5


def test_release_and_reuse():
    torch, nb = gpu()
    pm, v = ics.plummer(3000, 77)
    p = to_dev(torch, pm, torch.float32)
    a = nb.accel(p, 0.01)
    vv = to_dev(torch, v, torch.float32)
    acc = torch.empty_like(p)
    nb.leapfrog_kdk(p.clone(), vv.clone(), acc, 0.01, 1e-3, 3, graph=True)
    torch.cuda.synchronize()
    nb.release()
    b = nb.accel(p, 0.01)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
