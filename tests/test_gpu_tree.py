"""Tree code on the ORB cells (paper Section IV.A walk and monopole cells over
the Section IV.B ORB recursion) on the device against the oracle.

Moments and interaction lists are integer/decision work defined in FP64 with
a fixed operation order, so they must match the oracle bit for bit; forces
are FP32 pair arithmetic over the same lists and are held to an RMS relative
error of 1e-6 in the compensated modes (2e-6 in plain FP32), inside the 2e-6
bar of the direct-sum parity tests (the oracle evaluates the same lists in
FP64 with the cells at their exact FP64 centres of mass).
"""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, max_rel, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu


def _orb_input(torch, nb, pm, leaf):
    """Bodies gathered into the device ORB order (FP32), plus the host copy."""
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    perm = nb.orb_order(p, leaf)
    q = nb.permute(p, perm)
    torch.cuda.synchronize()
    return q, q.cpu().numpy()


@pytest.mark.parametrize("n,leaf", [(1, 1), (5, 8), (64, 8), (65, 8), (1000, 1), (3000, 8), (20001, 16),
                                    (50000, 4), (4096, 64)])
def test_moments_bitexact(orc, n, leaf):
    torch, nb = gpu()
    pm, _ = ics.plummer(max(n, 2), 300 + n)
    q, qh = _orb_input(torch, nb, pm[:n], leaf)
    mom, box = nb.tree_moments(q, leaf)
    torch.cuda.synchronize()
    mom, box = mom.cpu().numpy(), box.cpu().numpy()
    want = orc.tree_moments(qh, leaf)
    assert np.array_equal(mom[:, 0], want["mass"])
    assert np.array_equal(mom[:, 1:4], want["com"])
    assert np.array_equal(mom[:, 4], want["diag2"])
    assert np.array_equal(box[:, :3].astype(np.float64), want["lo"])
    assert np.array_equal(box[:, 3:].astype(np.float64), want["hi"])


def test_moments_zero_masses_and_repeat(orc):
    """Massless cells take the box centre; a second call on the same shape
    (counters reset by the first) gives the same bits."""
    torch, nb = gpu()
    pm, _ = ics.uniform_ball(4000, 310)
    pm = pm.copy()
    pm[::3, 3] = 0.0
    pm[pm[:, 0] < -0.4, 3] = 0.0  # a massless region: whole cells without mass
    q, qh = _orb_input(torch, nb, pm, 8)
    want = orc.tree_moments(qh, 8)
    for _ in range(2):
        mom, _ = nb.tree_moments(q, 8)
        torch.cuda.synchronize()
        mom = mom.cpu().numpy()
        assert np.array_equal(mom[:, 0], want["mass"])
        assert np.array_equal(mom[:, 1:4], want["com"])
    assert (want["mass"] == 0).any()


def _oracle_sets(orc, qh, leaf, theta):
    """Oracle lists per group, without the leaves inside the group (the
    device sums those as the group's own range)."""
    nodes = orc.tree_nodes(qh.shape[0], leaf)
    L = orc.tree_lists(qh, leaf, 64, theta)
    fo = np.r_[0, np.cumsum(L["far_cnt"])]
    no = np.r_[0, np.cumsum(L["near_cnt"])]
    far, near = [], []
    for g, gid in enumerate(L["group_id"]):
        gb, ge = nodes[gid, :2]
        far.append(set(L["far"][fo[g]:fo[g + 1]].tolist()))
        near.append({int(c) for c in L["near"][no[g]:no[g + 1]] if not (gb <= nodes[c, 0] and nodes[c, 1] <= ge)})
    return far, near


@pytest.mark.parametrize("n,leaf,theta,kind", [
    (3000, 8, 0.5, "plummer"), (3000, 8, 1.2, "plummer"), (20000, 8, 0.7, "collide"),
    (20000, 4, 0.4, "ball"), (9000, 16, 3.0, "plummer"), (776, 1, 0.8, "collide"), (5000, 8, 0.0, "ball")])
def test_lists_match_oracle(orc, n, leaf, theta, kind):
    torch, nb = gpu()
    gen = {"plummer": ics.plummer, "collide": ics.colliding_pair, "ball": ics.uniform_ball}[kind]
    pm, _ = gen(n, 320 + n)
    q, qh = _orb_input(torch, nb, pm, leaf)
    fc, ncnt, _, _ = nb.tree_lists(q, theta, leaf)
    torch.cuda.synchronize()
    mf, mn = int(fc.max().item()), int(ncnt.max().item())
    fc, ncnt, fi, ni = nb.tree_lists(q, theta, leaf, max(mf, 1), max(mn, 1))
    torch.cuda.synchronize()
    fc, ncnt, fi, ni = fc.cpu().numpy(), ncnt.cpu().numpy(), fi.cpu().numpy(), ni.cpu().numpy()
    far, near = _oracle_sets(orc, qh, leaf, theta)
    assert len(far) == fc.shape[0]
    for g in range(fc.shape[0]):
        assert fc[g] == len(far[g]) and ncnt[g] == len(near[g]), g
        assert set(fi[g, :fc[g]].tolist()) == far[g], g
        assert set(ni[g, :ncnt[g]].tolist()) == near[g], g
    if theta == 0.0:
        assert fc.sum() == 0


@pytest.mark.parametrize("prec,tol_rms,tol_max", [("F32_F64ACC", 1e-6, 2e-5), ("F32_KAHAN", 1e-6, 2e-5),
                                                  ("F32", 2e-6, 1e-4)])
@pytest.mark.parametrize("theta", [0.0, 0.5, 1.0])
def test_force_matches_oracle(orc, prec, tol_rms, tol_max, theta):
    torch, nb = gpu()
    n, leaf, eps = 12000, 8, 0.01
    pm, _ = ics.plummer(n, 330)
    q, qh = _orb_input(torch, nb, pm, leaf)
    out = nb.tree_accel(q, eps, theta, leaf, prec=getattr(nb, prec))
    torch.cuda.synchronize()
    got = host(out)
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps)
    assert rms_rel(got[:, :3], a) < tol_rms
    assert max_rel(got[:, :3], a) < tol_max
    assert rms_rel(got[:, 3], p) < tol_rms


def test_theta_zero_equals_direct_sum(orc):
    """theta = 0 accepts no cell: the tree force is the exact direct sum."""
    torch, nb = gpu()
    n, leaf, eps = 9000, 8, 0.005
    pm, _ = ics.colliding_pair(n, 340)
    q, qh = _orb_input(torch, nb, pm, leaf)
    tr = host(nb.tree_accel(q, eps, 0.0, leaf, prec=nb.F32_F64ACC))
    di = host(nb.accel(q, eps, prec=nb.F32_F64ACC))
    ad, pd = orc.accel(widen32(qh), eps)
    assert rms_rel(tr[:, :3], ad) < 1e-6 and rms_rel(di[:, :3], ad) < 1e-6
    assert rms_rel(tr[:, :3], di[:, :3]) < 1e-6
    assert rms_rel(tr[:, 3], pd) < 1e-6


@pytest.mark.parametrize("n", [1, 2, 7, 63, 64, 65, 129, 1000])
def test_small_and_ragged(orc, n):
    torch, nb = gpu()
    pm, _ = ics.uniform_ball(max(n, 2), 350 + n)
    pm = pm[:n].copy()
    pm[:, 3] = 1.0 / n
    q, qh = _orb_input(torch, nb, pm, 4)
    got = host(nb.tree_accel(q, 0.05, 0.8, 4, prec=nb.F32_F64ACC))
    a, p = orc.tree_accel(widen32(qh), 4, 64, 0.8, 0.05)
    if n == 1:
        assert np.all(got == 0.0)
        return
    assert rms_rel(got[:, :3], a) < 1e-6
    assert rms_rel(got[:, 3], p) < 1e-6


def test_eps_zero_and_massless(orc):
    """eps = 0 with distinct positions and a share of massless bodies (test
    particles feel the field, exert none)."""
    torch, nb = gpu()
    n = 6000
    pm, _ = ics.plummer(n, 360)
    pm = pm.copy()
    pm[::4, 3] = 0.0
    q, qh = _orb_input(torch, nb, pm, 8)
    got = host(nb.tree_accel(q, 0.0, 0.6, 8, prec=nb.F32_F64ACC))
    a, p = orc.tree_accel(widen32(qh), 8, 64, 0.6, 0.0)
    assert np.isfinite(got).all()
    assert rms_rel(got[:, :3], a) < 1e-6


def test_large_sampled_and_error_against_direct(orc):
    """N = 2^20 colliding pair, the launch the benchmark times: sampled
    targets against the oracle's tree force, and the monopole truncation
    against the exact sum reported for the record."""
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    n, eps, leaf, theta = w["n"], w["eps"], 8, 0.7
    pm, _ = ics.colliding_pair(n, w["seed"])
    q, qh = _orb_input(torch, nb, pm, leaf)
    got = host(nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC))
    tg = np.random.default_rng(7).choice(n, 384, replace=False)
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps, targets=tg)
    assert rms_rel(got[tg, :3], a) < 1e-6
    assert rms_rel(got[tg, 3], p) < 1e-6
    ad, _ = orc.accel(widen32(qh), eps, targets=tg)
    trunc = rms_rel(got[tg, :3], ad)
    print(f"tree theta {theta}: rms relative error against the direct sum {trunc:.3e}")
    assert trunc < 0.1 * theta ** 2


@pytest.mark.parametrize("n,ng,cells,ocells", [(1 << 19, 8192, "CELLS_LOCAL", 4), (1 << 19, 8192, "CELLS_MONOPOLE", 0),
                                              (1100001, 29241, "CELLS_LOCAL", 4)])
def test_dispatch_order_changes_nothing(orc, n, ng, cells, ocells):
    """With 8192 groups or more the local-expansion walk runs the groups with
    the largest boxes first (the monopole walk keeps ORB order either way).
    Every body's result equals the ORB-order walk's (NBODY_TREE_ORDER=0) bit
    for bit, every output record is written, and sampled targets match the
    oracle.  A Plummer sphere of 2^19 bodies with leaf 4 has exactly 8192
    groups of 64; 1100001 bodies give 29241 groups, more than one chunk of
    the ordering kernel and not a multiple of its 1024 threads."""
    import os
    torch, nb = gpu()
    leaf, theta, eps = 4, 0.6, 0.01
    pm, _ = ics.plummer(n, 780)
    q, qh = _orb_input(torch, nb, pm, leaf)
    assert nb.tree_shape(n, leaf)[1] == ng
    c = getattr(nb, cells)
    out = torch.full_like(q, float("nan"))
    nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, out=out, cells=c)
    os.environ["NBODY_TREE_ORDER"] = "0"
    try:
        ref = torch.full_like(q, float("nan"))
        nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, out=ref, cells=c)
    finally:
        del os.environ["NBODY_TREE_ORDER"]
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    assert torch.equal(out, ref)
    tg = np.random.default_rng(9).choice(n, 64, replace=False)
    a, p = orc.tree_accel(widen32(qh), leaf, 64, theta, eps, targets=tg, cells=ocells)
    got = host(out)
    assert rms_rel(got[tg, :3], a) < 1e-6
    assert rms_rel(got[tg, 3], p) < 1e-6


def test_repeat_and_shape_change_same_bits():
    """Cached tables: the same call twice gives the same bits, also after a
    call of another shape in between."""
    torch, nb = gpu()
    pm, _ = ics.plummer(5000, 370)
    q, _ = _orb_input(torch, nb, pm, 8)
    pm2, _ = ics.plummer(3000, 371)
    q2, _ = _orb_input(torch, nb, pm2, 16)
    r1 = host(nb.tree_accel(q, 0.01, 0.7, 8))
    _ = host(nb.tree_accel(q2, 0.01, 0.7, 16))
    r2 = host(nb.tree_accel(q, 0.01, 0.7, 8))
    assert np.array_equal(r1, r2)


# ---- tree leapfrog -----------------------------------------------------------------

def _kdk_oracle(orc, q, v, eps, dt, steps, accel):
    """FP64 kick-drift-kick (one force evaluation per step) with the given
    oracle force on the fixed ORB order."""
    x = widen32(q).copy()
    vv = np.asarray(v, dtype=np.float64)[:, :3].copy()
    a, _ = accel(x)
    for _ in range(steps):
        vv += 0.5 * dt * a
        x[:, :3] += dt * vv
        a, _ = accel(x)
        vv += 0.5 * dt * a
    return x, vv


def test_tree_leapfrog_is_kdk_with_tree_forces(orc):
    """Ten steps taken one call at a time: every force the integrator used
    is the oracle's tree force at the integrator's own positions (FP32
    tolerance), every step satisfies the kick-drift-kick recurrence, and one
    ten-step call reproduces the ten single steps.  The trajectory as a whole
    stays closer to the oracle's tree-force integration than to the direct
    sum (the tree decisions depend on the last bits of the positions, so the
    two FP64/FP32 trajectories are compared only this way)."""
    torch, nb = gpu()
    n, leaf, theta, eps, dt, steps = 3000, 8, 0.6, 0.01, 1e-3, 10
    pm, v0 = ics.plummer(n, 380)
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    perm = nb.orb_order(p, leaf)
    q = nb.permute(p, perm)
    v = nb.permute(to_dev(torch, np.c_[v0[:, :3], np.zeros(n)].astype(np.float32), torch.float32), perm)
    q1, v1 = q.clone(), v.clone()
    qh, vh = q.cpu().numpy(), v.cpu().numpy()
    a = nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC)
    h = 0.5 * dt
    for _ in range(steps):
        xk, vk, ak = host(q), host(v), host(a)
        at, _ = orc.tree_accel(xk, leaf, 64, theta, eps)
        assert rms_rel(ak[:, :3], at) < 1e-6
        nb.tree_leapfrog(q, v, a, eps, theta, dt, 1, leaf, acc_valid=True, prec=nb.F32_F64ACC)
        x1, v1_, a1 = host(q), host(v), host(a)
        np.testing.assert_allclose(x1[:, :3], xk[:, :3] + dt * (vk[:, :3] + h * ak[:, :3]), rtol=0, atol=1e-6)
        np.testing.assert_allclose(v1_[:, :3], vk[:, :3] + h * (ak[:, :3] + a1[:, :3]), rtol=0, atol=1e-6)
    a1 = torch.empty_like(q1)
    nb.tree_leapfrog(q1, v1, a1, eps, theta, dt, steps, leaf, prec=nb.F32_F64ACC)
    assert rms_rel(host(q1)[:, :3], host(q)[:, :3]) < 1e-7
    assert rms_rel(host(v1)[:, :3] - vh[:, :3], host(v)[:, :3] - vh[:, :3]) < 1e-6
    dv = host(v)[:, :3] - vh[:, :3].astype(np.float64)
    base = vh[:, :3].astype(np.float64)
    _, vt = _kdk_oracle(orc, qh, vh, eps, dt, steps, lambda x: orc.tree_accel(x, leaf, 64, theta, eps))
    _, vd = _kdk_oracle(orc, qh, vh, eps, dt, steps, lambda x: orc.accel(x, eps))
    e_tree, e_direct = rms_rel(dv, vt - base), rms_rel(dv, vd - base)
    print(f"tree leapfrog: dv against tree oracle {e_tree:.2e}, against direct sum {e_direct:.2e}")
    assert e_tree < 0.5 * e_direct


def test_tree_leapfrog_theta_zero_and_reordering_match_direct(orc):
    """theta = 0 is the exact sum, so the tree leapfrog with re-ordering every
    3 steps, mapped back through `order`, equals the direct leapfrog on the
    caller's order up to FP32 rounding; `order` stays a permutation."""
    torch, nb = gpu()
    n, leaf, eps, dt, steps = 2500, 8, 0.02, 2e-3, 10
    pm, v0 = ics.plummer(n, 390)
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    v = to_dev(torch, np.c_[v0[:, :3], np.zeros(n)].astype(np.float32), torch.float32)
    a = torch.empty_like(p)
    pd, vd, ad = p.clone(), v.clone(), torch.empty_like(p)
    order, _ = nb.tree_leapfrog(p, v, a, eps, 0.0, dt, steps, leaf, reorder_every=3, prec=nb.F32_F64ACC)
    nb.leapfrog_kdk(pd, vd, ad, eps, dt, steps, prec=nb.F32_F64ACC)
    o = order.cpu().numpy()
    assert np.array_equal(np.sort(o), np.arange(n))
    back_x = np.empty((n, 4)); back_v = np.empty((n, 4))
    back_x[o] = host(p); back_v[o] = host(v)
    assert rms_rel(back_x[:, :3], host(pd)[:, :3]) < 1e-6
    assert rms_rel(back_v[:, :3] - v0[:, :3], host(vd)[:, :3] - v0[:, :3]) < 1e-5
    assert np.array_equal(back_x[:, 3], host(pd)[:, 3])


def test_tree_leapfrog_energy():
    """Energy output of the tree leapfrog (tree potential) over 200 steps of
    a Plummer sphere, re-ordered every 20 steps: the FP64 energies are
    reported per step and the drift stays small."""
    torch, nb = gpu()
    n, leaf, theta, eps, dt, steps = 16384, 8, 0.5, 0.01, 1e-3, 200
    pm, v0 = ics.plummer(n, 400)
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    v = to_dev(torch, np.c_[v0[:, :3], np.zeros(n)].astype(np.float32), torch.float32)
    a = torch.empty_like(p)
    _, en = nb.tree_leapfrog(p, v, a, eps, theta, dt, steps, leaf, reorder_every=20, energy=True,
                             prec=nb.F32_F64ACC)
    e = en.cpu().numpy().sum(1)
    drift = np.abs(e / e[0] - 1.0).max()
    print(f"tree leapfrog energy: max |dE/E| over {steps} steps {drift:.2e}")
    assert np.isfinite(e).all()
    assert drift < 1e-3
    k_end, u_end = nb.energy(p, v, a).cpu().numpy()
    assert abs((k_end + u_end) / e[-1] - 1.0) < 1e-12


@pytest.mark.parametrize("n,cells", [(20000, "CELLS_MONOPOLE"), (1 << 19, "CELLS_LOCAL")])
def test_tree_force_replays_in_a_captured_graph(n, cells):
    """After the first call for a shape (which uploads the node table), the
    tree force is kernel launches only: captured in a HIP graph it replays
    bit for bit like eager calls, with eager work in between.  At 2^19
    bodies the local-expansion walk's dispatch-order kernels are captured
    too."""
    torch, nb = gpu()
    c = getattr(nb, cells)
    pm, _ = ics.plummer(n, 410)
    q, _ = _orb_input(torch, nb, pm, 4)
    out_e = nb.tree_accel(q, 0.01, 0.6, 4, prec=nb.F32_F64ACC, cells=c)
    out_g = torch.empty_like(q)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        nb.tree_accel(q, 0.01, 0.6, 4, prec=nb.F32_F64ACC, out=out_g, cells=c)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        nb.tree_accel(q, 0.01, 0.6, 4, prec=nb.F32_F64ACC, out=out_g, cells=c)
    for rep in range(3):
        out_g.zero_()
        graph.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()
        ref = nb.tree_accel(q, 0.01, 0.6, 4, prec=nb.F32_F64ACC, cells=c)
        torch.cuda.synchronize()
        assert torch.equal(out_g, ref) and torch.equal(ref, out_e), rep
        del junk
