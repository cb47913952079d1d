"""Bit-reversible fixed-point kick-drift-kick on the device and its
checkpoint-free adjoint: the reverse pass must rebuild the initial integer
state exactly (which needs the fused VJP's force to equal the force kernel's
bit for bit), the forward must track the ordinary leapfrog, and the gradient
must match the oracle's reverse mode at the FP32 bar of the other adjoint
tests."""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, normwise, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu


def _inputs(torch, n, seed):
    pm, v = ics.plummer(n, seed)
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    vv = to_dev(torch, np.c_[v[:, :3], np.zeros(n)].astype(np.float32), torch.float32)
    return pm, v, p, vv


@pytest.mark.parametrize("n,steps", [(300, 25), (3000, 30), (4099, 7)])
def test_exact_reversal(n, steps):
    """Forward nsteps, then the adjoint rewinds the state: the integers come
    back bit for bit (n = 300 runs the unsplit kernel shape, the larger ones
    split the sources)."""
    torch, nb = gpu()
    _, _, p, vv = _inputs(torch, n, 600 + n)
    st0, _, _ = nb.janus_forward(p, vv, 0.01, 1e-3, 0)
    st, pT, vT = nb.janus_forward(p, vv, 0.01, 1e-3, steps)
    assert not torch.equal(st, st0)
    xb = torch.randn_like(p); xb[:, 3] = 0
    vb = torch.randn_like(p); vb[:, 3] = 0
    nb.janus_adjoint(st, p, 0.01, 1e-3, steps, xb, vb)
    torch.cuda.synchronize()
    assert torch.equal(st, st0)


def test_forward_tracks_leapfrog(orc):
    """Against the FP64 leapfrog from the same FP32 start: positions at the
    FP32 bar, and velocity changes no worse than the FP32-state leapfrog's
    (whose velocities carry an FP32 rounding per half kick; the integer
    velocity quantum here is 2^-40)."""
    torch, nb = gpu()
    n, steps = 2048, 40
    pm, v, p, vv = _inputs(torch, n, 610)
    _, pT, vT = nb.janus_forward(p, vv, 0.01, 1e-3, steps)
    q, u, a = p.clone(), vv.clone(), torch.empty_like(p)
    nb.leapfrog_kdk(q, u, a, 0.01, 1e-3, steps, prec=nb.F32_F64ACC)
    v0 = widen32(np.c_[v[:, :3], np.zeros(n)])
    ref = orc.leapfrog(widen32(pm), v0, 0.01, 1e-3, steps)
    dv_ref = ref["v"] - v0[:, :3]
    ej = (rms_rel(host(pT)[:, :3], ref["x"]), rms_rel(host(vT)[:, :3] - v0[:, :3], dv_ref))
    eo = (rms_rel(host(q)[:, :3], ref["x"]), rms_rel(host(u)[:, :3] - v0[:, :3], dv_ref))
    print("janus vs fp64 leapfrog", ej, "fp32-state leapfrog", eo)
    assert ej[0] < 1e-6
    assert ej[1] < 1e-4 and ej[1] <= 1.5 * eo[1]
    assert torch.equal(pT[:, 3], p[:, 3])


def test_gradient_matches_oracle_and_reversal_scheme(orc):
    """L = sum |x_T - y|^2: the checkpoint-free adjoint against the oracle's
    FP64 reverse mode (measured 3.4e-6, bar 1e-5) and against the checkpointed reversal
    scheme of the ordinary leapfrog."""
    torch, nb = gpu()
    n, eps, dt, steps = 1024, 0.01, 1e-3, 40
    pm, v, p, vv = _inputs(torch, n, 620)
    y = ics.perturbed_snapshot(pm, 621)
    st, pT, vT = nb.janus_forward(p, vv, eps, dt, steps)
    yd = to_dev(torch, y.astype(np.float32), torch.float32)
    xb = torch.zeros_like(p); xb[:, :3] = 2 * (pT[:, :3] - yd)
    vb = torch.zeros_like(p)
    pc, vc, mc = nb.janus_adjoint(st, p, eps, dt, steps, xb, vb)
    torch.cuda.synchronize()
    L, gx, gv, gm = orc.traj_grad(widen32(pm), widen32(np.c_[v[:, :3], np.zeros(n)]), y, eps, dt, steps)
    e = (normwise(host(pc)[:, :3], gx), normwise(host(vc)[:, :3], gv), normwise(host(mc), gm))
    ck = nb.trajectory_forward(p.clone(), vv.clone(), eps, dt, steps, 20, prec=nb.F32_F64ACC)
    xb2 = torch.zeros_like(p); xb2[:, :3] = 2 * (ck[-1, 0][:, :3] - yd)
    pc2, vc2, mc2 = nb.trajectory_adjoint(ck, eps, dt, steps, 20, xb2, vb, prec=nb.F32_F64ACC)
    e2 = (normwise(host(pc2)[:, :3], gx), normwise(host(vc2)[:, :3], gv), normwise(host(mc2), gm))
    print("janus adjoint grad errors", e, "checkpointed reversal scheme", e2)
    # the integer state carries no FP32 rounding of x and v, so this gradient
    # is closer to the FP64 one than the FP32-state adjoint's
    assert max(e) <= 1e-5
    assert e[0] <= e2[0] and e[2] <= e2[2]


def test_nonpositive_mass_is_refused():
    torch, nb = gpu()
    _, _, p, vv = _inputs(torch, 500, 630)
    p[7, 3] = 0.0
    st, _, _ = nb.janus_forward(p, vv, 0.01, 1e-3, 3)
    z = torch.zeros_like(p)
    with pytest.raises(nb.NBodyError, match="positive"):
        nb.janus_adjoint(st, p, 0.01, 1e-3, 3, z, z)


def test_autograd_function_matches_oracle(orc):
    """ReversibleTrajectory through torch autograd: L = sum |x_T - y|^2,
    gradients in (x0, v0, m) against the oracle's FP64 reverse mode (bar 1e-5,
    as for the adjoint call itself)."""
    torch, nb = gpu()
    n, eps, dt, steps = 1024, 0.01, 1e-3, 40
    pm, v, p, vv = _inputs(torch, n, 640)
    y = ics.perturbed_snapshot(pm, 641)
    x0 = p[:, :3].clone().requires_grad_(True)
    v0 = vv[:, :3].clone().requires_grad_(True)
    m = p[:, 3].clone().requires_grad_(True)
    xT, vT = nb.ReversibleTrajectory.apply(x0, v0, m, eps, dt, steps)
    yd = to_dev(torch, y[:, :3].astype(np.float32), torch.float32)
    loss = ((xT - yd) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    L, gx, gv, gm = orc.traj_grad(widen32(pm), widen32(np.c_[v[:, :3], np.zeros(n)]), y, eps, dt, steps)
    e = (normwise(host(x0.grad), gx), normwise(host(v0.grad), gv), normwise(host(m.grad), gm))
    print("reversible autograd grad errors", e)
    assert max(e) <= 1e-5
    # a second backward through a fresh forward gives the same gradient
    x1 = p[:, :3].clone().requires_grad_(True)
    xT1, _ = nb.ReversibleTrajectory.apply(x1, vv[:, :3].clone(), m.detach(), eps, dt, steps)
    ((xT1 - yd) ** 2).sum().backward()
    assert torch.equal(x1.grad, x0.grad)


def test_exact_reversal_at_full_size():
    """N = 2^20 colliding pair (the headline workload), 2 steps: the reverse
    pass restores the initial integer state bit for bit at the full size and
    kernel shape, and the decoded final positions agree with the ordinary
    leapfrog's to FP32 rounding."""
    torch, nb = gpu()
    w = ics.WORKLOADS["collide1m"]
    pm, v = ics.colliding_pair(w["n"], w["seed"])
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    vv = to_dev(torch, np.c_[v[:, :3], np.zeros(len(v))].astype(np.float32), torch.float32)
    print(f"fixed-point reversal N={p.shape[0]}", flush=True)
    st0, _, _ = nb.janus_forward(p, vv, w["eps"], w["dt"], 0)
    st, pT, _ = nb.janus_forward(p, vv, w["eps"], w["dt"], 2)
    xb = torch.zeros_like(p)
    nb.janus_adjoint(st, p, w["eps"], w["dt"], 2, xb, torch.zeros_like(p))
    torch.cuda.synchronize()
    assert torch.equal(st, st0)
    q, u, a = p.clone(), vv.clone(), torch.empty_like(p)
    nb.leapfrog_kdk(q, u, a, w["eps"], w["dt"], 2, prec=nb.F32_F64ACC)
    assert rms_rel(host(pT)[:, :3], host(q)[:, :3]) < 1e-7


def test_reversal_survives_a_tuning_change_between_calls():
    """Pinning another kernel shape for the VJP between the forward and the
    adjoint does not change the fixed-point path's forces: the state still
    comes back bit for bit."""
    torch, nb = gpu()
    _, _, p, vv = _inputs(torch, 3000, 650)
    st0, _, _ = nb.janus_forward(p, vv, 0.01, 1e-3, 0)
    st, _, _ = nb.janus_forward(p, vv, 0.01, 1e-3, 10)
    try:
        nb.set_tuning(nb.KERNEL_VJP, nb.F32_F64ACC, 1, 4, 1024, 0)
        z = torch.zeros_like(p)
        nb.janus_adjoint(st, p, 0.01, 1e-3, 10, z, z)
        torch.cuda.synchronize()
    finally:
        nb.set_tuning(nb.KERNEL_VJP, nb.F32_F64ACC)
    assert torch.equal(st, st0)


@pytest.mark.parametrize("n,steps,G,sx,sv", [(1, 5, 1.0, 40, 40), (2, 7, 1.0, 40, 40), (500, 0, 1.0, 40, 40),
                                             (700, 9, 2.5, 40, 40), (600, 6, 1.0, 50, 34)])
def test_reversal_edge_cases(n, steps, G, sx, sv):
    """One and two bodies, zero steps (the adjoint passes the cotangents
    through), G != 1 (G sits in the kick and the cotangent scale) and other
    fixed-point shifts: the state comes back bit for bit."""
    torch, nb = gpu()
    pm, v = ics.plummer(max(n, 2), 660 + n)
    pm, v = pm[:n].copy(), v[:n].copy()
    pm[:, 3] = 1.0 / n
    p = to_dev(torch, np.asarray(pm, dtype=np.float32), torch.float32)
    vv = to_dev(torch, np.c_[v[:, :3], np.zeros(n)].astype(np.float32), torch.float32)
    st0, _, _ = nb.janus_forward(p, vv, 0.01, 1e-3, 0, sx, sv, G)
    st, pT, vT = nb.janus_forward(p, vv, 0.01, 1e-3, steps, sx, sv, G)
    xb = torch.randn_like(p); xb[:, 3] = 0
    vb = torch.randn_like(p); vb[:, 3] = 0
    pc, vc, mc = nb.janus_adjoint(st, p, 0.01, 1e-3, steps, xb, vb, sx, sv, G)
    torch.cuda.synchronize()
    assert torch.equal(st, st0)
    if steps == 0:
        assert torch.equal(pc[:, :3], xb[:, :3]) and torch.equal(vc[:, :3], vb[:, :3])
        assert torch.all(mc == 0)
    if n == 1:
        # a lone body moves in a straight line and feels nothing
        np.testing.assert_allclose(host(pT)[0, :3], pm[0, :3] + steps * 1e-3 * v[0, :3], rtol=0, atol=1e-6)
        assert torch.equal(pc[:, :3], xb[:, :3])
