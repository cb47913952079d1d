"""Parity of the fused force + VJP kernel (nbody_accel_vjp) and of the
checkpointed trajectory adjoint with the FP64 oracle (reverse-mode
derivative of the paper's force law and of the leapfrog around it)."""
import numpy as np
import pytest

import ics
from nbtest import gpu, host, normwise, rms_rel, to_dev, widen32

pytestmark = pytest.mark.gpu


def _cot(n, seed, phi):
    g = ics.rng(seed)
    c = np.zeros((n, 4))
    c[:, :3] = g.standard_normal((n, 3))
    if phi:
        c[:, 3] = g.standard_normal(n)
    return c


@pytest.mark.parametrize("n", [1, 2, 65, 300, 1029])
@pytest.mark.parametrize("phi", [False, True])
def test_vjp_f64(orc, n, phi):
    torch, nb = gpu()
    pm, _ = ics.plummer(max(n, 2), 60 + n)
    pm = pm[:n].copy()
    pm[:, 3] *= np.linspace(0.5, 1.5, n)
    cot = _cot(n, 61, phi)
    pc, mc, ap = nb.accel_vjp(to_dev(torch, pm, torch.float64), to_dev(torch, cot, torch.float64), 0.03)
    torch.cuda.synchronize()
    xb, mb = orc.vjp(pm, 0.03, cot[:, :3], cot[:, 3] if phi else None)
    if n == 1:
        assert np.all(host(pc) == 0) and np.all(host(mc) == 0)
        return
    assert normwise(host(pc)[:, :3], xb) <= 1e-12
    assert normwise(host(mc), mb) <= 1e-12
    assert np.all(host(pc)[:, 3] == 0)
    acc, pot = orc.accel(pm, 0.03)
    assert rms_rel(host(ap)[:, :3], acc) <= 1e-12 and rms_rel(host(ap)[:, 3], pot) <= 1e-12


@pytest.mark.parametrize("mode", ["F32_KAHAN", "F32_F64ACC", "F32"])
def test_vjp_f32(orc, mode):
    torch, nb = gpu()
    n = 4000
    pm, _ = ics.plummer(n, 62)
    cot = _cot(n, 63, True)
    pm32, cot32 = widen32(pm), widen32(cot)
    pc, mc, ap = nb.accel_vjp(to_dev(torch, pm32, torch.float32), to_dev(torch, cot32, torch.float32), 0.01,
                              prec=getattr(nb, mode))
    torch.cuda.synchronize()
    xb, mb = orc.vjp(pm32, 0.01, cot32[:, :3], cot32[:, 3])
    assert normwise(host(pc)[:, :3], xb) <= 1e-5
    assert normwise(host(mc), mb) <= 1e-5


def test_vjp_invariants_on_gpu():
    """Translation invariance (sum xbar = 0) and mass homogeneity
    (sum m mbar = sum abar . a + phibar phi) of the GPU result."""
    torch, nb = gpu()
    n = 2000
    pm, _ = ics.plummer(n, 64)
    cot = _cot(n, 65, True)
    pc, mc, ap = nb.accel_vjp(to_dev(torch, pm, torch.float64), to_dev(torch, cot, torch.float64), 0.02)
    torch.cuda.synchronize()
    pc, mc, ap = host(pc), host(mc), host(ap)
    assert np.abs(pc[:, :3].sum(axis=0)).max() <= 1e-11 * np.abs(pc).sum()
    lhs = (pm[:, 3] * mc).sum()
    rhs = (cot[:, :3] * ap[:, :3]).sum() + (cot[:, 3] * ap[:, 3]).sum()
    assert abs(lhs - rhs) <= 1e-11 * np.abs(pm[:, 3] * mc).sum()


@pytest.mark.parametrize("scheme", ["ADJ_RECOMPUTE", "ADJ_REVERSE"])
def test_trajectory_gradient_f64(orc, scheme):
    torch, nb = gpu()
    n, eps, dt, steps, C = 64, 0.05, 2e-3, 40, 10
    pm, v = ics.plummer(n, 66)
    pm[:, 3] *= np.linspace(0.5, 1.5, n)
    y = ics.perturbed_snapshot(pm, 67, 0.05)
    L, gx, gv, gm = orc.traj_grad(pm, v, y, eps, dt, steps)
    p, vv = to_dev(torch, pm, torch.float64), to_dev(torch, v, torch.float64)
    ck = nb.trajectory_forward(p, vv, eps, dt, steps, C)
    xb = torch.zeros_like(p)
    xb[:, :3] = 2 * (p[:, :3] - to_dev(torch, y, torch.float64))
    vb = torch.zeros_like(p)
    pc, vc, mc = nb.trajectory_adjoint(ck, eps, dt, steps, C, xb, vb, scheme=getattr(nb, scheme))
    torch.cuda.synchronize()
    assert abs(float(((host(p)[:, :3] - y) ** 2).sum()) - L) <= 1e-12 * L
    assert normwise(host(pc)[:, :3], gx) <= 1e-11
    assert normwise(host(vc)[:, :3], gv) <= 1e-11
    assert normwise(host(mc), gm) <= 1e-11


@pytest.mark.parametrize("scheme", ["ADJ_RECOMPUTE", "ADJ_REVERSE"])
def test_trajectory_gradient_f32_and_autograd(orc, scheme):
    torch, nb = gpu()
    n, eps, dt, steps, C = 1024, 0.01, 1e-3, 40, 20
    pm, v = ics.plummer(n, 68)
    y = ics.perturbed_snapshot(pm, 69)
    pm32, v32 = widen32(pm), widen32(v)
    L, gx, gv, gm = orc.traj_grad(pm32, v32, y, eps, dt, steps)
    x0 = to_dev(torch, pm32[:, :3], torch.float32).requires_grad_(True)
    v0 = to_dev(torch, v32[:, :3], torch.float32).requires_grad_(True)
    m = to_dev(torch, pm32[:, 3], torch.float32).requires_grad_(True)
    xT, vT = nb.NBodyTrajectory.apply(x0, v0, m, eps, dt, steps, C, 1.0, None, getattr(nb, scheme))
    loss = ((xT - to_dev(torch, y, torch.float32)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    print(scheme, "f32 grad errors", normwise(host(x0.grad), gx), normwise(host(v0.grad), gv), normwise(host(m.grad), gm))
    assert normwise(host(x0.grad), gx) <= 1e-4
    assert normwise(host(v0.grad), gv) <= 1e-4
    assert normwise(host(m.grad), gm) <= 1e-4


def test_trajectory_gradient_velocity_cotangent_and_zero_steps(orc):
    """A cotangent on the final velocity flows through the kicks; with zero
    steps the adjoint is the identity."""
    torch, nb = gpu()
    n, eps, dt, steps, C = 40, 0.05, 2e-3, 20, 5
    pm, v = ics.plummer(n, 70)
    p, vv = to_dev(torch, pm, torch.float64), to_dev(torch, v, torch.float64)
    ck = nb.trajectory_forward(p, vv, eps, dt, 0, C)
    g = ics.rng(71)
    xb = torch.zeros_like(p); xb[:, :3] = to_dev(torch, g.standard_normal((n, 3)), torch.float64)
    vb = torch.zeros_like(p); vb[:, :3] = to_dev(torch, g.standard_normal((n, 3)), torch.float64)
    pc, vc, mc = nb.trajectory_adjoint(ck, eps, dt, 0, C, xb, vb)
    torch.cuda.synchronize()
    assert torch.equal(pc, xb) and torch.equal(vc, vb) and torch.all(mc == 0)
    # FD of s(x0, v0) = <vb, v_T> through the oracle leapfrog
    p, vv = to_dev(torch, pm, torch.float64), to_dev(torch, v, torch.float64)
    ck = nb.trajectory_forward(p, vv, eps, dt, steps, C)
    for scheme in (nb.ADJ_RECOMPUTE, nb.ADJ_REVERSE):
        pc, vc, mc = nb.trajectory_adjoint(ck, eps, dt, steps, C, torch.zeros_like(p), vb, scheme=scheme)
        torch.cuda.synchronize()
        vbn = host(vb)[:, :3]
        d = np.zeros((n, 4)); d[:, :3] = g.standard_normal((n, 3))
        hh = 1e-6
        fp = (orc.leapfrog(pm + hh * d, v, eps, dt, steps)["v"] * vbn).sum()
        fm = (orc.leapfrog(pm - hh * d, v, eps, dt, steps)["v"] * vbn).sum()
        fd = (fp - fm) / (2 * hh)
        an = (host(pc)[:, :3] * d[:, :3]).sum()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9


@pytest.mark.parametrize("scheme", ["ADJ_RECOMPUTE", "ADJ_REVERSE"])
def test_trajectory_gradient_with_massless_body(orc, scheme):
    """A zero mass switches the adjoint to the general VJP form."""
    torch, nb = gpu()
    n, eps, dt, steps, C = 48, 0.05, 2e-3, 20, 10
    pm, v = ics.plummer(n, 72)
    pm[5, 3] = 0.0
    y = ics.perturbed_snapshot(pm, 73, 0.05)
    L, gx, gv, gm = orc.traj_grad(pm, v, y, eps, dt, steps)
    p, vv = to_dev(torch, pm, torch.float64), to_dev(torch, v, torch.float64)
    ck = nb.trajectory_forward(p, vv, eps, dt, steps, C)
    xb = torch.zeros_like(p)
    xb[:, :3] = 2 * (p[:, :3] - to_dev(torch, y, torch.float64))
    pc, vc, mc = nb.trajectory_adjoint(ck, eps, dt, steps, C, xb, torch.zeros_like(p), scheme=getattr(nb, scheme))
    torch.cuda.synchronize()
    assert normwise(host(pc)[:, :3], gx) <= 1e-11
    assert normwise(host(vc)[:, :3], gv) <= 1e-11
    assert normwise(host(mc), gm) <= 1e-11


@pytest.mark.parametrize("scheme", ["ADJ_RECOMPUTE", "ADJ_REVERSE"])
def test_energy_gradient_potential_path_f64(orc, scheme):
    """Cotangents of the final total energy: vbar_T = m v_T and phibar_T = m/2
    on the final potential (the adjoint's potential path) against the
    oracle's reverse mode with the same cotangents."""
    torch, nb = gpu()
    n, eps, dt, steps, C = 64, 0.05, 2e-3, 40, 10
    pm, v = ics.plummer(n, 70)
    pm[:, 3] *= np.linspace(0.5, 1.5, n)
    r = orc.leapfrog(pm, v, eps, dt, steps)
    m = pm[:, 3]
    gx, gv, gm = orc.traj_grad_cot(pm, v, eps, dt, steps, np.zeros((n, 3)), m[:, None] * r["v"], 0.5 * m)
    p, vv = to_dev(torch, pm, torch.float64), to_dev(torch, v, torch.float64)
    ck = nb.trajectory_forward(p, vv, eps, dt, steps, C)
    xb = torch.zeros_like(p)
    vb = torch.zeros_like(p)
    vb[:, :3] = vv[:, :3] * p[:, 3:4]
    pc, vc, mc = nb.trajectory_adjoint(ck, eps, dt, steps, C, xb, vb, scheme=getattr(nb, scheme),
                                       phibar_T=0.5 * p[:, 3])
    torch.cuda.synchronize()
    assert normwise(host(pc)[:, :3], gx) <= 1e-11
    assert normwise(host(vc)[:, :3], gv) <= 1e-11
    assert normwise(host(mc), gm) <= 1e-11


def test_energy_loss_autograd_f32(orc):
    """d E(T) / d(x0, v0, m) through NBodyTrajectory(with_potential=True),
    with the energy written in torch (autograd supplies the explicit mass
    terms), against the oracle."""
    torch, nb = gpu()
    n, eps, dt, steps, C = 1024, 0.01, 1e-3, 40, 20
    pm, v = ics.plummer(n, 71)
    pm32, v32 = widen32(pm), widen32(v)
    r = orc.leapfrog(pm32, v32, eps, dt, steps)
    m = pm32[:, 3]
    gx, gv, gm = orc.traj_grad_cot(pm32, v32, eps, dt, steps, np.zeros((n, 3)), m[:, None] * r["v"], 0.5 * m)
    gm = gm + 0.5 * (r["v"] ** 2).sum(1) + 0.5 * r["pot"]
    x0 = to_dev(torch, pm32[:, :3], torch.float32).requires_grad_(True)
    v0 = to_dev(torch, v32[:, :3], torch.float32).requires_grad_(True)
    mm = to_dev(torch, m, torch.float32).requires_grad_(True)
    xT, vT, phiT = nb.NBodyTrajectory.apply(x0, v0, mm, eps, dt, steps, C, 1.0, None, nb.ADJ_REVERSE, True)
    E = 0.5 * (mm * (vT ** 2).sum(1)).sum() + 0.5 * (mm * phiT).sum()
    E.backward()
    torch.cuda.synchronize()
    e_ref = 0.5 * float((m * (r["v"] ** 2).sum(1)).sum()) + 0.5 * float((m * r["pot"]).sum())
    assert abs(float(E.detach()) / e_ref - 1.0) < 1e-5
    print("energy grad errors", normwise(host(x0.grad), gx), normwise(host(v0.grad), gv), normwise(host(mm.grad), gm))
    assert normwise(host(x0.grad), gx) <= 1e-4
    assert normwise(host(v0.grad), gv) <= 1e-4
    assert normwise(host(mm.grad), gm) <= 1e-4
