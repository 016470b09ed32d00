"""The hand-written adjoint on the solid-mask path (arbitrary voxel masks:
bounce-back links from each node's neighbour word, the wall averages of
Eqs. (36)-(37) and the window of Eq. (38) at every solid node with a fluid
neighbour) against the oracle's reverse mode (torch autograd through the
FP64 CPU oracle step with the same mask), and end to end against the
oracle and central finite differences of the GPU forward."""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import DT, make_sim, oracle_params, rel_err, say
from oracle import eos, lbm
from paper_2504_03819_amd import autograd as lag
from paper_2504_03819_amd import inputs

pytestmark = pytest.mark.gpu

OM = [1.0, 1.0, 1.0, 0.5] + [1.0] * 7  # omega_3 = 1/2 next to solids at 0.7 T_c


def _mask(kind, shape):
    if kind == "obstacles":
        return inputs.mask_obstacles(shape)
    if kind == "pillars":
        return inputs.mask_pillars(shape, plate=2, pitch=8, width=3, height=4)
    return inputs.mask_planes(shape)


def _rho(shape, T, mask, seed=0, noise=1e-3):
    rl, rv = eos.maxwell(eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"], T)
    nz, ny, nx = shape
    rho = inputs.sphere(shape, (0.5 * nx, 0.5 * ny, 0.4 * nz), min(shape) / 3.0, rl, rv)
    rho = rho + inputs.uniform_noise(shape, noise, seed)
    rho[mask.astype(bool)] = rv
    return rho


def _oracle_vjp(f, lam, p):
    kappa = torch.tensor(p.kappa, dtype=DT, requires_grad=True)
    wet = torch.tensor(p.wet_value, dtype=DT, requires_grad=True)
    nu = torch.tensor(p.nu, dtype=DT, requires_grad=True)
    pt = dataclasses.replace(p, kappa=kappa, wet_value=wet, nu=nu)
    fr = f.clone().requires_grad_(True)
    (lbm.step(fr, pt) * lam).sum().backward()
    gw = float(wet.grad) if wet.grad is not None else 0.0
    return fr.grad, float(kappa.grad), gw, float(nu.grad)


CASES = [
    ("obstacles neutral", "obstacles", (10, 9, 12), dict(wet_mode=0)),
    ("obstacles phi 1.4", "obstacles", (10, 9, 12), dict(wet_mode=1, wet_value=1.4)),
    ("obstacles drho 0.9", "obstacles", (10, 9, 12), dict(wet_mode=2, wet_value=0.9)),
    ("pillars phi 1.3 ragged", "pillars", (14, 19, 21), dict(wet_mode=1, wet_value=1.3)),
    ("planes drho 1.2", "planes", (9, 8, 11), dict(wet_mode=2, wet_value=1.2)),
    ("obstacles 70 wide, several tiles", "obstacles", (8, 6, 70), dict(wet_mode=1, wet_value=1.6)),
    ("pillars drho 0.9, three z-chunks", "pillars", (36, 9, 11), dict(wet_mode=2, wet_value=0.9)),
]


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("label,kind,shape,extra", CASES, ids=[c[0] for c in CASES])
def test_mask_adjoint_step_matches_oracle_reverse_mode(label, kind, shape, extra, form):
    say(f"mask adjoint {label} {form}")
    T = eos.temperature(0.7)
    nz, ny, nx = shape
    mask = _mask(kind, shape)
    sim = make_sim(nx=nx, ny=ny, nz=nz, T=T, omega=OM, solid=mask, adjoint=1, precision=form, **extra)
    p = oracle_params(sim)
    g = np.random.Generator(np.random.PCG64(31))
    u0 = 0.03 * g.uniform(-1, 1, (3,) + shape)
    f0 = lbm.init(torch.tensor(_rho(shape, T, mask)), p, torch.tensor(u0))
    f = f0 + torch.tensor(inputs.uniform_noise(tuple(f0.shape), 2e-4, 3)) * (f0 != 0)
    solid = torch.tensor(mask.astype(bool))
    lam = torch.tensor(g.uniform(-1, 1, (27,) + shape)) * (~solid)
    sim.set_populations(f)
    state = sim.get_state().clone()
    sim.adjoint_seed_populations(lam)
    sim.adjoint_step(state)
    lg = sim.adjoint_state().cpu()
    gg = sim.adjoint_grads()
    lo, ko, wo, no = _oracle_vjp(f, lam, p)
    fl = (~solid).expand(27, *shape)
    e = rel_err(lg[fl], lo[fl])
    assert float(lg[~fl].abs().max()) == 0.0  # solid nodes hold no lambda
    ek = abs(gg["kappa"] - ko) / max(abs(ko), 1e-300)
    en = abs(gg["nu"] - no) / max(abs(no), 1e-300)
    ew = abs(gg["wet_value"] - wo) / max(abs(wo), 1e-12) if p.wet_mode else abs(gg["wet_value"] - wo)
    say(f"{label} {form}: lambda err={e:.2e} dkappa {ek:.1e} dnu {en:.1e} dwet={gg['wet_value']:.6e}/{wo:.6e} "
        f"({ew:.1e})")
    # FP32: the adjoint and the stored state in FP32 against the FP64 oracle;
    # dL/dnu sums per-node terms of both signs (1e-4 level in FP32)
    tol = 1e-11 if form == "fp64" else 2e-5
    assert e < tol
    assert ek < (1e-9 if form == "fp64" else 1e-4) and en < (1e-9 if form == "fp64" else 1e-3)
    assert ew < (1e-9 if form == "fp64" else 1e-4)


def test_mask_end_to_end_gradients_vs_oracle_and_fd():
    """12 steps on a pillared substrate with phi wetting: dL/drho0, dL/dkappa,
    dL/d(phi) of L = sum over fluid nodes (rho_T - target)^2 through the
    autograd Function, against oracle autograd and central differences."""
    shape = (12, 10, 11)
    nz, ny, nx = shape
    T = eos.temperature(0.7)
    mask = _mask("pillars", shape)
    solid = torch.tensor(mask.astype(bool))
    rho0 = _rho(shape, T, mask, seed=9, noise=1e-2)
    rl, rv = eos.maxwell(eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"], T)
    tgt = torch.tensor(rho0 + 1e-3 * (rl - rv) * inputs.uniform_noise(shape, 1.0, 12))
    steps, phi, kappa = 12, 1.3, 0.02
    cfg = lag.StepConfig(nx=nx, ny=ny, nz=nz, steps=steps, checkpoint_every=4, T=T, wet_mode=1, omega=OM,
                         solid=mask)
    r0 = torch.tensor(rho0, device="cuda", requires_grad=True)
    kap = torch.tensor(kappa, dtype=DT, requires_grad=True)
    wet = torch.tensor(phi, dtype=DT, requires_grad=True)
    rT = lag.simulate(r0, kap, wet, cfg)
    fluid_d = (~solid).to("cuda")
    loss = (((rT - tgt.to("cuda")) ** 2) * fluid_d).sum()
    loss.backward()
    g_r0 = r0.grad.cpu()
    p = lbm.Params(nx, ny, nz, T=T, wet_mode=1, omega=OM, solid=solid)
    pr = p.coexistence()
    ko = torch.tensor(kappa, dtype=DT, requires_grad=True)
    wo = torch.tensor(phi, dtype=DT, requires_grad=True)
    ro = torch.tensor(rho0, requires_grad=True)
    po = dataclasses.replace(p, kappa=ko, wet_value=wo, rho_l=pr[0], rho_v=pr[1])
    fT = lbm.run(lbm.init(ro, po), po, steps)
    lo = (((lbm.aux_fields(fT, po)["rho"] - tgt) ** 2) * (~solid)).sum()
    lo.backward()
    fl = ~solid
    e_r0 = rel_err(g_r0[fl], ro.grad[fl])
    e_k = abs(float(kap.grad) - float(ko.grad)) / abs(float(ko.grad))
    e_w = abs(float(wet.grad) - float(wo.grad)) / max(abs(float(wo.grad)), 1e-12)
    say(f"mask end-to-end: dL/drho0 {e_r0:.2e} dL/dkappa {float(kap.grad):.8e}/{float(ko.grad):.8e} ({e_k:.1e}) "
        f"dL/dphi {float(wet.grad):.8e}/{float(wo.grad):.8e} ({e_w:.1e})")
    assert abs(float(loss.detach()) - float(lo)) < 1e-10 * float(lo)
    assert e_r0 < 1e-9 and e_k < 1e-9 and e_w < 1e-9

    def gpu_loss(r, k, w):
        sim = cfg.make(k, w)
        sim.init_density(torch.tensor(r))
        sim.step(steps)
        out = float((((sim.fields()["rho"].cpu() - tgt) ** 2) * fl).sum())
        sim.close()
        return out

    h = 1e-6
    fd_k = (gpu_loss(rho0, kappa + h, phi) - gpu_loss(rho0, kappa - h, phi)) / (2 * h)
    say(f"  FD dL/dkappa={fd_k:.8e}")
    assert abs(fd_k - float(kap.grad)) < 1e-5 * abs(fd_k)
    g = np.random.Generator(np.random.PCG64(4))
    fluid_idx = np.argwhere(~mask.astype(bool))
    for nd in (tuple(int(v) for v in fluid_idx[int(g.integers(0, len(fluid_idx)))]) for _ in range(3)):
        rp, rm = rho0.copy(), rho0.copy()
        rp[nd] += 1e-6
        rm[nd] -= 1e-6
        fd = (gpu_loss(rp, kappa, phi) - gpu_loss(rm, kappa, phi)) / 2e-6
        say(f"  FD dL/drho0{nd}={fd:.8e} adjoint={float(g_r0[nd]):.8e}")
        assert abs(fd - float(g_r0[nd])) < 1e-5 * max(abs(fd), 1e-6)
