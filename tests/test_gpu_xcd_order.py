"""The XCD-contiguous tile order (on by default from 2^26 nodes) only changes
which workgroup runs which tile: forced on and off at small sizes it must
give the same states, fields, adjoint state and gradients bit for bit, on
the two-read step, the fused step, the solid-mask path and the adjoint."""
import numpy as np
import pytest
import torch

from gpu_util import droplet_rho, make_sim, say
from oracle import eos
from paper_2504_03819_amd import inputs, lbfe

pytestmark = pytest.mark.gpu

OM = [1.0, 1.0, 1.0, 0.5] + [1.0] * 7


def _sim(remap, sched=None, **kw):
    order = lbfe.ORDER_XCD if remap == "1" else lbfe.ORDER_ROUND_ROBIN
    return make_sim(tile_order=order, **(sched or {}), **kw)


def _raw(t):
    return t.detach().contiguous().view(torch.uint8).cpu()


CASES = [
    # (label, shape (nz, ny, nx), walls, extra, schedule)
    ("periodic fp32 ragged", (40, 37, 70), False, dict(precision="fp32"), {"step_path": 1}),
    ("walls fp64 fused", (21, 26, 40), True, dict(precision="fp64", wet_mode=1, wet_value=1.3, omega=OM),
     {"step_path": 2}),
    ("periodic fp32 ragged fused", (40, 37, 70), False, dict(precision="fp32"), {"step_path": 2}),
    ("mask fp16dev", (14, 20, 23), False, dict(precision="fp16dev", wet_mode=2, wet_value=0.9, omega=OM, mask=True),
     {}),
]


@pytest.mark.parametrize("label,shape,walls,extra,sched", CASES, ids=[c[0] for c in CASES])
def test_tile_order_changes_nothing(label, shape, walls, extra, sched):
    say(f"XCD tile order: {label}")
    T = eos.temperature(0.7 if walls or extra.get("mask") else 0.85)
    nz, ny, nx = shape
    kw = dict(nx=nx, ny=ny, nz=nz, T=T, walls_z=int(walls), **extra)
    if kw.pop("mask", False):
        kw["solid"] = inputs.mask_obstacles(shape)
    sims = [_sim("0", sched, **kw), _sim("1", sched, **kw)]
    rho0 = droplet_rho(shape, T, walls=walls, radius=min(ny, nx) / 3.0)
    g = np.random.Generator(np.random.PCG64(3))
    u0 = torch.tensor(0.02 * g.uniform(-1, 1, (3,) + shape))
    for s in sims:
        s.init_density(torch.tensor(rho0), u0)
    for n in (1, 2, 5):
        for s in sims:
            s.step(n)
        assert torch.equal(_raw(sims[0].get_state()), _raw(sims[1].get_state())), label
        fa, fb = (s.fields() for s in sims)
        for name in ("rho", "u", "mu", "F"):
            assert torch.equal(fa[name].cpu(), fb[name].cpu()), f"{label}: {name}"
    assert sims[0].reduce() == sims[1].reduce()


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_tile_order_changes_nothing_in_the_adjoint(form):
    shape = (12, 19, 21)
    say(f"XCD tile order, adjoint: {form}")
    T = eos.temperature(0.7)
    kw = dict(nx=21, ny=19, nz=12, T=T, walls_z=1, wet_mode=1, wet_value=1.3, precision=form, adjoint=1, omega=OM)
    sims = [_sim("0", **kw), _sim("1", **kw)]
    rho0 = droplet_rho(shape, T, walls=True, radius=5.0, noise=1e-2, seed=4)
    for s in sims:
        s.init_density(torch.tensor(rho0))
    states = []
    for _ in range(4):
        states.append(sims[0].get_state())
        for s in sims:
            s.step(1)
    seed = torch.tensor(inputs.uniform_noise(shape, 1.0, 13), device="cuda")
    for s in sims:
        s.adjoint_seed(seed)
    for t in range(3, -1, -1):
        for s in sims:
            s.adjoint_step(states[t])
    assert torch.equal(sims[0].adjoint_state().cpu(), sims[1].adjoint_state().cpu())
    assert sims[0].adjoint_grads() == sims[1].adjoint_grads()
    ga, gb = (s.adjoint_init_density().cpu() for s in sims)
    assert torch.equal(ga, gb)
