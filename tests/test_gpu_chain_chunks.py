"""The stencil chain marches each workgroup through a chunk of z-planes, the
chunk length being chosen per grid.  Every node's arithmetic is the same
whatever the chunk, so forcing other lengths (1, 3, 8, 32, 64 planes, ragged
last chunks included) must leave the states and fields unchanged bit for
bit, with walls (whose chemical potential a chunk takes from its first or
last fluid plane) and on the fused path."""
import numpy as np
import pytest
import torch

from gpu_util import droplet_rho, make_sim, say
from oracle import eos

pytestmark = pytest.mark.gpu

OM = [1.0, 1.0, 1.0, 0.5] + [1.0] * 7
CASES = [
    # (label, shape (nz, ny, nx), walls, extra, schedule)
    ("periodic fp64 ragged", (40, 37, 70), False, dict(precision="fp64"), {"step_path": 1}),
    ("walls phi fp32", (34, 21, 45), True, dict(precision="fp32", wet_mode=1, wet_value=1.4, omega=OM),
     {"step_path": 1}),
    ("walls drho fp64 3-plane", (3, 20, 33), True, dict(precision="fp64", wet_mode=2, wet_value=0.9, omega=OM),
     {"step_path": 1}),
    ("fused periodic fp32 ragged", (40, 37, 70), False, dict(precision="fp32"), {"step_path": 2}),
    ("fused walls fp64", (21, 26, 40), True, dict(precision="fp64", wet_mode=1, wet_value=1.3, omega=OM),
     {"step_path": 2}),
]


def _sim(chunk, sched, **kw):
    return make_sim(chain_chunk=chunk or 0, **sched, **kw)


def _raw(t):
    return t.detach().contiguous().view(torch.uint8).cpu()


@pytest.mark.parametrize("label,shape,walls,extra,sched", CASES, ids=[c[0] for c in CASES])
def test_chain_chunk_length_changes_nothing(label, shape, walls, extra, sched):
    say(f"chain chunks: {label}")
    T = eos.temperature(0.7 if walls else 0.85)
    nz, ny, nx = shape
    kw = dict(nx=nx, ny=ny, nz=nz, T=T, walls_z=int(walls), **extra)
    sims = [_sim(c, sched, **kw) for c in (None, 1, 3, 8, 32, 64)]
    rho0 = droplet_rho(shape, T, walls=walls, radius=min(ny, nx) / 3.0)
    g = np.random.Generator(np.random.PCG64(9))
    u0 = torch.tensor(0.02 * g.uniform(-1, 1, (3,) + shape))
    for s in sims:
        s.init_density(torch.tensor(rho0), u0)
    for step in range(4):
        for s in sims:
            s.step(1 + step)
        ref = _raw(sims[0].get_state())
        for s in sims[1:]:
            assert torch.equal(_raw(s.get_state()), ref), f"{label}: state differs after call {step}"
        f0 = sims[0].fields()
        for s in sims[1:]:
            f = s.fields()
            for name in ("rho", "u", "mu", "F"):
                assert torch.equal(f[name].cpu(), f0[name].cpu()), f"{label}: {name} differs"
