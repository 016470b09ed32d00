"""The fused collide-stream-moments step against the unfused reference path
(separate moments pass and collide-stream kernel): both sum the moments in
the same fixed order, so populations, density, momentum and the derived
fields must agree bit for bit after every step, for every storage form, on
grids smaller than a tile, ragged grids spanning several tiles and chunks,
walled boxes, and walled boxes with moving walls (the wall term applied after
the fused kernel)."""
import numpy as np
import pytest
import torch

from gpu_util import droplet_rho, make_sim, say
from oracle import eos
from paper_2504_03819_amd import lbfe

pytestmark = pytest.mark.gpu

FORMS = ["fp64", "fp32", "fp16dev", "fp16dev_f0fp32"]
CASES = [
    # (label, shape (nz, ny, nx), walls, extra)
    ("small 7x8x9", (7, 8, 9), False, {}),
    ("ragged 40x37x70", (40, 37, 70), False, {}),
    ("walls phi 1.4 34x21x45", (34, 21, 45), True, dict(wet_mode=1, wet_value=1.4)),
    ("walls drho 0.9 3-plane", (3, 20, 33), True, dict(wet_mode=2, wet_value=0.9)),
    ("moving walls phi 1.3 30x22x41", (30, 22, 41), True,
     dict(wet_mode=1, wet_value=1.3, wall_u=(0.08, -0.03, -0.05, 0.02))),
    ("moving walls 3-plane", (3, 17, 35), True, dict(wall_u=(0.1, 0.0, -0.1, 0.05))),
]


def _sim(unfused, **kw):
    return make_sim(step_path=lbfe.PATH_TWO_PASS if unfused else lbfe.PATH_FUSED, **kw)


def _raw(t):
    return t.detach().contiguous().view(torch.uint8).cpu()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("label,shape,walls,extra", CASES, ids=[c[0] for c in CASES])
def test_fused_equals_unfused_bitwise(form, label, shape, walls, extra):
    say(f"fused vs unfused: {label} {form}")
    T = eos.temperature(0.7 if walls else 0.85)
    nz, ny, nx = shape
    kw = dict(nx=nx, ny=ny, nz=nz, T=T, walls_z=int(walls), precision=form, **extra)
    if walls:
        kw["omega"] = [1.0, 1.0, 1.0, 0.5] + [1.0] * 7
    sims = [_sim(False, **kw), _sim(True, **kw)]
    rho0 = droplet_rho(shape, T, walls=walls, radius=min(shape) / 3.0 if not walls else min(ny, nx) / 3.0)
    g = np.random.Generator(np.random.PCG64(5))
    u0 = torch.tensor(0.02 * g.uniform(-1, 1, (3,) + shape))
    for s in sims:
        s.init_density(torch.tensor(rho0), u0)
    for step in range(1, 7):
        for s in sims:
            s.step(1)
        a, b = (_raw(s.get_state()) for s in sims)
        if not torch.equal(a, b):
            fa, fb = (s.populations().cpu() for s in sims)
            d = (fa - fb).abs()
            raise AssertionError(f"{label} {form}: populations differ at step {step}: max |diff| "
                                 f"{float(d.max()):.3e} at {np.unravel_index(int(d.argmax()), d.shape)}, "
                                 f"{int((d > 0).sum())} of {d.numel()} entries")
    fa, fb = (s.fields() for s in sims)
    for k in fa:
        assert torch.equal(_raw(fa[k]), _raw(fb[k])), (label, form, k)
    ra, rb = (s.reduce() for s in sims)
    assert ra == rb


@pytest.mark.parametrize("form", ["fp64", "fp16dev"])
def test_restart_from_state_is_bitwise_continuous(form):
    """A state restored mid-run (moments re-formed by the moments pass) steps
    on exactly like the uninterrupted fused run."""
    T = eos.temperature(0.85)
    shape = (36, 33, 40)
    sim = _sim(False, nx=40, ny=33, nz=36, T=T, precision=form)
    sim.init_density(torch.tensor(droplet_rho(shape, T)))
    sim.step(4)
    s4 = sim.get_state().clone()
    sim.step(5)
    s9 = _raw(sim.get_state())
    r9 = sim.fields()["rho"]
    sim.set_state(s4, 4)
    sim.step(5)
    assert torch.equal(_raw(sim.get_state()), s9)
    assert torch.equal(sim.fields()["rho"], r9)
