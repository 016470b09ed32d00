"""The moment-representation state path (every rate but omega_1 at 1, the
paper's setting stated after Eq. (26) of Sec. II B): between the steps of one
call each node holds 16 post-collision numbers instead of 27 populations.
The rebuilt populations are those of the population path's collision, so the
state path agrees bit for bit with the two-pass path for any split of the
steps into calls (entering and leaving the state form each time), for FP64
and FP32, on boxes smaller than a tile, ragged boxes spanning several tiles
and z-chunks, walled boxes with each wetting mode, and degenerate boxes; and
with the oracle to 1e-11 (FP64) over several steps from off-equilibrium
states, so the collide and moments passes of the state form are both
covered."""
import numpy as np
import pytest
import torch

from gpu_util import DT, droplet_rho, make_sim, oracle_params, rel_err, sampled_windows, say
from oracle import eos, lbm
from paper_2504_03819_amd import inputs, lbfe

pytestmark = pytest.mark.gpu

FORMS = ["fp64", "fp32"]
CASES = [
    # (label, shape (nz, ny, nx), walls, extra)
    ("small 7x8x9", (7, 8, 9), False, {}),
    ("ragged 40x37x70", (40, 37, 70), False, {}),
    ("no corr4 16x16x16", (16, 16, 16), False, dict(corr4=0)),
    ("walls neutral 12x9x7", (12, 9, 7), True, dict(wet_mode=0)),
    ("walls phi 1.4 34x21x45", (34, 21, 45), True, dict(wet_mode=1, wet_value=1.4)),
    ("walls drho 0.9 3-plane", (3, 20, 33), True, dict(wet_mode=2, wet_value=0.9)),
    ("single z-plane 1x7x9", (1, 7, 9), False, {}),
    ("single node 1x1x1", (1, 1, 1), False, {}),
]
SPLITS = (1, 3, 4, 2)  # steps per call


def _raw(t):
    return t.detach().contiguous().view(torch.uint8).cpu()


def _pair(form, shape, walls, extra, T):
    nz, ny, nx = shape
    kw = dict(nx=nx, ny=ny, nz=nz, T=T, walls_z=int(walls), precision=form, **extra)
    return [make_sim(step_path=lbfe.PATH_TWO_PASS, **kw), make_sim(step_path=lbfe.PATH_STATE, **kw)]


def _init(sims, shape, walls, T, seed=5):
    nz, ny, nx = shape
    rho0 = droplet_rho(shape, T, walls=walls, radius=max(1.0, (min(ny, nx) if walls else min(shape)) / 3.0))
    g = np.random.Generator(np.random.PCG64(seed))
    u0 = torch.tensor(0.02 * g.uniform(-1, 1, (3,) + shape))
    for s in sims:
        s.init_density(torch.tensor(rho0), u0)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("label,shape,walls,extra", CASES, ids=[c[0] for c in CASES])
def test_state_path_equals_two_pass_bitwise(form, label, shape, walls, extra):
    say(f"state vs two-pass: {label} {form}")
    T = eos.temperature(0.7 if walls else 0.85)
    sims = _pair(form, shape, walls, extra, T)
    assert sims[1].params.step_path == lbfe.PATH_STATE
    _init(sims, shape, walls, T)
    done = 0
    for n in SPLITS:
        for s in sims:
            s.step(n)
        done += n
        a, b = (_raw(s.get_state()) for s in sims)
        if not torch.equal(a, b):
            fa, fb = (s.populations().cpu() for s in sims)
            d = (fa - fb).abs()
            raise AssertionError(f"{label} {form}: populations differ after {done} steps: max |diff| "
                                 f"{float(d.max()):.3e} at {np.unravel_index(int(d.argmax()), d.shape)}, "
                                 f"{int((d > 0).sum())} of {d.numel()} entries")
        assert sims[1].step_count == done
    fa, fb = (s.fields() for s in sims)
    for k in fa:
        assert torch.equal(_raw(fa[k]), _raw(fb[k])), (label, form, k)
    assert sims[0].reduce() == sims[1].reduce()


@pytest.mark.parametrize("label,shape,walls,extra", [
    ("ragged 10x12x17", (10, 12, 17), False, {}),
    ("walls phi 1.6", (12, 9, 7), True, dict(wet_mode=1, wet_value=1.6)),
    ("walls drho 1.8", (12, 9, 7), True, dict(wet_mode=2, wet_value=1.8)),
], ids=lambda v: v if isinstance(v, str) else None)
def test_state_path_matches_oracle(label, shape, walls, extra):
    """Three steps in one call (enter, two collide passes, two moments passes,
    leave) from an off-equilibrium state, FP64, against three oracle steps."""
    T = eos.temperature(0.7 if walls else 0.85)
    nz, ny, nx = shape
    sim = make_sim(nx=nx, ny=ny, nz=nz, T=T, walls_z=int(walls), step_path=lbfe.PATH_STATE, **extra)
    p = oracle_params(sim)
    rho0 = droplet_rho(shape, T, walls=walls)
    g = np.random.Generator(np.random.PCG64(29))
    u0 = 0.03 * g.uniform(-1, 1, (3,) + shape)
    f = lbm.init(torch.tensor(rho0), p, torch.tensor(u0))
    f = f + torch.tensor(inputs.uniform_noise(tuple(f.shape), 2e-4, 31)) * (f != 0)
    sim.set_populations(f)
    sim.step(3)
    fo = f
    for _ in range(3):
        fo = lbm.step(fo, p)
    fg = sim.populations().cpu()
    sl = slice(1, -1) if walls else slice(None)
    err = max(rel_err(fg[i, sl], fo[i, sl]) for i in range(27))
    say(f"{label}: state path vs oracle after 3 steps: {err:.2e}")
    assert err < 1e-11


def test_state_path_timed_and_divergence():
    T = eos.temperature(0.85)
    shape = (20, 24, 40)
    sims = _pair("fp64", shape, False, {}, T)
    _init(sims, shape, False, T)
    kms = sims[1].step_timed(3)
    sims[0].step(3)
    assert torch.equal(_raw(sims[0].get_state()), _raw(sims[1].get_state()))
    say(f"state path step_timed: {kms}")
    assert kms["moments"] > 0 and kms["chain"] > 0 and kms["collide_stream"] > 0 and kms["wall_rho"] == 0
    # a node pushed out of the EOS domain: diverged at the first check, and
    # the context leaves the state form (populations readable, counter set)
    sim = make_sim(nx=8, ny=8, nz=8, T=T, check_every=1, step_path=lbfe.PATH_STATE)
    sim.init_density(torch.full((8, 8, 8), 2.0, dtype=DT))
    f = sim.populations()
    f[13, 2, 2, 2] += 12.0
    sim.set_populations(f)
    with pytest.raises(lbfe.LBFEError) as ei:
        sim.step(4)
    assert ei.value.code == lbfe.E_DIVERGED
    assert sim.step_count == 1
    assert sim.populations().shape == (27, 8, 8, 8)


def test_state_path_large_sampled_against_two_pass():
    """256^3 periodic droplet pair in the schedule the benchmark uses for
    large grids (XCD tile order, many z-chunks), FP32: ten steps in one call
    equal the two-pass path bit for bit."""
    T = eos.temperature(0.85)
    n = 256
    shape = (n, n, n)
    rl, rv = eos.maxwell(eos.PAPER["a"], eos.PAPER["b"], 1.0, T)
    rho0 = inputs.sphere(shape, (n * 0.35, n / 2, n / 2), 40, rl, rv)
    rho0 = np.maximum(rho0, inputs.sphere(shape, (n * 0.65, n / 2, n / 2), 40, rl, rv))
    sims = _pair("fp32", shape, False, {}, T)
    for s in sims:
        s.init_density(torch.tensor(rho0))
        s.step(10)
    a, b = (s.get_state() for s in sims)
    assert torch.equal(a, b)
    say("256^3 fp32: state path equals two-pass after 10 steps")


@pytest.mark.parametrize("form", FORMS)
def test_state_path_long_run_equals_two_pass(form):
    """500 steps in one call (498 of them inside the state form) on the 64^3
    stationary-droplet setup with a small flow, then 1 and 7 more: the same
    bits as the two-pass path."""
    T = eos.temperature(0.85)
    shape = (64, 64, 64)
    sims = _pair(form, shape, False, {}, T)
    _init(sims, shape, False, T, seed=13)
    for n in (500, 1, 7):
        for s in sims:
            s.step(n)
        assert torch.equal(sims[0].get_state(), sims[1].get_state()), (form, n)
    say(f"64^3 {form}: state path equals two-pass after 508 steps")


def test_state_path_full_size_collision_sampled():
    """The 512^3 head-on collision (the benchmark's `fp64_state` form) on the
    state path, 10 steps in one call and one more: sampled windows of f(t)
    stepped by the oracle against f(t+1), FP64 tolerance."""
    n = 512
    T = eos.temperature(0.85)
    sim = make_sim(nx=n, ny=n, nz=n, T=T, check_every=1000, step_path=lbfe.PATH_STATE)
    assert sim.params.step_path == lbfe.PATH_STATE
    rl, rv = eos.maxwell(eos.PAPER["a"], eos.PAPER["b"], 1.0, T)
    rho0, u0 = inputs.head_on_collision(rl, rv)
    sim.init_density(torch.tensor(rho0), torch.tensor(u0))
    del rho0, u0
    sim.step(10)
    f_t = sim.populations()
    sim.step(1)
    f_t1 = sim.populations()
    centres = [(256, 256, 176 + 64), (256, 256, 336 - 64), (256, 256 + 64, 176), (0, 0, 0), (511, 300, 20)]
    sampled_windows(sim, f_t, f_t1, centres, 1e-11, "512^3 collision, state path FP64")
    del f_t, f_t1
    sim.close()
    torch.cuda.empty_cache()
