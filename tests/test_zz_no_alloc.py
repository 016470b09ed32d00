"""lbfe_reduce_into, the reduction for callers that cannot allocate: its
block partials live in the library's static device scratch instead of the
workspace, and it writes the results to a caller-owned device buffer.  It
runs the same kernels in the same order as lbfe_reduce, so the results must
be bit for bit those of lbfe_reduce, on two calls in a row (the second on a
smaller context, so the scratch holds the first call's partials when it
starts), and it must refuse contexts beyond the scratch size before touching
the device."""
import pytest
import torch

from gpu_util import droplet_rho, make_sim, say
from oracle import eos
from paper_2504_03819_amd import lbfe

pytestmark = pytest.mark.gpu

OM = [1.0, 1.0, 1.0, 0.5] + [1.0] * 7


def _state(shape, walls, form, steps, **kw):
    nz, ny, nx = shape
    T = eos.temperature(0.7 if walls else 0.85)
    sim = make_sim(nx=nx, ny=ny, nz=nz, T=T, walls_z=int(walls), precision=form, **kw)
    sim.init_density(torch.tensor(droplet_rho(shape, T, walls=walls, radius=min(ny, nx) / 3.0, seed=7)))
    sim.step(steps)
    return sim


def test_reduce_into_equals_reduce_on_two_calls_in_a_row():
    cases = [
        ("periodic fp64 40x37x70", (40, 37, 70), False, "fp64", {}),
        ("walls fp32 12x9x11", (12, 9, 11), True, "fp32", dict(wet_mode=1, wet_value=1.3, omega=OM)),
    ]
    for label, shape, walls, form, kw in cases:
        say(f"reduce_into: {label}")
        sim = _state(shape, walls, form, 5, **kw)
        out = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda:0")
        sim.reduce_into(out)
        torch.cuda.synchronize()
        ref = sim.reduce()
        got = out.cpu().tolist()
        assert got == ref, (label, got, ref)
        assert ref[0] > 0  # the fluid mass
        sim.close()


def test_reduce_into_rejects_contexts_beyond_the_scratch():
    # 2^24 + 1 fluid nodes cannot fit 2^16 block partials of 256 nodes; the
    # size is checked before any device work (no workspace needed)
    p = lbfe.default_params(nx=4097, ny=4096, nz=1)
    ctx = lbfe.c_void_p()
    assert lbfe.lib().lbfe_create(lbfe.byref(p), None, lbfe.byref(ctx)) == lbfe.OK
    try:
        dummy = torch.zeros(8, dtype=torch.float64, device="cuda:0")
        rc = lbfe.lib().lbfe_reduce_into(ctx, lbfe.c_void_p(dummy.data_ptr()))
        assert rc == lbfe.E_INVAL
        assert b"static scratch" in lbfe.lib().lbfe_last_error(ctx)
    finally:
        lbfe.lib().lbfe_destroy(ctx)
