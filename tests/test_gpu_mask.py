"""The solid-mask path (arbitrary voxel masks, lbfe_set_solid) against the
CPU oracle: initialiser, per-step fields and populations (FP64, 1e-11),
trajectories, the plane mask against the built-in flat walls, mass
conservation, and the FP32 form against FP64."""
import numpy as np
import pytest
import torch

from gpu_util import droplet_rho, gpu_fields, make_sim, oracle_fields, oracle_params, rel_err, say
from oracle import eos, lbm
from paper_2504_03819_amd import inputs, lbfe

pytestmark = pytest.mark.gpu
TOL = 1e-11
OM = [1.0, 1.0, 1.0, 0.5] + [1.0] * 7  # omega_3 = 1/2 next to solids at 0.7 T_c


def _mask(kind, shape):
    if kind == "obstacles":
        return inputs.mask_obstacles(shape)
    if kind == "pillars":
        return inputs.mask_pillars(shape, plate=2, pitch=8, width=3, height=4)
    return inputs.mask_planes(shape)


def _rho(shape, T, mask, seed=0):
    rl, rv = eos.maxwell(eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"], T)
    nz, ny, nx = shape
    rho = inputs.sphere(shape, (0.5 * nx, 0.5 * ny, 0.4 * nz), min(shape) / 3.0, rl, rv)
    rho = rho + inputs.uniform_noise(shape, 1e-3, seed)
    rho[mask.astype(bool)] = rv  # ignored at solid nodes
    return rho


CASES = [
    # (label, mask kind, shape (nz, ny, nx), extra params)
    ("obstacles neutral", "obstacles", (10, 9, 12), dict(wet_mode=0)),
    ("obstacles phi 1.4", "obstacles", (10, 9, 12), dict(wet_mode=1, wet_value=1.4)),
    ("obstacles drho 0.9", "obstacles", (10, 9, 12), dict(wet_mode=2, wet_value=0.9)),
    ("pillars phi 1.3 ragged", "pillars", (14, 19, 21), dict(wet_mode=1, wet_value=1.3)),
    ("planes drho 1.2", "planes", (9, 8, 11), dict(wet_mode=2, wet_value=1.2)),
    ("obstacles 70 wide, several blocks", "obstacles", (8, 6, 70), dict(wet_mode=1, wet_value=1.6)),
]


@pytest.mark.parametrize("label,kind,shape,extra", CASES, ids=[c[0] for c in CASES])
def test_mask_one_step_parity(label, kind, shape, extra):
    say(f"mask case {label}")
    T = eos.temperature(0.7)
    nz, ny, nx = shape
    mask = _mask(kind, shape)
    sim = make_sim(nx=nx, ny=ny, nz=nz, T=T, omega=OM, solid=mask, **extra)
    p = oracle_params(sim)
    assert p.solid is not None and int(p.solid.sum()) == int(mask.sum())
    rho0 = _rho(shape, T, mask)
    g = np.random.Generator(np.random.PCG64(17))
    u0 = 0.03 * g.uniform(-1, 1, (3,) + shape)
    f0 = lbm.init(torch.tensor(rho0), p, torch.tensor(u0))
    sim.init_density(torch.tensor(rho0), torch.tensor(u0))
    e_init = rel_err(sim.populations().cpu(), f0)
    assert e_init < TOL, e_init
    f = f0 + torch.tensor(inputs.uniform_noise(tuple(f0.shape), 2e-4, 23)) * (f0 != 0)
    sim.set_populations(f)
    gf = gpu_fields(sim)
    of = oracle_fields(f, p)
    errs = {k: rel_err(gf[k], of[k]) for k in of}
    sim.step(1)
    errs["f"] = max(rel_err(sim.populations().cpu()[i], lbm.step(f, p)[i]) for i in range(27))
    say(f"{label}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v < TOL, (label, k, v)


def test_mask_trajectory():
    """25 steps of a droplet among obstacles (phi = 1.4) against the oracle."""
    shape = (10, 12, 13)
    T = eos.temperature(0.7)
    mask = _mask("obstacles", shape)
    sim = make_sim(nx=13, ny=12, nz=10, T=T, omega=OM, solid=mask, wet_mode=1, wet_value=1.4)
    p = oracle_params(sim)
    rho0 = _rho(shape, T, mask, seed=4)
    sim.init_density(torch.tensor(rho0))
    f = lbm.init(torch.tensor(rho0), p)
    for _ in range(25):
        f = lbm.step(f, p)
    sim.step(25)
    e = rel_err(sim.populations().cpu(), f)
    er = rel_err(sim.fields()["rho"].cpu(), lbm.aux_fields(f, p)["rho"])
    say(f"mask trajectory 25 steps: f {e:.2e} rho {er:.2e}")
    assert e < 1e-10 and er < 1e-10


@pytest.mark.parametrize("form", ["fp64", "fp32", "fp16dev_f0fp32"])
def test_plane_mask_matches_flat_walls(form):
    """The mask of the planes z = 0, nz-1 against the built-in walls path
    (a different kernel set: the stencil chain in LDS tiles vs per-node
    gathers) over 40 steps."""
    shape = (20, 18, 24)
    nz, ny, nx = shape
    T = eos.temperature(0.7)
    kw = dict(nx=nx, ny=ny, nz=nz, T=T, omega=OM, wet_mode=1, wet_value=1.3, precision=form)
    a = make_sim(walls_z=1, **kw)
    b = make_sim(solid=inputs.mask_planes(shape), **kw)
    rho0 = droplet_rho(shape, T, walls=True, radius=7.0)
    for s in (a, b):
        s.init_density(torch.tensor(rho0))
        s.step(40)
    e = rel_err(b.populations().cpu()[:, 1:-1], a.populations().cpu()[:, 1:-1])
    say(f"plane mask vs walls {form}: {e:.2e}")
    assert e < {"fp64": 1e-12, "fp32": 5e-6, "fp16dev_f0fp32": 2e-4}[form]


def test_mask_mass_conservation():
    shape = (24, 32, 32)
    T = eos.temperature(0.7)
    mask = _mask("pillars", shape)
    sim = make_sim(nx=32, ny=32, nz=24, T=T, omega=OM, solid=mask, wet_mode=1, wet_value=1.3)
    sim.init_density(torch.tensor(_rho(shape, T, mask)))
    m0 = sim.reduce()[0]
    sim.step(300)
    m1 = sim.reduce()[0]
    say(f"mask mass drift over 300 steps: {abs(m1 - m0) / m0:.2e}")
    assert abs(m1 - m0) <= 1e-12 * m0


def test_mask_fp32_against_fp64():
    shape = (16, 20, 20)
    T = eos.temperature(0.7)
    mask = _mask("obstacles", shape)
    rho0 = _rho(shape, T, mask, seed=8)
    out = {}
    for form in ("fp64", "fp32"):
        s = make_sim(nx=20, ny=20, nz=16, T=T, omega=OM, solid=mask, wet_mode=2, wet_value=0.9, precision=form)
        s.init_density(torch.tensor(rho0))
        s.step(50)
        out[form] = s.fields()["rho"].cpu()
    rl, rv = eos.maxwell(eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"], T)
    e = float((out["fp32"] - out["fp64"]).abs().max()) / (rl - rv)
    say(f"mask fp32 vs fp64 rho after 50 steps: {e:.2e} of rho_l - rho_v")
    assert e < 2e-5


def test_mask_call_order_errors():
    sim = make_sim(nx=8, ny=8, nz=8, solid_mask=1)
    with pytest.raises(lbfe.LBFEError) as e:
        sim.init_density(torch.full((8, 8, 8), 3.0, dtype=torch.float64))
    assert e.value.code == lbfe.E_STATE
    plain = make_sim(nx=8, ny=8, nz=8)
    with pytest.raises(lbfe.LBFEError) as e:
        plain.set_solid(np.zeros((8, 8, 8), dtype=np.uint8))
    assert e.value.code == lbfe.E_STATE


def test_y_walls_by_mask_match_z_walls_transposed():
    """Walls at y = 0 and y = ny-1 given as a mask reproduce the built-in
    z-wall path with the y and z axes exchanged (state, directions and box),
    over 30 steps of a sessile droplet with phi = 1.4."""
    nzw, nyw, nx = 16, 14, 18           # z-wall box (nz, ny, nx)
    T = eos.temperature(0.7)
    kw = dict(T=T, omega=OM, wet_mode=1, wet_value=1.4)
    a = make_sim(nx=nx, ny=nyw, nz=nzw, walls_z=1, **kw)
    mask = np.zeros((nyw, nzw, nx), dtype=np.uint8)  # box (nz', ny', nx) = (nyw, nzw, nx)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    b = make_sim(nx=nx, ny=nzw, nz=nyw, solid=mask, **kw)
    rho = droplet_rho((nzw, nyw, nx), T, walls=True, radius=5.0)
    a.init_density(torch.tensor(rho))
    b.init_density(torch.tensor(np.ascontiguousarray(rho.transpose(1, 0, 2))))
    a.step(30)
    b.step(30)
    fa = a.populations().cpu()                         # (27, z, y, x)
    fb = b.populations().cpu()                         # (27, z' = y, y' = z, x)
    from oracle.lattice import C
    perm = [C.index((c[0], c[2], c[1])) for c in C]    # direction with c_y and c_z exchanged
    fb_back = fb[perm].transpose(1, 2)
    e = rel_err(fb_back, fa)
    say(f"y-walls by mask vs z-walls: {e:.2e}")
    assert e < 1e-12
