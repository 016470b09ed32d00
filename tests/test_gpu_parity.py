"""Parity of the HIP FP64 path with the CPU oracle: per-step fields and
populations from identical states (max relative error 1e-11 per field, per
population), short trajectories, and sampled nodes at the 128^3 benchmark
size in the launch configuration the benchmark times."""
import numpy as np
import pytest
import torch

from gpu_util import (DT, droplet_rho, fluid_slice, gpu_fields, make_sim, oracle_fields, oracle_params, rel_err,
                      sampled_windows, say)
from oracle import eos, lbm
from paper_2504_03819_amd import inputs, lbfe

pytestmark = pytest.mark.gpu
TOL = 1e-11


def check_state(sim, f_state, label):
    """Fields of f(t) and populations of f(t+1), GPU vs oracle."""
    p = oracle_params(sim)
    sim.set_populations(f_state)
    g = gpu_fields(sim)
    o = oracle_fields(f_state, p)
    # a field that vanishes identically (F and Q on a one-node periodic box,
    # where every link returns to the node) holds rounding residue on both
    # sides: compare it absolutely
    errs = {k: rel_err(g[k], o[k]) if float(o[k].abs().max()) > 1e-14 else float((g[k] - o[k]).abs().max())
            for k in o}
    sim.step(1)
    fg = sim.populations().cpu()
    fo = lbm.step(f_state, p)
    sl = slice(1, -1) if p.walls_z else slice(None)
    errs["f"] = max(rel_err(fg[i, sl], fo[i, sl]) for i in range(27))
    say(f"{label}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v < TOL, (label, k, v)


CASES = [
    # (label, shape (nz, ny, nx), walls, extra params)
    ("periodic 8^3", (8, 8, 8), False, {}),
    ("ragged 10x12x17", (10, 12, 17), False, {}),
    ("flat 128x4x4", (128, 4, 4), False, {}),
    ("rates random, no corr4", (9, 11, 13), False,
     dict(omega=[0.7, 1.0, 1.3, 0.6, 1.8, 1.1, 0.5, 1.9, 0.9, 1.4, 1.2], corr4=0)),
    ("walls neutral", (12, 9, 7), True, dict(wet_mode=0)),
    ("walls phi 1.6", (12, 9, 7), True, dict(wet_mode=1, wet_value=1.6)),
    ("walls drho 1.8", (12, 9, 7), True, dict(wet_mode=2, wet_value=1.8)),
    ("moving walls phi 1.4", (12, 9, 7), True, dict(wet_mode=1, wet_value=1.4, wall_u=(0.08, -0.03, -0.05, 0.02))),
    ("moving walls, one fluid plane", (3, 9, 7), True, dict(wall_u=(0.1, 0.0, -0.1, 0.05))),
    # degenerate boxes: a periodic extent of 1 wraps every link onto the node itself
    ("single z-plane 1x7x9", (1, 7, 9), False, {}),
    ("single y-row 6x1x5", (6, 1, 5), False, {}),
    ("single x-column 5x6x1", (5, 6, 1), False, {}),
    ("single node 1x1x1", (1, 1, 1), False, {}),
]


@pytest.mark.parametrize("label,shape,walls,extra", CASES, ids=[c[0] for c in CASES])
def test_one_step_parity(label, shape, walls, extra):
    say(f"case {label}")
    T = eos.temperature(0.7 if walls else 0.85)
    nz, ny, nx = shape
    sim = make_sim(nx=nx, ny=ny, nz=nz, T=T, walls_z=int(walls), **extra)
    p = oracle_params(sim)
    rho0 = droplet_rho(shape, T, walls=walls)
    g = np.random.Generator(np.random.PCG64(17))
    u0 = 0.03 * (g.uniform(-1, 1, (3,) + shape))
    f0 = lbm.init(torch.tensor(rho0), p, torch.tensor(u0))
    # GPU initialiser parity
    sim.init_density(torch.tensor(rho0), torch.tensor(u0))
    e_init = rel_err(sim.populations().cpu(), f0)
    say(f"{label}: init f err={e_init:.2e}")
    assert e_init < TOL
    # leave the equilibrium manifold so every moment order is exercised
    f = f0 + torch.tensor(inputs.uniform_noise(tuple(f0.shape), 2e-4, 23)) * (f0 != 0)
    check_state(sim, f, label)


def test_trajectory_stationary_droplet_32():
    """The stationary-droplet workload: 32^3 at 0.9 Tc, radius 8, noise 1e-6,
    its full 500 steps; fields and all 27 populations against the oracle
    every 100 steps."""
    T = eos.temperature(0.9)
    sim = make_sim(nx=32, ny=32, nz=32, T=T)
    p = oracle_params(sim)
    rho0, _ = inputs.stationary_droplet(sim.rho_l, sim.rho_v)
    sim.init_density(torch.tensor(rho0))
    f = lbm.init(torch.tensor(rho0), p)
    for t in range(100, 501, 100):
        sim.step(100)
        f = lbm.run(f, p, 100)
        g = gpu_fields(sim)
        o = oracle_fields(f, p)
        # a field that vanishes identically (F and Q on a one-node periodic
        # box, where every link returns to the node) holds rounding residue on
        # both sides: compare it absolutely
        errs = {k: rel_err(g[k], o[k]) if float(o[k].abs().max()) > 1e-14 else float((g[k] - o[k]).abs().max())
                for k in o}
        fg = sim.populations().cpu()
        errs["f"] = rel_err(fg, f)
        errs["f_i"] = max(rel_err(fg[i], f[i]) for i in range(27))  # each direction on its own scale
        say(f"droplet32 t={t}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        for k, v in errs.items():
            assert v < TOL, (t, k, v)


def test_trajectory_sessile_droplet_walls():
    T = eos.temperature(0.7)
    shape = (14, 12, 16)
    sim = make_sim(nx=16, ny=12, nz=14, T=T, walls_z=1, wet_mode=lbfe.WET_PHI, wet_value=1.3)
    p = oracle_params(sim)
    rho0 = droplet_rho(shape, T, radius=5.0, walls=True, noise=0)
    sim.init_density(torch.tensor(rho0))
    f = lbm.init(torch.tensor(rho0), p)
    sim.step(30)
    f = lbm.run(f, p, 30)
    fg = sim.populations().cpu()
    e = rel_err(fg[:, 1:-1], f[:, 1:-1])
    g = gpu_fields(sim)
    o = oracle_fields(f, p)
    # a field that vanishes identically (F and Q on a one-node periodic box,
    # where every link returns to the node) holds rounding residue on both
    # sides: compare it absolutely
    errs = {k: rel_err(g[k], o[k]) if float(o[k].abs().max()) > 1e-14 else float((g[k] - o[k]).abs().max())
            for k in o}
    say(f"sessile t=30: f={e:.2e} " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert e < TOL and all(v < TOL for v in errs.values())


def test_trajectory_moving_walls():
    """Droplet between walls moving in opposite directions (the moving-wall
    boundary of the Sec. III B test), 30 steps against the oracle."""
    T = eos.temperature(0.7)
    shape = (14, 12, 16)
    sim = make_sim(nx=16, ny=12, nz=14, T=T, walls_z=1, wall_u=(0.1, 0.0, -0.1, 0.02),
                   omega=[1.0, 1.0, 1.0, 0.5] + [1.0] * 7)
    p = oracle_params(sim)
    rho0 = droplet_rho(shape, T, radius=4.0, noise=0)
    rho0[0] = rho0[-1] = sim.rho_v
    sim.init_density(torch.tensor(rho0))
    f = lbm.init(torch.tensor(rho0), p)
    sim.step(30)
    f = lbm.run(f, p, 30)
    fg = sim.populations().cpu()
    e = rel_err(fg[:, 1:-1], f[:, 1:-1])
    g = gpu_fields(sim)
    o = oracle_fields(f, p)
    # a field that vanishes identically (F and Q on a one-node periodic box,
    # where every link returns to the node) holds rounding residue on both
    # sides: compare it absolutely
    errs = {k: rel_err(g[k], o[k]) if float(o[k].abs().max()) > 1e-14 else float((g[k] - o[k]).abs().max())
            for k in o}
    say(f"moving walls t=30: f={e:.2e} " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    assert e < TOL and all(v < TOL for v in errs.values())


def test_full_size_moving_droplet_sampled():
    """128^3 moving droplet (the benchmark workload), one step in the
    benchmark's launch configuration; the oracle recomputes sampled nodes
    from windows of f(t) around them."""
    n = 128
    T = eos.temperature(0.85)
    sim = make_sim(nx=n, ny=n, nz=n, T=T)
    rho0, u0 = inputs.moving_droplet(sim.rho_l, sim.rho_v)
    sim.init_density(torch.tensor(rho0), torch.tensor(u0))
    sim.step(20)
    f_t = sim.populations()
    sim.step(1)
    f_t1 = sim.populations()
    g = np.random.Generator(np.random.PCG64(5))
    # sample centres on the interface, in the liquid and in the vapour
    centres = [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(4)]
    centres += [(64, 64, 64 + 24), (64, 64 + 24, 64), (0, 0, 0), (127, 64, 40)]
    sampled_windows(sim, f_t, f_t1, centres, TOL, "128^3 moving droplet")


def test_full_size_spinodal_sampled():
    """256^3 spinodal decomposition in FP64 (the bandwidth workload), 30
    steps in, sampled windows against the oracle."""
    n = 256
    T = eos.temperature(0.8)
    sim = make_sim(nx=n, ny=n, nz=n, T=T, check_every=1000)
    rho0, _ = inputs.spinodal(sim.rho_l, sim.rho_v)
    sim.init_density(torch.tensor(rho0))
    sim.step(30)
    f_t = sim.populations()
    sim.step(1)
    f_t1 = sim.populations()
    g = np.random.Generator(np.random.PCG64(6))
    centres = [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(6)] + [(0, 255, 128), (255, 0, 0)]
    sampled_windows(sim, f_t, f_t1, centres, TOL, "256^3 spinodal")


def test_full_size_wetting_sampled():
    """192x192x96 sessile droplet between walls (the wetting workload, FP64
    here), 30 steps in, sampled windows next to both walls, at the contact
    line and in the bulk."""
    T = eos.temperature(0.7)
    sim = make_sim(nx=192, ny=192, nz=96, T=T, walls_z=1, wet_mode=lbfe.WET_PHI, wet_value=1.3,
                   omega=[1.0, 1.0, 1.0, 0.5] + [1.0] * 7)
    rho0, _ = inputs.sessile_droplet(sim.rho_l, sim.rho_v)
    sim.init_density(torch.tensor(rho0))
    sim.step(30)
    f_t = sim.populations()
    sim.step(1)
    f_t1 = sim.populations()
    centres = [(2, 96, 96), (3, 96, 96 + 32), (1, 96 + 31, 96), (2, 0, 0), (93, 50, 60), (94, 96, 96),
               (20, 96, 96 + 28), (48, 10, 150)]
    sampled_windows(sim, f_t, f_t1, centres, TOL, "192x192x96 wetting")


def test_full_size_collision_512_fp32_sampled():
    """512^3 head-on collision in FP32 storage and arithmetic (the largest
    configuration), 10 steps in: sampled windows of the FP32 state stepped by
    the FP64 oracle agree to the FP32 level."""
    n = 512
    T = eos.temperature(0.85)
    sim = make_sim(nx=n, ny=n, nz=n, T=T, precision="fp32", check_every=1000)
    rho0, u0 = inputs.head_on_collision(sim.rho_l, sim.rho_v)
    sim.init_density(torch.tensor(rho0), torch.tensor(u0))
    del rho0, u0
    sim.step(10)
    f_t = sim.populations()
    sim.step(1)
    f_t1 = sim.populations()
    centres = [(256, 256, 176 + 64), (256, 256, 336 - 64), (256, 256 + 64, 176), (256, 256, 256), (0, 0, 0),
               (300, 200, 176)]
    sampled_windows(sim, f_t, f_t1, centres, 2e-6, "512^3 collision FP32")


def test_full_size_collision_512_fp64_sampled():
    """The benchmark's headline configuration: the 512^3 head-on collision
    in FP64 on the path and schedule the library picks for it (the fused
    collide-stream-moments kernel, XCD-contiguous tile order, 64-plane
    chunks), 10 steps in: sampled windows against the oracle to the FP64
    tolerance of the one-step cases."""
    n = 512
    T = eos.temperature(0.85)
    sim = make_sim(nx=n, ny=n, nz=n, T=T, check_every=1000)
    assert sim.params.step_path == lbfe.PATH_FUSED and sim.params.tile_order == lbfe.ORDER_XCD
    rho0, u0 = inputs.head_on_collision(sim.rho_l, sim.rho_v)
    sim.init_density(torch.tensor(rho0), torch.tensor(u0))
    del rho0, u0
    sim.step(10)
    f_t = sim.populations()
    sim.step(1)
    f_t1 = sim.populations()
    centres = [(256, 256, 176 + 64), (256, 256, 336 - 64), (256, 256 + 64, 176), (256, 256, 256), (0, 0, 0),
               (300, 200, 176), (511, 511, 511), (64, 448, 100)]
    sampled_windows(sim, f_t, f_t1, centres, TOL, "512^3 collision FP64 (fused)")
    del f_t, f_t1
    sim.close()
    torch.cuda.empty_cache()


def test_step_is_deterministic():
    T = eos.temperature(0.8)
    sim = make_sim(nx=24, ny=20, nz=16, T=T)
    rho0 = droplet_rho((16, 20, 24), T, noise=1e-2, seed=4)
    out = []
    for _ in range(2):
        sim.init_density(torch.tensor(rho0))
        sim.step(10)
        out.append(sim.get_state().clone())
    assert torch.equal(out[0], out[1])


def test_reductions_and_invariants():
    T = eos.temperature(0.85)
    n = 20
    sim = make_sim(nx=n, ny=n, nz=n, T=T)
    rho0 = droplet_rho((n, n, n), T, noise=1e-2)
    g = np.random.Generator(np.random.PCG64(8))
    u0 = 0.02 * g.uniform(-1, 1, (3, n, n, n))
    sim.init_density(torch.tensor(rho0), torch.tensor(u0))
    r0 = sim.reduce()
    assert abs(r0[0] - rho0.sum()) < 1e-12 * rho0.sum()
    for _ in range(5):
        r = sim.reduce()
        sim.step(1)
        r1 = sim.reduce()
        assert abs(r1[0] - r0[0]) < 1e-13 * r0[0]
        for a in range(3):  # momentum balance: sum j(t+1) - sum j(t) = sum F(t)
            assert abs((r1[1 + a] - r[1 + a]) - r[4 + a]) < 1e-12
    fl = sim.fields()
    assert abs(float(fl["u"].norm(dim=0).max()) - r1[7]) < 1e-14


@pytest.mark.parametrize("walls", [False, True], ids=["periodic", "walls"])
def test_reductions_against_the_oracle(walls):
    """lbfe_reduce (mass, momentum, total force, max |u|) against the same
    sums of the oracle's fields of the same state: sums to 1e-12 of the sum
    of magnitudes, the maximum to 1e-12."""
    T = eos.temperature(0.7 if walls else 0.85)
    shape = (18, 20, 22)
    nz, ny, nx = shape
    extra = dict(walls_z=1, wet_mode=lbfe.WET_PHI, wet_value=1.3, omega=[1.0, 1.0, 1.0, 0.5] + [1.0] * 7) \
        if walls else {}
    sim = make_sim(nx=nx, ny=ny, nz=nz, T=T, **extra)
    p = oracle_params(sim)
    rho0 = droplet_rho(shape, T, walls=walls, noise=1e-2, seed=12)
    g = np.random.Generator(np.random.PCG64(14))
    u0 = 0.03 * g.uniform(-1, 1, (3,) + shape)
    sim.init_density(torch.tensor(rho0), torch.tensor(u0))
    sim.step(7)
    f = sim.populations().cpu()
    A = lbm.aux_fields(f, p)
    fl = fluid_slice(p)
    rho, j, F, u = A["rho"][fl], A["j"][:, fl], A["F"][:, fl], A["u"][:, fl]
    ref = [float(rho.sum())] + [float(j[a].sum()) for a in range(3)] + [float(F[a].sum()) for a in range(3)] \
        + [float(u.norm(dim=0).max())]
    scale = [float(rho.abs().sum())] + [float(j[a].abs().sum()) for a in range(3)] \
        + [float(F[a].abs().sum()) for a in range(3)] + [ref[7]]
    got = sim.reduce()
    errs = [abs(a - b) / s for a, b, s in zip(got, ref, scale)]
    say(f"reductions vs oracle ({'walls' if walls else 'periodic'}): max err {max(errs):.2e}")
    assert max(errs) < 1e-12, list(zip(got, ref))


def test_invalid_density_and_divergence_flag():
    T = eos.temperature(0.85)
    sim = make_sim(nx=8, ny=8, nz=8, T=T, check_every=1)
    rho0 = torch.full((8, 8, 8), 2.0, dtype=DT)
    rho0[3, 3, 3] = float("nan")
    with pytest.raises(lbfe.LBFEError) as ei:
        sim.init_density(rho0)
    assert ei.value.code == lbfe.E_INVAL
    rho0[3, 3, 3] = 11.0   # beyond 1/b = 10.5
    with pytest.raises(lbfe.LBFEError):
        sim.init_density(rho0)
    with pytest.raises(lbfe.LBFEError) as ei:
        sim.step(1)        # no state yet
    assert ei.value.code == lbfe.E_STATE
    rho0[3, 3, 3] = 2.0
    sim.init_density(rho0)
    f = sim.populations()
    f[13, 2, 2, 2] += 12.0  # push one node outside the EOS domain
    sim.set_populations(f)
    with pytest.raises(lbfe.LBFEError) as ei:
        sim.step(2)
    assert ei.value.code == lbfe.E_DIVERGED


def test_state_roundtrip_and_counter():
    T = eos.temperature(0.85)
    sim = make_sim(nx=12, ny=12, nz=12, T=T)
    rho0 = droplet_rho((12, 12, 12), T)
    sim.init_density(torch.tensor(rho0))
    sim.step(3)
    s3 = sim.get_state().clone()
    sim.step(4)
    s7 = sim.get_state().clone()
    assert sim.step_count == 7
    sim.set_state(s3, 3)
    sim.step(4)
    assert sim.step_count == 7
    assert torch.equal(sim.get_state(), s7)


def test_zero_steps_change_nothing():
    T = eos.temperature(0.85)
    sim = make_sim(nx=9, ny=8, nz=7, T=T)
    sim.init_density(torch.tensor(droplet_rho((7, 8, 9), T)))
    s0 = sim.get_state().clone()
    sim.step(0)
    assert torch.equal(sim.get_state(), s0)
    assert sim.step_count == 0
