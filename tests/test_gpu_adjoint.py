"""The hand-written discrete adjoint against (1) the oracle's reverse mode
(torch autograd through the FP64 CPU oracle step), (2) central finite
differences of the GPU forward path, and (3) itself under different
checkpoint intervals (bitwise)."""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import DT, droplet_rho, make_sim, oracle_params, rel_err, say
from oracle import eos, lbm
from paper_2504_03819_amd import autograd as lag
from paper_2504_03819_amd import inputs, lbfe

pytestmark = pytest.mark.gpu


def _oracle_vjp(f, lam, p):
    kappa = torch.tensor(p.kappa, dtype=DT, requires_grad=True)
    wet = torch.tensor(p.wet_value, dtype=DT, requires_grad=True)
    nu = torch.tensor(p.nu, dtype=DT, requires_grad=True)
    pt = dataclasses.replace(p, kappa=kappa, wet_value=wet, nu=nu)
    fr = f.clone().requires_grad_(True)
    fn = lbm.step(fr, pt)
    (fn * lam).sum().backward()
    gw = float(wet.grad) if wet.grad is not None else 0.0
    return fr.grad, float(kappa.grad), gw, float(nu.grad)


CASES = [
    ("periodic 7x8x9", (9, 8, 7), False, {}),
    ("periodic random rates", (8, 8, 8), False,
     dict(omega=[0.7, 1.0, 1.3, 0.6, 1.8, 1.1, 0.5, 1.9, 0.9, 1.4, 1.2])),
    ("periodic no corr4", (8, 6, 10), False, dict(corr4=0)),
    ("walls phi 1.4", (12, 8, 9), True, dict(wet_mode=1, wet_value=1.4)),
    ("walls drho 1.2", (12, 8, 9), True, dict(wet_mode=2, wet_value=1.2)),
    ("walls neutral", (10, 7, 8), True, dict(wet_mode=0)),
    # several tiles and z-chunks of the z-marching kernels, ragged edges
    ("periodic multi-tile 37x11x35", (35, 11, 37), False, {}),
    ("walls phi 1.3 multi-tile 33x10x34", (34, 10, 33), True, dict(wet_mode=1, wet_value=1.3)),
    ("moving walls phi 1.4", (12, 8, 9), True, dict(wet_mode=1, wet_value=1.4, wall_u=(0.08, -0.03, -0.05, 0.02))),
    ("moving walls, one fluid plane", (3, 8, 9), True, dict(wall_u=(0.1, 0.0, -0.1, 0.05))),
]


@pytest.mark.parametrize("label,shape,walls,extra", CASES, ids=[c[0] for c in CASES])
def test_adjoint_step_matches_oracle_reverse_mode(label, shape, walls, extra):
    say(f"adjoint case {label}")
    T = eos.temperature(0.7 if walls else 0.85)
    nz, ny, nx = shape
    sim = make_sim(nx=nx, ny=ny, nz=nz, T=T, walls_z=int(walls), adjoint=1, **extra)
    p = oracle_params(sim)
    rho0 = droplet_rho(shape, T, walls=walls, radius=min(shape) / 3)
    g = np.random.Generator(np.random.PCG64(31))
    u0 = 0.03 * g.uniform(-1, 1, (3,) + shape)
    f0 = lbm.init(torch.tensor(rho0), p, torch.tensor(u0))
    f = f0 + torch.tensor(inputs.uniform_noise(tuple(f0.shape), 2e-4, 3)) * (f0 != 0)
    lam = torch.tensor(g.uniform(-1, 1, (27,) + shape))
    if walls:
        lam[:, 0] = 0
        lam[:, -1] = 0
    sim.set_populations(f)
    state = sim.get_state().clone()
    sim.adjoint_seed_populations(lam)
    sim.adjoint_step(state)
    lg = sim.adjoint_state().cpu()
    gg = sim.adjoint_grads()
    lo, ko, wo, no = _oracle_vjp(f, lam, p)
    sl = slice(1, -1) if walls else slice(None)
    e = rel_err(lg[:, sl], lo[:, sl])
    ek = abs(gg["kappa"] - ko) / max(abs(ko), 1e-300)
    en = abs(gg["nu"] - no) / max(abs(no), 1e-300)
    ew = abs(gg["wet_value"] - wo) / max(abs(wo), 1e-12) if walls and p.wet_mode else abs(gg["wet_value"] - wo)
    say(f"{label}: lambda err={e:.2e} dkappa={gg['kappa']:.6e}/{ko:.6e} ({ek:.1e}) "
        f"dnu={gg['nu']:.6e}/{no:.6e} ({en:.1e}) dwet={gg['wet_value']:.6e}/{wo:.6e} ({ew:.1e})")
    assert e < 1e-11
    assert ek < 1e-9 and en < 1e-9 and ew < 1e-9


def _loss_setup(shape, walls, wet_mode, wet_value, steps, wall_u=(0.0, 0.0, 0.0, 0.0)):
    T = eos.temperature(0.7)
    nz, ny, nx = shape
    rho0 = droplet_rho(shape, T, walls=walls, radius=min(shape) / 3, noise=1e-2, seed=9)
    rl, rv = eos.maxwell(eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"], T)
    tgt = rho0 + 1e-3 * (rl - rv) * inputs.uniform_noise(shape, 1.0, 12)
    cfg = lag.StepConfig(nx=nx, ny=ny, nz=nz, steps=steps, checkpoint_every=4, T=T, walls_z=int(walls),
                         wet_mode=wet_mode, wall_u=wall_u)
    return rho0, tgt, cfg


def _gpu_loss(rho0, tgt, cfg, kappa, wet, walls):
    sim = cfg.make(kappa, wet)
    sim.init_density(torch.tensor(rho0))
    sim.step(cfg.steps)
    r = sim.fields()["rho"].cpu()
    t = torch.tensor(tgt)
    sl = slice(1, -1) if walls else slice(None)
    return float(((r - t)[sl] ** 2).sum())


@pytest.mark.parametrize("walls,wet_mode,wet_value,wall_u", [
    (False, 0, 1.0, (0.0, 0.0, 0.0, 0.0)), (True, 1, 1.3, (0.0, 0.0, 0.0, 0.0)), (True, 2, 0.6, (0.0, 0.0, 0.0, 0.0)),
    (True, 1, 1.3, (0.06, -0.02, -0.04, 0.03))])
def test_end_to_end_gradients_vs_oracle_and_fd(walls, wet_mode, wet_value, wall_u):
    shape = (10, 8, 8) if walls else (8, 8, 8)
    steps = 12
    rho0, tgt, cfg = _loss_setup(shape, walls, wet_mode, wet_value, steps, wall_u)
    say(f"end-to-end walls={walls} mode={wet_mode} wall_u={wall_u}")
    # GPU adjoint through the autograd Function
    r0 = torch.tensor(rho0, device="cuda", requires_grad=True)
    kap = torch.tensor(0.02, dtype=DT, requires_grad=True)
    wet = torch.tensor(wet_value, dtype=DT, requires_grad=True)
    rT = lag.simulate(r0, kap, wet, cfg)
    sl = slice(1, -1) if walls else slice(None)
    loss = ((rT - torch.tensor(tgt, device="cuda"))[sl] ** 2).sum()
    loss.backward()
    g_r0 = r0.grad.cpu()
    # oracle reverse mode through init + steps + loss
    p = lbm.Params(shape[2], shape[1], shape[0], walls_z=walls, T=cfg.T, wet_mode=wet_mode, wall_u=wall_u)
    rl, rv = p.coexistence()
    ko = torch.tensor(0.02, dtype=DT, requires_grad=True)
    wo = torch.tensor(wet_value, dtype=DT, requires_grad=True)
    ro = torch.tensor(rho0, requires_grad=True)
    po = dataclasses.replace(p, kappa=ko, wet_value=wo, rho_l=rl, rho_v=rv)
    f = lbm.run(lbm.init(ro, po), po, steps)
    rho_T = lbm.aux_fields(f, po)["rho"]
    lo = ((rho_T - torch.tensor(tgt))[sl] ** 2).sum()
    lo.backward()
    fl = slice(1, -1) if walls else slice(None)
    e_r0 = rel_err(g_r0[fl], ro.grad[fl])
    e_k = abs(float(kap.grad) - float(ko.grad)) / abs(float(ko.grad))
    say(f"  dL/drho0 err={e_r0:.2e}  dL/dkappa gpu={float(kap.grad):.8e} oracle={float(ko.grad):.8e} ({e_k:.1e})")
    assert abs(float(loss.detach()) - float(lo)) < 1e-10 * float(lo)
    assert e_r0 < 1e-9 and e_k < 1e-9
    if walls and wet_mode:
        e_w = abs(float(wet.grad) - float(wo.grad)) / max(abs(float(wo.grad)), 1e-12)
        say(f"  dL/dwet gpu={float(wet.grad):.8e} oracle={float(wo.grad):.8e} ({e_w:.1e})")
        assert e_w < 1e-9
    # central finite differences of the GPU forward in FP64
    h = 1e-6
    fd_k = (_gpu_loss(rho0, tgt, cfg, 0.02 + h, wet_value, walls) -
            _gpu_loss(rho0, tgt, cfg, 0.02 - h, wet_value, walls)) / (2 * h)
    say(f"  FD dL/dkappa={fd_k:.8e}")
    assert abs(fd_k - float(kap.grad)) < 1e-5 * abs(fd_k)
    if walls and wet_mode:
        hw = 1e-6
        fd_w = (_gpu_loss(rho0, tgt, cfg, 0.02, wet_value + hw, walls) -
                _gpu_loss(rho0, tgt, cfg, 0.02, wet_value - hw, walls)) / (2 * hw)
        say(f"  FD dL/dwet={fd_w:.8e}")
        assert abs(fd_w - float(wet.grad)) < 1e-5 * max(abs(fd_w), 1e-8)
    g = np.random.Generator(np.random.PCG64(4))
    nodes = [tuple(int(v) for v in (g.integers(1 if walls else 0, shape[0] - (1 if walls else 0)),
                                    g.integers(0, shape[1]), g.integers(0, shape[2]))) for _ in range(4)]
    for nd in nodes:
        rp, rm = rho0.copy(), rho0.copy()
        rp[nd] += 1e-6
        rm[nd] -= 1e-6
        fd = (_gpu_loss(rp, tgt, cfg, 0.02, wet_value, walls) - _gpu_loss(rm, tgt, cfg, 0.02, wet_value, walls)) / 2e-6
        say(f"  FD dL/drho0{nd}={fd:.8e} adjoint={float(g_r0[nd]):.8e}")
        assert abs(fd - float(g_r0[nd])) < 1e-5 * max(abs(fd), 1e-6)


def test_gradients_come_back_on_the_input_devices():
    """rho0, kappa and the wetting value may live on the host or on the GPU:
    each gradient comes back on its input's device, with the same values."""
    shape = (10, 8, 8)
    rho0, tgt, cfg = _loss_setup(shape, True, 1, 1.3, 8)
    out = {}
    for dev in ("cpu", "cuda"):
        r0 = torch.tensor(rho0, device=dev, requires_grad=True)
        kap = torch.tensor(0.02, dtype=DT, device=dev, requires_grad=True)
        wet = torch.tensor(1.3, dtype=DT, device=dev, requires_grad=True)
        rT = lag.simulate(r0, kap, wet, cfg)
        ((rT - torch.tensor(tgt, device=rT.device)) ** 2).sum().backward()
        assert r0.grad.device.type == dev and kap.grad.device.type == dev and wet.grad.device.type == dev
        out[dev] = (r0.grad.cpu(), float(kap.grad), float(wet.grad))
    assert torch.equal(out["cpu"][0], out["cuda"][0]) and out["cpu"][1:] == out["cuda"][1:]


def test_checkpoint_interval_does_not_change_gradients():
    """Uniform checkpoints every 1, 4, 9 steps (with and without the kept
    forward fields) and the binomial schedule with zero, one and two
    snapshots give bitwise identical gradients."""
    shape = (10, 8, 8)
    rho0, tgt, cfg = _loss_setup(shape, True, 1, 1.3, 9)
    grads = []
    for K, mode, keep, snaps in ((1, "uniform", True, 0), (4, "uniform", True, 0), (4, "uniform", False, 0),
                                 (9, "uniform", True, 0), (9, "uniform", False, 0), (0, "binomial", False, 2),
                                 (0, "binomial", False, 1), (0, "binomial", False, 0)):
        cfg.checkpoint_every = max(K, 1)
        cfg.checkpoint, cfg.snapshots, cfg.keep_aux = mode, snaps, keep
        r0 = torch.tensor(rho0, device="cuda", requires_grad=True)
        kap = torch.tensor(0.02, dtype=DT, requires_grad=True)
        wet = torch.tensor(1.3, dtype=DT, requires_grad=True)
        rT = lag.simulate(r0, kap, wet, cfg)
        ((rT - torch.tensor(tgt, device="cuda"))[1:-1] ** 2).sum().backward()
        grads.append((r0.grad.cpu().clone(), float(kap.grad), float(wet.grad)))
    for g in grads[1:]:
        assert torch.equal(g[0], grads[0][0]) and g[1] == grads[0][1] and g[2] == grads[0][2]


def test_fp32_adjoint_close_to_fp64():
    shape = (12, 10, 10)
    T = eos.temperature(0.7)
    rho0 = droplet_rho(shape, T, walls=True, radius=4.0, noise=1e-2, seed=2)
    out = {}
    for prec in ("fp64", "fp32"):
        cfg = lag.StepConfig(nx=10, ny=10, nz=12, steps=20, checkpoint_every=5, T=T, walls_z=1, wet_mode=1,
                             precision=prec)
        r0 = torch.tensor(rho0, device="cuda", requires_grad=True)
        kap = torch.tensor(0.02, dtype=DT, requires_grad=True)
        wet = torch.tensor(1.3, dtype=DT, requires_grad=True)
        rT = lag.simulate(r0, kap, wet, cfg)
        (rT[1:-1] ** 2).sum().backward()
        out[prec] = (r0.grad.cpu(), float(kap.grad), float(wet.grad))
    e = rel_err(out["fp32"][0], out["fp64"][0])
    ek = abs(out["fp32"][1] - out["fp64"][1]) / abs(out["fp64"][1])
    ew = abs(out["fp32"][2] - out["fp64"][2]) / abs(out["fp64"][2])
    say(f"fp32 vs fp64 adjoint: drho0 {e:.2e} dkappa {ek:.2e} dwet {ew:.2e}")
    assert e < 1e-4 and ek < 1e-4 and ew < 1e-4


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_adjoint_step_with_kept_aux_is_bitwise_the_same(form):
    """lbfe_step_aux + lbfe_adjoint_step_aux against lbfe_step +
    lbfe_adjoint_step (recomputed fields) over 6 steps of a walled droplet:
    the same forward state, lambda and parameter gradients bit for bit."""
    shape = (10, 9, 11)
    T = eos.temperature(0.7)
    rho0 = droplet_rho(shape, T, walls=True, radius=3.5, noise=1e-2, seed=3)
    kw = dict(nx=11, ny=9, nz=10, T=T, walls_z=1, wet_mode=1, wet_value=1.3, precision=form, adjoint=1)
    a, b = make_sim(**kw), make_sim(**kw)
    states, recs = [], []
    for s in (a, b):
        s.init_density(torch.tensor(rho0))
    for _ in range(6):
        states.append(a.get_state().clone())
        a.step(1)
        recs.append(b.aux_record())
        b.step_aux(recs[-1])
    assert torch.equal(a.get_state(), b.get_state())
    g = torch.tensor(inputs.uniform_noise(shape, 1.0, 7), device="cuda")
    a.adjoint_seed(g)
    b.adjoint_seed(g)
    for t in range(5, -1, -1):
        a.adjoint_step(states[t])
        b.adjoint_step_aux(states[t], recs[t])
    assert torch.equal(a.adjoint_state().cpu(), b.adjoint_state().cpu())
    assert a.adjoint_grads() == b.adjoint_grads()
    bad = b.aux_record()
    with pytest.raises(lbfe.LBFEError) as e:
        b.adjoint_step_aux(states[0], bad[8:])
    assert e.value.code == lbfe.E_INVAL


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_adjoint_step_from_the_current_state(form):
    """lbfe_adjoint_step with a NULL state takes the context's current state:
    a sweep that sets each f(t) in the context and steps from it there ends
    with the lambda and gradients of a sweep over stored copies, bit for bit.
    Without a current state the call is refused."""
    shape = (10, 9, 11)
    T = eos.temperature(0.7)
    rho0 = droplet_rho(shape, T, walls=True, radius=3.5, noise=1e-2, seed=5)
    kw = dict(nx=11, ny=9, nz=10, T=T, walls_z=1, wet_mode=1, wet_value=1.3, precision=form, adjoint=1)
    a, b = make_sim(**kw), make_sim(**kw)
    for s in (a, b):
        s.init_density(torch.tensor(rho0))
    states = []
    for _ in range(5):
        states.append(a.get_state())
        a.step(1)
    g = torch.tensor(inputs.uniform_noise(shape, 1.0, 9), device="cuda")
    a.adjoint_seed(g)
    b.adjoint_seed(g)
    for t in range(4, -1, -1):
        a.adjoint_step(states[t])
        b.set_state(states[t], t)
        b.adjoint_step(None)
        assert torch.equal(b.get_state(), states[t])  # only read
    assert torch.equal(a.adjoint_state().cpu(), b.adjoint_state().cpu())
    assert a.adjoint_grads() == b.adjoint_grads()
    c = make_sim(**kw)
    c.adjoint_seed(g)
    with pytest.raises(lbfe.LBFEError) as e:
        c.adjoint_step(None)
    assert e.value.code == lbfe.E_STATE


@pytest.mark.parametrize("form", ["fp64", "fp32", "fp16dev"])
@pytest.mark.parametrize("shape", [(9, 8, 10), (6, 4, 67)])
def test_reading_lambda_mid_sweep_changes_nothing(form, shape):
    """lambda(t) is left without its last term between adjoint steps (the
    next step's gather adds it, taking the x +- 1 terms from the adjacent
    lanes); reading it out completes it in place.  A sweep interrupted by
    adjoint_state() after every step, and one restarted through the
    population seed, end bit for bit where an uninterrupted sweep does.
    The x extents put row ends inside waves and waves across rows and
    planes."""
    T = eos.temperature(0.7)
    rho0 = droplet_rho(shape, T, walls=True, radius=min(shape) / 3.0, noise=1e-2, seed=5)
    kw = dict(nx=shape[2], ny=shape[1], nz=shape[0], T=T, walls_z=1, wet_mode=2, wet_value=0.6, adjoint=1,
              precision=form)
    sims = [make_sim(**kw) for _ in range(3)]
    states = []
    for s in sims:
        s.init_density(torch.tensor(rho0))
    for _ in range(5):
        states.append(sims[0].get_state().clone())
        for s in sims:
            s.step(1)
    g = torch.tensor(inputs.uniform_noise(shape, 1.0, 11), device="cuda")
    for s in sims:
        s.adjoint_seed(g)
    mids = []
    lam3 = None
    for t in range(4, -1, -1):
        sims[0].adjoint_step(states[t])
        sims[1].adjoint_step(states[t])
        mids.append(sims[1].adjoint_state().clone())  # completes lambda(t) in place
        if t == 3:
            lam3 = mids[-1]
    # the third context starts at lambda(3) through the general seed
    sims[2].adjoint_seed_populations(lam3)
    for t in range(2, -1, -1):
        sims[2].adjoint_step(states[t])
    a, b, c = (s.adjoint_state().cpu() for s in sims)
    assert torch.equal(a, b) and torch.equal(a, c)
    assert torch.equal(mids[-1].cpu(), a)
    assert sims[0].adjoint_grads() == sims[1].adjoint_grads()


@pytest.mark.parametrize("walls", [False, True])
def test_dot_product_of_one_step(walls):
    """The adjoint of one step is the transpose of its derivative:
    <J v, w> = <v, J^T w> for random v, w, with J v by central differences
    of the GPU forward step (FP64, h = 1e-6) and J^T w by the adjoint step
    seeded with w.  The state sits away from the wetting window's edges, so
    the difference quotient sees one branch."""
    shape = (10, 9, 11)
    nz, ny, nx = shape
    T = eos.temperature(0.7 if walls else 0.85)
    kw = dict(nx=nx, ny=ny, nz=nz, T=T, adjoint=1)
    if walls:
        kw.update(walls_z=1, wet_mode=1, wet_value=1.3)
    sim = make_sim(**kw)
    rho0 = droplet_rho(shape, T, walls=walls, radius=3.5, noise=1e-3, seed=13)
    sim.init_density(torch.tensor(rho0))
    sim.step(3)
    f = sim.populations().cpu()
    g = np.random.Generator(np.random.PCG64(41))
    mask = (f != 0).double()
    v = torch.tensor(g.uniform(-1, 1, (27,) + shape)) * mask * 1e-3
    w = torch.tensor(g.uniform(-1, 1, (27,) + shape)) * mask
    h = 1e-3

    def step_of(ff):
        sim.set_populations(ff)
        sim.step(1)
        return sim.populations().cpu()

    Jv = (step_of(f + h * v) - step_of(f - h * v)) / (2 * h)
    sim.set_populations(f)
    state = sim.get_state().clone()
    sim.adjoint_seed_populations(w)
    sim.adjoint_step(state)
    JTw = sim.adjoint_state().cpu()
    a, b = float((Jv * w).sum()), float((v * JTw).sum())
    rel = abs(a - b) / abs(b)
    say(f"dot-product test walls={walls}: <Jv,w> = {a:.12e}, <v,J^T w> = {b:.12e}, rel {rel:.1e}")
    assert rel < 1e-8


FULL = [
    # (label, shape (nz, ny, nx), extra Simulation keywords, density builder)
    ("sessile 192x192x96", (96, 192, 192), dict(walls_z=1),
     lambda rl, rv: inputs.sessile_droplet(rl, rv)[0]),
    ("pillars mask 192x192x96", (96, 192, 192), dict(),
     lambda rl, rv: np.where(_pillars((96, 192, 192)).astype(bool), rv,
                             inputs.sphere((96, 192, 192), (96.0, 96.0, 8.0), 32.0, rl, rv))),
    ("moving walls 128^3", (128, 128, 128), dict(walls_z=1, wall_u=(0.1, 0.0, 0.1, 0.0)),
     lambda rl, rv: inputs.sphere((128, 128, 128), (64, 64, 64), 30.0, rl, rv)),
]


def _pillars(shape):
    return inputs.mask_pillars(shape, plate=2, pitch=12, width=4, height=6)


@pytest.mark.parametrize("label,shape,extra,rho_of", FULL, ids=[c[0] for c in FULL])
def test_dot_product_of_one_step_full_size(label, shape, extra, rho_of):
    """The dot-product test on full-size workloads of the benchmark (FP64,
    0.7 T_c, omega_3 = 1/2): the 192x192x96 sessile droplet between walls
    and the droplet on the pillared solid mask (72 tiles and six z-chunks of
    the transposed-stencil march), and the 128^3 droplet between moving
    walls.  Neutral wetting (no window of Eq. (38), so no branch for the
    difference quotient to straddle).  J v by central differences of the GPU
    forward step, J^T w by one adjoint step; every tensor stays on the
    device.  The rounding of the difference quotient, about
    1e-16 |f| / (h |v|) per term with random signs, keeps the relative gap
    near 1e-9 at any size; the bound is 1e-8 as for the small boxes."""
    nz, ny, nx = shape
    T = eos.temperature(0.7)
    kw = dict(extra)
    if label.startswith("pillars"):
        kw["solid"] = _pillars(shape)
    sim = make_sim(nx=nx, ny=ny, nz=nz, T=T, wet_mode=0, adjoint=1, omega=[1.0, 1.0, 1.0, 0.5] + [1.0] * 7, **kw)
    rl, rv = eos.maxwell(eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"], T)
    sim.init_density(torch.tensor(rho_of(rl, rv)))
    sim.step(20)
    f = sim.populations()
    gen = torch.Generator(device=f.device)
    gen.manual_seed(43)
    fluid = (f != 0).double()
    v = (torch.rand(f.shape, generator=gen, device=f.device, dtype=DT) * 2 - 1) * fluid * 1e-3
    w = (torch.rand(f.shape, generator=gen, device=f.device, dtype=DT) * 2 - 1) * fluid
    h = 1e-3

    def step_of(ff):
        sim.set_populations(ff)
        sim.step(1)
        return sim.populations()

    Jv = (step_of(f + h * v) - step_of(f - h * v)) / (2 * h)
    sim.set_populations(f)
    state = sim.get_state().clone()
    sim.adjoint_seed_populations(w)
    sim.adjoint_step(state)
    JTw = sim.adjoint_state()
    a, b = float((Jv * w).sum()), float((v * JTw).sum())
    rel = abs(a - b) / abs(b)
    say(f"full-size dot-product test {label}: <Jv,w> = {a:.12e}, <v,J^T w> = {b:.12e}, rel {rel:.1e}")
    assert rel < 1e-8
