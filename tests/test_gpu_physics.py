"""The paper's validation cases run on the GPU FP64 path (the oracle is too
slow for them): flat-interface coexistence, the fourth-order correction's
effect on stability, spurious currents, Young-Laplace, Galilean invariance
of a moving droplet, and contact angles of the wetting boundary."""
import math

import numpy as np
import pytest
import torch

from gpu_util import make_sim, say
from oracle import eos, phys
from paper_2504_03819_amd import inputs, lbfe

pytestmark = pytest.mark.gpu
A, B, R = eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"]
# omega_3 for runs with solid walls at 0.7 T_c: with all higher-order rates
# at 1 a halfway bounce-back wall next to the 0.7 T_c vapour is linearly
# unstable (x-odd tangential mode, spectral radius 1.19); omega_3 <= 0.5 is
# stable.  Static equilibria do not depend on any rate.
WALL_OMEGA = [1.0, 1.0, 1.0, 0.5] + [1.0] * 7


@pytest.mark.parametrize("tr,nu", [(0.7, 0.15), (0.7, 0.03), (0.8, 0.15), (0.9, 0.15)])
def test_flat_interface_coexistence(tr, nu):
    """Sec. III A: 4x4x128 periodic slab.  The LB steady state is a discrete
    equilibrium (mu uniform to 1e-10; a Newton solve of the discrete
    equilibrium started from it moves it by < 1e-7, the Newton system being
    nearly singular along the lattice-translation mode of the slab), its bulk
    densities match Maxwell's rule, and at 0.7 T_c the surface tension is
    0.204."""
    T = eos.temperature(tr)
    sim = make_sim(nx=4, ny=4, nz=128, T=T, nu=nu, check_every=5000)
    rho0 = inputs.flat_slab((128, 4, 4), sim.rho_l, sim.rho_v)
    sim.init_density(torch.tensor(rho0))
    sim.step(40000)
    f = sim.fields()
    rz = f["rho"][:, 0, 0].cpu().numpy()
    mu = f["mu"].cpu().numpy()
    r_newton, _ = phys.flat_equilibrium(rz, A, B, R, T, 0.02)
    rl, rv = eos.maxwell(A, B, R, T)
    sig = phys.surface_tension(np.roll(rz, 32 - int(np.argmax(np.abs(np.gradient(rz))[:64]))), 0.02)
    say(f"flat Tr={tr} nu={nu}: rho_l={rz.max():.6f} (Maxwell {rl:.6f}) rho_v={rz.min():.6f} (Maxwell {rv:.6f}) "
        f"mu spread={mu.max() - mu.min():.2e} |LB-Newton|={np.abs(rz - r_newton).max():.2e} sigma={sig:.5f}")
    assert mu.max() - mu.min() < 1e-10
    assert np.abs(rz - r_newton).max() < 1e-7
    assert abs(rz.max() - rl) < 1e-4 * rl and abs(rz.min() - rv) < 1e-4 * rv
    if tr == 0.7:
        assert round(sig, 3) == 0.204


def test_fourth_order_correction_needed_for_curved_interface():
    """Sec. III B: 128^3 droplet r = 30 at 0.7 T_c.  Without Eq. (28) the run
    blows up within the first hundred steps (the paper reports divergence
    shortly after t = 86); with it the initial flow decays."""
    T = eos.temperature(0.7)
    rho0 = inputs.sphere((128,) * 3, (64, 64, 64), 30.0, *eos.maxwell(A, B, R, T))
    sim = make_sim(nx=128, ny=128, nz=128, T=T, corr4=0, check_every=1)
    sim.init_density(torch.tensor(rho0))
    with pytest.raises(lbfe.LBFEError) as ei:
        sim.step(300)
    assert ei.value.code == lbfe.E_DIVERGED
    t_div = sim.step_count
    sim = make_sim(nx=128, ny=128, nz=128, T=T, corr4=1, check_every=100)
    sim.init_density(torch.tensor(rho0))
    sim.step(100)
    u100 = sim.reduce()[7]
    sim.step(1400)
    u1500 = sim.reduce()[7]
    say(f"corr4 off: diverged at step {t_div}; corr4 on: max|u| t=100 {u100:.3e}, t=1500 {u1500:.3e}")
    assert t_div < 200 and u1500 < 0.2 * u100


def test_spurious_velocity_after_1e5_steps():
    """Sec. III B: with the correction the maximum spurious velocity of the
    128^3, r = 30, 0.7 T_c droplet is about 2.4e-11 at t = 100 000."""
    T = eos.temperature(0.7)
    sim = make_sim(nx=128, ny=128, nz=128, T=T, check_every=10000)
    sim.init_density(torch.tensor(inputs.sphere((128,) * 3, (64, 64, 64), 30.0, sim.rho_l, sim.rho_v)))
    sim.step(100000)
    umax = sim.reduce()[7]
    say(f"spurious max|u| at t=1e5: {umax:.3e} (paper 2.4e-11)")
    assert umax < 1e-10


def test_young_laplace():
    """Sec. III B, Fig. 4: droplets at 0.7 T_c reach a state of uniform mu with
    bulk densities on the same chemical-potential isoline; the pressure jump
    p0(in) - p0(out) follows 2 sigma / R (sigma of the flat interface, R the
    equimolar radius) to within 10 %, and Delta p R is the same for both radii
    to within 2 %."""
    T = eos.temperature(0.7)
    sig = 0.20422169457183298
    dpR = []
    for r0 in (16.0, 24.0):
        n = 96
        sim = make_sim(nx=n, ny=n, nz=n, T=T, check_every=10000)
        sim.init_density(torch.tensor(inputs.sphere((n,) * 3, (n / 2,) * 3, r0, sim.rho_l, sim.rho_v)))
        sim.step(40000)
        f = sim.fields()
        rho, mu = f["rho"].cpu().numpy(), f["mu"].cpu().numpy()
        rin, rout = float(rho[n // 2, n // 2, n // 2]), float(rho[0, 0, 0])
        Re = phys.equimolar_radius(rho, rin, rout)
        dp = eos.p0(rin, A, B, R, T) - eos.p0(rout, A, B, R, T)
        dmu = abs(eos.mu0(rin, A, B, R, T) - eos.mu0(rout, A, B, R, T))
        say(f"Laplace r0={r0}: R_e={Re:.3f} rho_in={rin:.6f} rho_out={rout:.6f} dp={dp:.6e} 2sigma/R={2 * sig / Re:.6e} "
            f"ratio={dp * Re / (2 * sig):.4f} |mu0(in)-mu0(out)|={dmu:.1e} mu spread={mu.max() - mu.min():.1e}")
        assert mu.max() - mu.min() < 1e-5
        assert dmu < 1e-6
        assert abs(dp * Re / (2 * sig) - 1) < 0.10
        dpR.append(dp * Re)
    assert abs(dpR[0] / dpR[1] - 1) < 0.02


def _com(ind):
    out = []
    for ax in (2, 1, 0):
        n = ind.shape[ax]
        prof = ind.sum(axis=tuple(a for a in range(3) if a != ax))
        c = (prof * np.exp(2j * np.pi * np.arange(n) / n)).sum()
        out.append((np.angle(c) % (2 * np.pi)) * n / (2 * np.pi))
    return np.array(out)


def _fshift(a, d):
    F = np.fft.fftn(a)
    kz, ky, kx = [np.fft.fftfreq(n) for n in a.shape]
    ph = np.exp(-2j * np.pi * (kx[None, None, :] * d[0] + ky[None, :, None] * d[1] + kz[:, None, None] * d[2]))
    return np.real(np.fft.ifftn(F * ph))


def _shape_ratio(ind):
    n = ind.shape[0]
    c = _com(ind)
    z, y, x = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")
    X = [((x - c[0] + n / 2) % n) - n / 2, ((y - c[1] + n / 2) % n) - n / 2, ((z - c[2] + n / 2) % n) - n / 2]
    I = np.array([[np.sum(ind * X[a] * X[b]) for b in range(3)] for a in range(3)])
    ev = np.sort(np.linalg.eigvalsh(I))
    return ev[-1] / ev[0]


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_galilean_invariance_moving_droplet(form):
    """Moving droplet, 128^3, 0.85 T_c, r = 24, u0 = (0.05, 0.02, 0), 10 000
    steps, against the same droplet at rest: after undoing the measured
    centre-of-mass displacement the density fields agree to an L2 error of
    2e-3 (rho_l - rho_v), the droplet keeps its shape (principal-moment ratio
    within 2e-4 of the rest droplet's) and its equimolar radius."""
    T = eos.temperature(0.85)
    out = {}
    for moving in (True, False):
        sim = make_sim(nx=128, ny=128, nz=128, T=T, precision=form, check_every=5000)
        vel = (0.05, 0.02, 0.0) if moving else (0.0, 0.0, 0.0)
        rho0, u0 = inputs.moving_droplet(sim.rho_l, sim.rho_v, velocity=vel)
        sim.init_density(torch.tensor(rho0), torch.tensor(u0))
        sim.step(10000)
        rho = sim.fields()["rho"].cpu().numpy()
        dl = sim.rho_l - sim.rho_v
        out[moving] = (rho, _com((rho - sim.rho_v) / dl))
    (rm, cm), (rr, cr) = out[True], out[False]
    back = _fshift(rm, -(cm - cr))
    l2 = float(np.sqrt(((back - rr) ** 2).mean()) / dl)
    im, ir = np.clip((back - sim.rho_v) / dl, 0, 1), np.clip((rr - sim.rho_v) / dl, 0, 1)
    sm, sr = _shape_ratio(im), _shape_ratio(ir)
    Rm, Rr = (3 * im.sum() / (4 * math.pi)) ** (1 / 3), (3 * ir.sum() / (4 * math.pi)) ** (1 / 3)
    disp = (cm - cr) % 128
    say(f"galilean {form}: COM displacement mod 128 = {disp} (u0 t mod 128 = [116, 72, 0]); "
        f"L2 after shift {l2:.2e}; shape ratio moving {sm:.6f} rest {sr:.6f}; R_e {Rm:.4f} / {Rr:.4f}")
    assert l2 < 2e-3
    assert abs(sm - sr) < 2e-4
    assert abs(Rm - Rr) < 1e-2


def test_moving_walls_droplet_keeps_its_shape():
    """The moving-wall droplet of Sec. III B: the stationary-droplet setup
    (128^3, r = 30) with the top and bottom planes as walls moving at
    U = 0.1 along x, here at 0.8 T_c (at 0.7 T_c the vapour next to the
    moving walls goes unstable after about 6e4 steps in this reading).  The
    induced flow carries the droplet; over 1e5 steps it stays round (largest
    to smallest principal moment within 3 %), keeps its mass and moves at
    more than half the wall speed."""
    n = 128
    T = eos.temperature(0.8)
    sim = make_sim(nx=n, ny=n, nz=n, T=T, walls_z=1, wall_u=(0.1, 0.0, 0.1, 0.0), check_every=5000)
    rl, rv = sim.rho_l, sim.rho_v
    sim.init_density(torch.tensor(inputs.sphere((n, n, n), (n / 2, n / 2, n / 2), 30.0, rl, rv)))
    m0 = sim.reduce()[0]
    sim.step(100000)
    f = sim.fields()
    rho, u = f["rho"].cpu().numpy(), f["u"].cpu().numpy()
    ind = np.clip((rho - rv) / (rl - rv), 0, 1)
    ind[0] = ind[-1] = 0
    ratio = _shape_ratio(ind)
    ud = float((ind * u[0]).sum() / ind.sum())
    drift = abs(sim.reduce()[0] - m0) / m0
    say(f"moving walls 0.8Tc t=1e5: shape ratio {ratio:.5f}, droplet u_x {ud:.4f}, mass drift {drift:.1e}")
    assert ratio < 1.03
    assert ud > 0.05
    assert drift < 1e-10


P15_NOT_REPRODUCED = ("the wetting reading here (window and limiter of Eq. (38) on the contact-line nodes only, the "
                      "solid density in the isotropic Laplacian) gives {}; the paper prints {}")


@pytest.mark.parametrize("label,mode,value,paper,steps", [
    ("neutral", lbfe.WET_PHI, 1.0, 89.9, 20000),
    pytest.param("phi 1.6", lbfe.WET_PHI, 1.6, 33.5, 30000, marks=pytest.mark.xfail(
        strict=True, reason=P15_NOT_REPRODUCED.format("30.3 deg (cap radius 95, measurement robust to the fit's "
                                                      "cut-off height)", "33.5 deg"))),
    pytest.param("drho 1.8", lbfe.WET_DELTA, 1.8, 153.4, 10000, marks=pytest.mark.xfail(
        strict=True, reason=P15_NOT_REPRODUCED.format("no attached state: the droplet leaves the wall within 2000 "
                                                      "steps and evaporates", "153.4 deg"))),
])
def test_contact_angle_paper_geometry(label, mode, value, paper, steps):
    """Sec. III C on the paper's geometry: Nx x Ny x Nz = 128 x 256 x 256,
    solid planes z = 0 and 255, a droplet of radius 30 centred on the wall
    plane, 0.7 T_c (omega_3 = 1/2, the wall reading of the oracle), FP32
    storage (angles agree with FP64 to 1e-3 deg).  The printed angles within
    2 deg, mu uniform over the fluid."""
    from oracle import phys as ph
    T = eos.temperature(0.7)
    nx, ny, nz = 128, 256, 256
    sim = make_sim(nx=nx, ny=ny, nz=nz, T=T, walls_z=1, wet_mode=mode, wet_value=value, omega=WALL_OMEGA,
                   precision="fp32", check_every=5000)
    rho0 = inputs.sphere((nz, ny, nx), (nx / 2, ny / 2, 0.5), 30.0, sim.rho_l, sim.rho_v)
    rho0[0] = rho0[-1] = sim.rho_v
    sim.init_density(torch.tensor(rho0))
    sim.step(steps)
    f = sim.fields()
    rho, mu = f["rho"].cpu().numpy(), f["mu"].cpu().numpy()[1:-1]
    th, zc, Rf = ph.contact_angle(rho, sim.rho_l, sim.rho_v)
    say(f"contact angle {label}: theta={th:.2f} deg (paper {paper}), cap radius {Rf:.1f}, "
        f"mu spread {mu.max() - mu.min():.1e}")
    assert abs(th - paper) <= 2.0
    assert mu.max() - mu.min() < 2e-3


@pytest.mark.parametrize("mode,value,lo,hi", [
    (lbfe.WET_PHI, 1.3, 55.0, 61.0),
    (lbfe.WET_DELTA, 0.9, 116.0, 123.0),
])
def test_contact_angle_calibration(mode, value, lo, hi):
    """Calibration points of the wetting workload (192x192x96, radius 32,
    0.7 T_c; no printed values in the paper: these angles were measured
    here and are kept as regression windows for the target angles 60 and
    120 deg)."""
    from oracle import phys as ph
    T = eos.temperature(0.7)
    sim = make_sim(nx=192, ny=192, nz=96, T=T, walls_z=1, wet_mode=mode, wet_value=value, omega=WALL_OMEGA,
                   check_every=5000)
    rho0, _ = inputs.sessile_droplet(sim.rho_l, sim.rho_v)
    sim.init_density(torch.tensor(rho0))
    sim.step(20000)
    f = sim.fields()
    rho, mu = f["rho"].cpu().numpy(), f["mu"].cpu().numpy()[1:-1]
    th, zc, Rf = ph.contact_angle(rho, sim.rho_l, sim.rho_v)
    say(f"contact angle mode={mode} value={value}: theta={th:.2f} deg (cap radius {Rf:.1f}), "
        f"mu spread {mu.max() - mu.min():.1e}")
    assert lo <= th <= hi
    assert mu.max() - mu.min() < 1e-3


@pytest.mark.parametrize("label,mode,value", [("hydrophobic", lbfe.WET_DELTA, 0.9), ("hydrophilic", lbfe.WET_PHI, 1.6)])
def test_droplet_on_pillars_cassie_or_wenzel(label, mode, value):
    """The wetting boundary on a patterned substrate (solid mask: plate of 2
    layers, 4 x 4 x 8 pillars at pitch 12, 96 x 96 x 48 box, 0.8 T_c): a
    droplet (r = 18) placed on the pillar tops stays suspended over vapour
    on a hydrophobic substrate (drho = 0.9, Cassie state) and fills the gaps
    between the pillars on a hydrophilic one (phi = 1.6, Wenzel state);
    the fluid mass is conserved either way."""
    shape = (48, 96, 96)
    plate, height = 2, 8
    top = plate + height
    mask = inputs.mask_pillars(shape, plate=plate, pitch=12, width=4, height=height)
    T = eos.temperature(0.8)
    sim = make_sim(nx=96, ny=96, nz=48, T=T, wet_mode=mode, wet_value=value, omega=WALL_OMEGA, solid=mask,
                   check_every=2000)
    rl, rv = sim.rho_l, sim.rho_v
    rho = inputs.sphere(shape, (48.0, 48.0, top + 17.0), 18.0, rl, rv)
    rho[mask.astype(bool)] = rv
    sim.init_density(torch.tensor(rho))
    m0 = sim.reduce()[0]
    sim.step(10000)
    r = sim.fields()["rho"].cpu().numpy()
    fluid = mask == 0
    gap = np.zeros(shape, bool)
    gap[plate:top, 36:60, 36:60] = True  # the texture below the droplet
    gap &= fluid
    liq = (r > 0.5 * (rl + rv)) & fluid
    frac = float((liq & gap).sum() / gap.sum())
    zc = float((np.arange(48)[:, None, None] * liq).sum() / liq.sum())
    drift = abs(sim.reduce()[0] - m0) / m0
    say(f"pillars {label}: liquid fraction of the gaps {frac:.3f}, liquid centre z {zc:.2f} (pillar tops {top}), "
        f"mass drift {drift:.1e}")
    if label == "hydrophobic":
        assert frac < 0.01 and zc > top + 14
    else:
        assert frac > 0.2 and zc < top + 8
    assert drift < 1e-10


def test_lb_droplet_converges_to_the_newton_equilibrium():
    """Pin P11: a 16^3 droplet at 0.7 T_c (tanh, radius 5) stepped by the
    GPU FP64 path relaxes to the discrete static equilibrium that Newton's
    method finds for the same mass (oracle.phys.static_equilibrium_3d):
    after 4e4 steps the density fields agree to 1e-8 of rho_l - rho_v and
    the velocity has decayed to rounding."""
    from oracle import phys as ph
    n = 16
    T = eos.temperature(0.7)
    sim = make_sim(nx=n, ny=n, nz=n, T=T, check_every=10000)
    rl, rv = sim.rho_l, sim.rho_v
    rho0 = ph.tanh_droplet((n, n, n), (n / 2, n / 2, n / 2), 5.0, rl, rv)
    r_newton, mu_star = ph.static_equilibrium_3d(rho0, eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"], T, 0.02)
    sim.init_density(torch.tensor(rho0))
    errs = []
    for _ in range(2):
        sim.step(20000)
        f = sim.fields()
        e = float(np.abs(f["rho"].cpu().numpy() - r_newton).max()) / (rl - rv)
        errs.append(e)
    umax = float(f["u"].abs().max())
    say(f"LB vs Newton droplet 16^3: rho err every 2e4 steps {['%.1e' % v for v in errs]}, max|u| {umax:.1e}, "
        f"mu - mu* {float((f['mu'] - mu_star).abs().max()):.1e}")
    # (measured: 6.6e-12 at 2e4 and 4e4 steps; beyond 5e4 steps a slow mode
    # of this small box grows from rounding, 1.9e-10 at 6e4 and 5e-4 at 1e5)
    assert errs[-1] < 1e-8
    assert umax < 1e-10
