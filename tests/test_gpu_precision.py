"""Reduced-precision storage forms against the GPU FP64 path (itself at
parity with the oracle): FP32 populations, FP16 deviations with the rest
population in FP32, and all-FP16 deviations.  Errors are stated per result:
density profile, mass drift, Laplace pressure and contact angle."""
import numpy as np
import pytest
import torch

from gpu_util import make_sim, sampled_windows, say
from oracle import eos
from paper_2504_03819_amd import inputs, lbfe

pytestmark = pytest.mark.gpu
A, B, R = eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"]
FORMS = ["fp32", "fp16dev_f0fp32", "fp16dev"]
# stated tolerances: (per-step rho, 100-step rho, mass drift / 1000 steps,
# Laplace pressure (relative), contact angle (degrees))
TOL = {"fp32": (1e-6, 1e-5, 1e-6, 1e-3, 0.1),
       "fp16dev_f0fp32": (1e-4, 1e-3, 1e-4, 1e-3, 0.1),
       "fp16dev": (2e-3, 1e-2, None, None, None)}
# All-FP16: the rest population carries the whole density contrast (f0 - w0
# reaches +6.5 in the liquid), so its half-precision rounding, repeated the
# same way at a steady node every step, drifts the mass by ~6 % per 1000
# steps and long runs leave the EOS domain.  Only the short-run density
# error is stated for it; the f0-in-FP32 variant is the usable FP16 form.
NO_LONG_RUNS = "all-FP16 storage drifts mass ~6%/1000 steps and diverges in long runs (see the short-run test)"


def _droplet(n, tr, r):
    T = eos.temperature(tr)
    rl, rv = eos.maxwell(A, B, R, T)
    return T, rl, rv, inputs.sphere((n,) * 3, (n / 2,) * 3, r, rl, rv) + inputs.uniform_noise((n,) * 3, 1e-3, 3)


@pytest.mark.parametrize("form", FORMS)
def test_density_error_and_mass_drift(form):
    n = 48
    T, rl, rv, rho0 = _droplet(n, 0.7, 12.0)
    ref = make_sim(nx=n, ny=n, nz=n, T=T)
    ref.init_density(torch.tensor(rho0))
    ref.step(50)
    f50 = ref.populations()
    sim = make_sim(nx=n, ny=n, nz=n, T=T, precision=form)
    sim.set_populations(f50)
    m0 = sim.reduce()[0]
    # one step from the same state (the reduced form starts from its own
    # encoding of it, so the error includes the storage rounding)
    ref.step(1)
    sim.step(1)
    e1 = float((sim.fields()["rho"] - ref.fields()["rho"]).abs().max()) / (rl - rv)
    ref.step(99)
    sim.step(99)
    e100 = float((sim.fields()["rho"] - ref.fields()["rho"]).abs().max()) / (rl - rv)
    sim.step(900)
    drift = abs(sim.reduce()[0] - m0) / m0
    say(f"{form}: rho error after 1 step {e1:.2e}, after 100 steps {e100:.2e} (x (rho_l - rho_v)); "
        f"relative mass drift over 1000 steps {drift:.2e}")
    t1, t100, tm, _, _ = TOL[form]
    assert e1 < t1 and e100 < t100
    if tm is not None:
        assert drift < tm


@pytest.mark.parametrize("form", FORMS)
def test_laplace_pressure_error(form):
    if TOL[form][3] is None:
        pytest.skip(NO_LONG_RUNS)
    n = 96
    T = eos.temperature(0.7)
    out = {}
    for f in ("fp64", form):
        sim = make_sim(nx=n, ny=n, nz=n, T=T, precision=f, check_every=10000)
        sim.init_density(torch.tensor(inputs.sphere((n,) * 3, (n / 2,) * 3, 24.0, sim.rho_l, sim.rho_v)))
        sim.step(30000)
        rho = sim.fields()["rho"].cpu().numpy()
        rin, rout = rho[n // 2, n // 2, n // 2], rho[0, 0, 0]
        out[f] = eos.p0(rin, A, B, R, T) - eos.p0(rout, A, B, R, T)
    err = abs(out[form] - out["fp64"]) / abs(out["fp64"])
    say(f"{form}: Laplace pressure {out[form]:.6e} vs FP64 {out['fp64']:.6e}: relative error {err:.2e}")
    assert err < TOL[form][3]


@pytest.mark.parametrize("form", FORMS)
def test_contact_angle_error(form):
    if TOL[form][4] is None:
        pytest.skip(NO_LONG_RUNS)
    from oracle import phys
    T = eos.temperature(0.7)
    om = [1.0, 1.0, 1.0, 0.5] + [1.0] * 7
    th = {}
    for f in ("fp64", form):
        sim = make_sim(nx=192, ny=192, nz=96, T=T, walls_z=1, wet_mode=lbfe.WET_PHI, wet_value=1.3, omega=om,
                       precision=f, check_every=5000)
        rho0, _ = inputs.sessile_droplet(sim.rho_l, sim.rho_v)
        sim.init_density(torch.tensor(rho0))
        sim.step(20000)
        th[f] = phys.contact_angle(sim.fields()["rho"].cpu().numpy(), sim.rho_l, sim.rho_v)[0]
    say(f"{form}: contact angle {th[form]:.3f} vs FP64 {th['fp64']:.3f} deg")
    assert abs(th[form] - th["fp64"]) < TOL[form][4]


# one step of an FP16 state: the GPU's FP32 arithmetic and half rounding of
# the result against the FP64 oracle stepping the same decoded state
# (normwise, max |error| / max |f|): the rounding of the stored deviations
# bounds it, a half ulp of h = f/w - 1 times w per population; with f0 in
# FP32 that is a few 1e-7 of max f, with f0 in half up to 2^-12 h0 w0 / f0 =
# 3.7e-4 at the 0.85 T_c liquid
ONE_STEP_TOL = {"fp16dev_f0fp32": 2e-6, "fp16dev": 1e-3}


@pytest.mark.parametrize("form", ["fp16dev_f0fp32", "fp16dev"])
def test_fp16_one_step_against_the_oracle(form):
    from gpu_util import oracle_params, rel_err
    from oracle import lbm
    T, rl, rv, rho0 = _droplet(24, 0.85, 7.0)
    sim = make_sim(nx=24, ny=24, nz=24, T=T, precision=form)
    sim.init_density(torch.tensor(rho0))
    sim.step(10)
    f_t = sim.populations().cpu()  # the decoded stored state
    sim.step(1)
    e = rel_err(sim.populations().cpu(), lbm.step(f_t, oracle_params(sim)))
    say(f"{form}: one step vs oracle {e:.2e}")
    assert e < ONE_STEP_TOL[form]


@pytest.mark.parametrize("form", ["fp16dev_f0fp32", "fp16dev"])
def test_fp16_full_size_spinodal_sampled(form):
    """The 256^3 spinodal workload in the FP16 forms, 20 steps in: sampled
    windows of the decoded state stepped by the FP64 oracle."""
    n = 256
    T = eos.temperature(0.8)
    sim = make_sim(nx=n, ny=n, nz=n, T=T, precision=form, check_every=1000)
    rho0, _ = inputs.spinodal(sim.rho_l, sim.rho_v)
    sim.init_density(torch.tensor(rho0))
    sim.step(20)
    f_t = sim.populations()
    sim.step(1)
    f_t1 = sim.populations()
    g = np.random.Generator(np.random.PCG64(16))
    centres = [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(5)] + [(0, 0, 0)]
    sampled_windows(sim, f_t, f_t1, centres, ONE_STEP_TOL[form], f"256^3 spinodal {form}")
