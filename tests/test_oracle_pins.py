"""Pins of the FP64 oracle against what the paper and mathematics fix
(closed forms, printed values, invariants, brute force, symmetry).  CPU only."""
import json
import math
import os
from fractions import Fraction
from itertools import product

import numpy as np
import pytest
import torch

from oracle import eos, lbm, phase_space as ps, phys
from oracle.lattice import C, OPP, REST, W_EXACT, W_T

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
A, B, R = eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"]
DT = torch.float64


def rng(seed):
    return torch.Generator().manual_seed(seed)


# ---------------------------------------------------------------- closure ---
def test_critical_point_exact():
    """Eq. (30) with a = 9/392, b = 2/21, R = 1 gives rho_c = 7/2, T_c = 1/14,
    p_c = 3/32 exactly (printed in Sec. III)."""
    a, b = Fraction(9, 392), Fraction(2, 21)
    assert 1 / (3 * b) == Fraction(7, 2)
    assert 8 * a / (27 * b) == Fraction(1, 14)
    assert a / (27 * b * b) == Fraction(3, 32)
    rc, tc, pc = eos.critical_point(A, B, R)
    assert abs(rc - 3.5) < 1e-14 and abs(tc - 1 / 14) < 1e-15 and abs(pc - 3 / 32) < 1e-15
    # the inflection conditions that define the critical point
    h = 1e-4
    d1 = (eos.p0(rc + h, A, B, R, tc) - eos.p0(rc - h, A, B, R, tc)) / (2 * h)
    d2 = (eos.p0(rc + h, A, B, R, tc) - 2 * eos.p0(rc, A, B, R, tc) + eos.p0(rc - h, A, B, R, tc)) / h ** 2
    assert abs(d1) < 1e-9 and abs(d2) < 1e-5


def test_maxwell_printed_values_and_equal_area():
    """Coexistence at 0.7 Tc matches the printed 7.49 / 0.448 / 16.7, and the
    pair satisfies the equal-area rule in the p-v plane, checked by
    quadrature (independent of the Newton formulation)."""
    from scipy.integrate import quad
    g = GOLD["coexistence_07Tc"]
    T = eos.temperature(0.7)
    rl, rv = eos.maxwell(A, B, R, T)
    assert round(rl, 2) == g["rho_l"] and round(rv, 3) == g["rho_v"] and round(rl / rv, 1) == g["ratio"]
    for tr in (0.7, 0.8, 0.85, 0.9):
        T = eos.temperature(tr)
        rl, rv = eos.maxwell(A, B, R, T)
        psat = eos.p0(rl, A, B, R, T)
        vl, vv = 1 / rl, 1 / rv
        area, _ = quad(lambda v: eos.p0(1 / v, A, B, R, T), vl, vv, epsabs=1e-13, epsrel=1e-13)
        assert abs(area - psat * (vv - vl)) < 1e-9 * psat * (vv - vl)


def test_mu0_is_derivative_of_psi():
    T = eos.temperature(0.8)
    for r in (0.5, 2.0, 3.5, 6.0, 8.0):
        h = 1e-6
        num = (eos.psi(r + h, A, B, R, T) - eos.psi(r - h, A, B, R, T)) / (2 * h)
        assert abs(num - eos.mu0(r, A, B, R, T)) < 1e-8
        # Eq. (4): p0 = rho mu0 - psi
        assert abs(r * eos.mu0(r, A, B, R, T) - eos.psi(r, A, B, R, T) - eos.p0(r, A, B, R, T)) < 1e-13
    # the torch closure used inside the step agrees with the scalar one
    p = lbm.Params(2, 2, 2, T=T)
    rr = torch.tensor([0.5, 2.0, 6.0], dtype=DT)
    for x, y in zip(lbm.mu_bulk(rr, p), (0.5, 2.0, 6.0)):
        assert abs(float(x) - eos.mu0(y, A, B, R, T)) < 1e-15


# ---------------------------------------------------------------- lattice ---
def test_lattice_isotropy_exact():
    """Eq. (17) weights: normalisation, second- and fourth-order isotropy with
    c_s^2 = 1/3, and the sixth-order moment 1/27 (tensor-product lattice)."""
    assert sum(W_EXACT) == 1
    cs2 = Fraction(1, 3)
    d = lambda a, b: 1 if a == b else 0
    for a, b in product(range(3), repeat=2):
        assert sum(w * c[a] * c[b] for w, c in zip(W_EXACT, C)) == cs2 * d(a, b)
        assert sum(w * c[a] for w, c in zip(W_EXACT, C)) == 0
    for a, b, g, h in product(range(3), repeat=4):
        s = sum(w * c[a] * c[b] * c[g] * c[h] for w, c in zip(W_EXACT, C))
        assert s == cs2 ** 2 * (d(a, b) * d(g, h) + d(a, g) * d(b, h) + d(a, h) * d(b, g))
    assert sum(w * c[0] ** 2 * c[1] ** 2 * c[2] ** 2 for w, c in zip(W_EXACT, C)) == Fraction(1, 27)
    assert C[REST] == (0, 0, 0) and all(C[OPP[i]] == tuple(-x for x in C[i]) for i in range(27))


def test_stencil_symbols_closed_form():
    """grad_h and lap_h applied to a plane wave reproduce the closed-form
    symbols of the isotropic D3Q27 stencils (product of 1-D factors)."""
    n = (6, 8, 10)  # nz, ny, nx
    z, y, x = torch.meshgrid(*[torch.arange(k, dtype=DT) for k in n], indexing="ij")
    kx, ky, kz = 2 * math.pi * 3 / 10, 2 * math.pi * 1 / 8, 2 * math.pi * 2 / 6
    ph = kx * x + ky * y + kz * z
    g = torch.cos(ph)
    fx, fy, fz = (2 + math.cos(kx)) / 3, (2 + math.cos(ky)) / 3, (2 + math.cos(kz)) / 3
    G = lbm.grad_h(g)
    exp = [-math.sin(kx) * fy * fz, -math.sin(ky) * fx * fz, -math.sin(kz) * fx * fy]
    for a in range(3):
        assert torch.allclose(G[a], exp[a] * torch.sin(ph), atol=1e-13)
    L = lbm.lap_h(g)
    assert torch.allclose(L, 6 * (fx * fy * fz - 1) * g, atol=1e-13)


# ------------------------------------------------------- moment transforms ---
def test_central_moments_match_definition_and_invert():
    """CMs through raw moments (Sec. II B) equal the literal Eq. (19) sum;
    the inverse route recovers f (invertibility)."""
    g = rng(2)
    f = torch.rand((27, 50), generator=g, dtype=DT)
    u = 0.4 * (torch.rand((3, 50), generator=g, dtype=DT) - 0.5)
    k = lbm.central_moments(f, u)
    kd = lbm.central_moments_direct(f, u)
    assert (k - kd).abs().max() < 1e-14 * kd.abs().max()
    f2 = lbm.populations_from_central(k, u)
    assert (f2 - f).abs().max() < 1e-14
    # at u = 0 central moments are raw moments
    assert torch.allclose(lbm.central_moments(f, 0 * u), lbm.raw_moments(f), atol=1e-15)


def test_phase_space_equilibrium_has_eq20_moments():
    """Eqs. (13)-(16) (tensor-product Hermite reading) have exactly the
    equilibrium CMs of Eq. (20); the oracle's initial populations (inverse CM
    of Eq. (20)) equal the phase-space f^eq."""
    g = rng(3)
    n = 200
    rho = 0.3 + 7 * torch.rand(n, generator=g, dtype=DT)
    u = 0.4 * (torch.rand((3, n), generator=g, dtype=DT) - 0.5)
    pm = 0.3 + 0.1 * torch.rand(n, generator=g, dtype=DT)
    feq = ps.f_eq(rho, u, pm)
    k = lbm.central_moments_direct(feq, u)
    keq = lbm.equilibrium_central(rho, pm)
    assert (k - keq).abs().max() < 1e-13
    assert (lbm.populations_from_central(keq, u) - feq).abs().max() < 1e-13


def test_isotropic_operator_closed_form():
    """Eq. (16) evaluates to E_i = 3 (w_i - delta_i,rest); so at u = 0,
    f^eq = (1 + mu) w_i + (rho - 1 - mu) delta_i,rest with p_m = (1 + mu)/3."""
    E = ps.E_iso(torch.zeros(()))
    exp = 3 * (W_T - torch.tensor([1.0 if i == REST else 0.0 for i in range(27)], dtype=DT))
    assert (E - exp).abs().max() < 1e-14
    rho, mu = torch.tensor(4.2, dtype=DT), torch.tensor(0.03, dtype=DT)
    feq = ps.f_eq(rho, torch.zeros(3, dtype=DT), (1 + mu) / 3)
    exp = (1 + mu) * W_T + (rho - 1 - mu) * torch.tensor([1.0 if i == REST else 0 for i in range(27)], dtype=DT)
    assert (feq - exp).abs().max() < 1e-14


# --------------------------------------------------------------- collision ---
def _random_collision_inputs(seed, n=64):
    g = rng(seed)
    rho = 0.5 + 6 * torch.rand(n, generator=g, dtype=DT)
    u = 0.2 * (torch.rand((3, n), generator=g, dtype=DT) - 0.5)
    pm = 0.32 + 0.03 * torch.rand(n, generator=g, dtype=DT)
    F = 0.01 * (torch.rand((3, n), generator=g, dtype=DT) - 0.5)
    Qd = tuple(0.01 * (torch.rand(n, generator=g, dtype=DT) - 0.5) for _ in range(6))
    return g, rho, u, pm, F, Qd


def test_collision_invariants():
    g, rho, u, pm, F, Qd = _random_collision_inputs(4)
    feq = ps.f_eq(rho, u, pm)
    fneq = 0.01 * (torch.rand((27, rho.numel()), generator=g, dtype=DT) - 0.5)
    f = feq + fneq
    # choose u consistent with Eq. (11): rho u = j + F/2
    j = torch.einsum("ia,i...->a...", torch.tensor(C, dtype=DT), f)
    uu = (j + 0.5 * F) / f.sum(0)
    k = lbm.central_moments(f, uu)
    assert torch.allclose(k[lbm.IDX.index((1, 0, 0))], -0.5 * F[0], atol=1e-15)
    for w0 in (0.0, 0.6, 1.0, 1.7):
        w = [w0] + [0.3 + 0.1 * i for i in range(10)]
        ks = lbm.collide(k, F, Qd, pm, w)
        assert torch.allclose(ks[0], f.sum(0), atol=1e-14)       # mass
        for a, idx in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            assert torch.allclose(ks[lbm.IDX.index(idx)], 0.5 * F[a], atol=1e-15)
        fs = lbm.populations_from_central(ks, uu)
        js = torch.einsum("ia,i...->a...", torch.tensor(C, dtype=DT), fs)
        assert torch.allclose(js, j + F, atol=1e-14)              # first raw moment gains F
    # equilibrium is a fixed point when F = Q = 0, for any rates
    k0 = lbm.central_moments(feq, u)
    w = [0.0, 1.3, 0.7, 1.9, 0.1, 1.0, 1.5, 0.4, 1.1, 0.8, 1.2]
    ks = lbm.collide(k0, 0 * F, tuple(0 * q for q in Qd), pm, w)
    assert (ks - k0).abs().max() < 1e-14
    # omega = 0 keeps the moments and adds only the source terms; each
    # diagonal second-order moment gains exactly its own Q (the combination
    # equations of Eq. (22) decouple), each fourth-order diagonal its own Q
    ks = lbm.collide(k, 0 * F, Qd, pm, [0.0] * 11)
    for idx, q in zip(((2, 0, 0), (0, 2, 0), (0, 0, 2), (2, 2, 0), (2, 0, 2), (0, 2, 2)), Qd):
        r = lbm.IDX.index(idx)
        assert torch.allclose(ks[r] - k[r], q, atol=1e-15)


def test_force_terms_are_central_moments_of_hermite_force():
    """With every rate zero and Q = 0, the collision adds to the CMs exactly
    the CMs (about u) of the force population F . d g^{eq,6} / du / rho,
    the velocity-derivative of the sixth-order Hermite equilibrium Eq. (14)."""
    g, rho, u, pm, F, Qd = _random_collision_inputs(5, n=16)
    k = torch.rand((27, 16), generator=g, dtype=DT)
    zero = tuple(0 * q for q in Qd)
    ks = lbm.collide(k, F, zero, pm, [0.0] * 11)
    uu = u.clone().requires_grad_(True)
    force_pop = torch.zeros((27, 16), dtype=DT)
    for i in range(27):
        gi = ps.g_eq6(rho, uu)[i].sum()
        (du,) = torch.autograd.grad(gi, uu)
        force_pop[i] = (F * du).sum(0) / rho
    kf = lbm.central_moments_direct(force_pop, u)
    assert (ks - k - kf).abs().max() < 1e-14


# ---------------------------------------------------------------- the step ---
def _droplet_state(p, seed=0, amp=0.0):
    rl, rv = p.coexistence()
    rho0 = phys.tanh_droplet((p.nz, p.ny, p.nx), (p.nx / 2, p.ny / 2, p.nz / 2), min(p.nx, p.ny, p.nz) / 4, rl, rv)
    rho0 = torch.tensor(rho0, dtype=DT)
    if amp:
        rho0 = rho0 + amp * (torch.rand(rho0.shape, generator=rng(seed), dtype=DT) - 0.5)
    return rho0


def test_mass_conservation_and_momentum_balance_periodic():
    """Sum of rho is invariant; the total momentum changes each step by the
    total force (the collision adds F to the first raw moment, streaming
    permutes), Eq. (11)-(12)."""
    p = lbm.Params(10, 12, 8, T=eos.temperature(0.85))
    rho0 = _droplet_state(p, amp=0.05)
    g = rng(7)
    u0 = 0.03 * (torch.rand((3,) + tuple(rho0.shape), generator=g, dtype=DT) - 0.5)
    f = lbm.init(rho0, p, u0)
    m0 = f.sum()
    for _ in range(6):
        fn, A = lbm.step(f, p, return_aux=True)
        assert abs(float(fn.sum() - m0)) < 1e-13 * float(m0)
        jn = torch.einsum("ia,i...->a", torch.tensor(C, dtype=DT), fn)
        j = torch.einsum("ia,i...->a", torch.tensor(C, dtype=DT), f)
        assert torch.allclose(jn - j, A["F"].sum((1, 2, 3)), atol=1e-12)
        f = fn


def test_uniform_state_is_invariant():
    p = lbm.Params(6, 5, 4, T=eos.temperature(0.8))
    rho0 = torch.full((4, 5, 6), 2.3, dtype=DT)
    u0 = torch.tensor([0.05, -0.02, 0.01], dtype=DT).view(3, 1, 1, 1).expand(3, 4, 5, 6)
    f = lbm.init(rho0, p, u0)
    fn = lbm.step(f, p)
    assert (fn - f).abs().max() < 1e-15


def _flat_state(p, tr, nz_fluid=None):
    rl, rv = p.coexistence()
    prof = phys.tanh_profile_1d(p.nz, rl, rv)
    r, mus = phys.flat_equilibrium(prof, p.a, p.b, p.R, p.T, p.kappa)
    rho0 = torch.tensor(r, dtype=DT).view(p.nz, 1, 1).expand(p.nz, p.ny, p.nx).contiguous()
    return rho0, r, mus


@pytest.mark.parametrize("tr,nu", [(0.7, 0.15), (0.8, 0.03), (0.9, 0.15)])
def test_discrete_flat_equilibrium_is_fixed_point(tr, nu):
    """Any density with uniform discrete mu and zero velocity is an exact
    fixed point of the step, for every rate (moving populations equal
    (1+mu) w_i and F = Q = 0).  The Newton flat profile is one."""
    p = lbm.Params(4, 4, 64, T=eos.temperature(tr), nu=nu)
    rho0, r, mus = _flat_state(p, tr)
    f = lbm.init(rho0, p)
    fn, A = lbm.step(f, p, return_aux=True)
    assert (fn - f).abs().max() < 1e-13
    assert (A["mu"] - mus).abs().max() < 1e-13
    moving = [i for i in range(27) if i != REST]
    assert (f[moving] - (1 + mus) * W_T[moving].view(-1, 1, 1, 1)).abs().max() < 1e-14


def test_flat_interface_surface_tension_and_densities():
    """Sec. III A: 4x4x128 at 0.7 Tc; the discrete equilibrium has bulk
    densities at the Maxwell pair and sigma = 0.204 (Eq. (33))."""
    T = eos.temperature(0.7)
    rl, rv = eos.maxwell(A, B, R, T)
    prof = phys.tanh_profile_1d(128, rl, rv)
    r, mus = phys.flat_equilibrium(prof, A, B, R, T, 0.02)
    assert abs(r.max() - rl) < 1e-4 * rl and abs(r.min() - rv) < 1e-4 * rv
    sig = phys.surface_tension(r, 0.02)   # [0, Nz/2) holds the interface at Nz/4
    assert round(sig, 3) == GOLD["surface_tension_07Tc"]["sigma"]
    # mu of the coexisting bulk phases
    assert abs(mus - eos.mu0(rl, A, B, R, T)) < 1e-5


def test_flat_interface_relaxes_to_newton_state():
    """A mass-preserving mirror-symmetric perturbation of the flat
    equilibrium decays under the LB step (the Newton state attracts)."""
    p = lbm.Params(2, 2, 48, T=eos.temperature(0.85), nu=0.15)
    rl, rv = p.coexistence()
    prof = phys.tanh_profile_1d(48, rl, rv, z1=12, z2=36)
    r, mus = phys.flat_equilibrium(prof, p.a, p.b, p.R, p.T, p.kappa)
    z = np.arange(48)
    pert = 1e-3 * np.cos(2 * np.pi * 3 * (z - 24) / 48)
    rho0 = torch.tensor(r + pert, dtype=DT).view(48, 1, 1).expand(48, 2, 2).contiguous()
    f = lbm.init(rho0, p)
    d0 = (f.sum(0)[:, 0, 0] - torch.tensor(r)).abs().max()
    f = lbm.run(f, p, 400)
    d1 = (f.sum(0)[:, 0, 0] - torch.tensor(r)).abs().max()
    assert d1 < 0.05 * d0


def test_cubic_symmetry():
    """Exchanging x and y (with the matching population permutation) and
    mirroring z commute with the step."""
    p = lbm.Params(6, 6, 6, T=eos.temperature(0.85))
    g = rng(9)
    rho0 = 3.5 + 0.5 * torch.rand((6, 6, 6), generator=g, dtype=DT)
    u0 = 0.02 * (torch.rand((3, 6, 6, 6), generator=g, dtype=DT) - 0.5)
    f = lbm.init(rho0, p, u0) + 1e-4 * torch.rand((27, 6, 6, 6), generator=g, dtype=DT)
    fn = lbm.step(f, p)
    perm_xy = [C.index((c[1], c[0], c[2])) for c in C]
    swap = lambda h: h[perm_xy].transpose(2, 3)
    assert (lbm.step(swap(f), p) - swap(fn)).abs().max() < 1e-13
    perm_z = [C.index((c[0], c[1], -c[2])) for c in C]
    mir = lambda h: torch.roll(torch.flip(h[perm_z], dims=(1,)), 1, dims=1)
    assert (lbm.step(mir(f), p) - mir(fn)).abs().max() < 1e-13


# ------------------------------------------------------------------ walls ---
def test_wall_density_weights_and_modes():
    """Eqs. (37)-(38) on a flat wall: rho_ave is the first-layer average with
    weights 4/9 (normal neighbour), 1/9 (edge) and 1/36 (corner) that follow
    from Eq. (17); the window and limiter act only inside
    [0.05 rl + 0.95 rv, 0.95 rl + 0.05 rv]."""
    T = eos.temperature(0.7)
    rl, rv = eos.maxwell(A, B, R, T)
    lo, hi = 0.05 * rl + 0.95 * rv, 0.95 * rl + 0.05 * rv
    g = rng(11)
    layer = rv + (rl - rv) * torch.rand((5, 5), generator=g, dtype=DT)
    rho = torch.zeros((4, 5, 5), dtype=DT)
    rho[1] = layer
    rho[2] = layer
    wts = {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}
    for mode, val in ((lbm.NEUTRAL, 1.0), (lbm.PHI, 1.6), (lbm.DELTA, 1.8)):
        p = lbm.Params(5, 5, 4, walls_z=True, T=T, wet_mode=mode, wet_value=val)
        out = lbm.wall_density(rho, lbm.fluid_mask(p), p)
        for (y, x) in ((0, 0), (2, 3), (4, 1)):
            ave = sum(wts[abs(dy) + abs(dx)] * float(layer[(y + dy) % 5, (x + dx) % 5])
                      for dy in (-1, 0, 1) for dx in (-1, 0, 1))
            if lo <= ave <= hi and mode == lbm.PHI:
                exp = min(max(val * ave, lo), hi)
            elif lo <= ave <= hi and mode == lbm.DELTA:
                exp = min(max(ave - val, lo), hi)
            else:
                exp = ave
            assert abs(float(out[0, y, x]) - exp) < 1e-14
            assert abs(float(out[3, y, x]) - exp) < 1e-14


@pytest.mark.parametrize("mode,val", [(0, 1.0), (1, 1.6), (2, 1.8)])
def test_wall_film_equilibrium_is_fixed_point(mode, val):
    """A liquid film on a wall (profile uniform in x, y) at the discrete
    equilibrium of the wall-density rule is a fixed point: halfway
    bounce-back reflects the uniform populations, mu(x_s) equals the
    uniform mu."""
    T = eos.temperature(0.7)
    rl, rv = eos.maxwell(A, B, R, T)
    lo, hi = 0.05 * rl + 0.95 * rv, 0.95 * rl + 0.05 * rv
    nz = 40
    zf = np.arange(1, nz - 1, dtype=np.float64)
    init = rv + 0.5 * (rl - rv) * (1 - np.tanh(2 * (zf - 12.0) / 5))
    if mode == 1:
        rw = lambda r: min(max(val * r, lo), hi) if lo <= r <= hi else r
        drw = lambda r: (val if lo <= val * r <= hi else 0.0) if lo <= r <= hi else 1.0
    elif mode == 2:
        rw = lambda r: min(max(r - val, lo), hi) if lo <= r <= hi else r
        drw = lambda r: (1.0 if lo <= r - val <= hi else 0.0) if lo <= r <= hi else 1.0
    else:
        rw, drw = (lambda r: r), (lambda r: 1.0)
    r, mus = phys.wall_flat_equilibrium(init, A, B, R, T, 0.02, rw, drw)
    p = lbm.Params(3, 3, nz, walls_z=True, T=T, wet_mode=mode, wet_value=val)
    rho0 = torch.zeros((nz, 3, 3), dtype=DT)
    rho0[1:-1] = torch.tensor(r, dtype=DT).view(-1, 1, 1)
    f = lbm.init(rho0, p)
    fn, Aux = lbm.step(f, p, return_aux=True)
    assert (fn - f).abs().max() < 1e-13
    assert (Aux["mu"] - mus).abs().max() < 1e-13


def test_mass_conservation_with_walls():
    p = lbm.Params(8, 6, 10, walls_z=True, T=eos.temperature(0.7), wet_mode=lbm.PHI, wet_value=1.4)
    rl, rv = p.coexistence()
    rho0 = torch.tensor(phys.tanh_droplet((10, 6, 8), (4, 3, 0.5), 4.0, rl, rv), dtype=DT)
    u0 = torch.zeros((3, 10, 6, 8), dtype=DT)
    u0[0] = 0.02
    f = lbm.init(rho0, p, u0)
    m0 = f.sum()
    for _ in range(5):
        f = lbm.step(f, p)
        assert abs(float(f.sum() - m0)) < 1e-13 * float(m0)
    assert float(f[:, 0].abs().max()) == 0.0 and float(f[:, -1].abs().max()) == 0.0


# ------------------------------------------------- Q correction, viscosity ---
def _moving_flat_error(scale, axis, monkeypatch, tr=0.9, u=0.05, T=100, n=64):
    """Max deviation (relative to rho_l - rho_v) between a flat interface
    advected T steps at uniform normal velocity u and the rest equilibrium
    profile shifted by u T (an integer number of nodes)."""
    shape = [1, 1, 1]
    shape[axis] = n
    p = lbm.Params(nx=shape[0], ny=shape[1], nz=shape[2], T=eos.temperature(tr), nu=0.15)
    rl, rv = p.coexistence()
    r, _ = phys.flat_equilibrium(phys.tanh_profile_1d(n, rl, rv), p.a, p.b, p.R, p.T, p.kappa)
    view = [1, 1, 1]
    view[2 - axis] = n
    rho0 = torch.tensor(r, dtype=DT).view(*view)
    u0 = torch.zeros((3,) + tuple(rho0.shape), dtype=DT)
    u0[axis] = u
    orig = lbm.aux_fields

    def scaled(f, pp):
        A_ = orig(f, pp)
        A_["Q"] = tuple(scale * q for q in A_["Q"])
        return A_

    monkeypatch.setattr(lbm, "aux_fields", scaled)
    f = lbm.init(rho0, p, u0)
    f = lbm.run(f, p, T)
    monkeypatch.setattr(lbm, "aux_fields", orig)
    rho = f.sum(0).reshape(-1).numpy()
    return np.abs(rho - np.roll(r, int(round(u * T)))).max() / (rl - rv)


@pytest.mark.parametrize("axis", [0, 2])
def test_q_correction_coefficient_minimises_galilean_error(axis, monkeypatch):
    """Eq. (27) restores the third-order diagonal moments lost to the lattice
    (c^3 = c); with it a flat interface advected along its normal stays a
    translated copy of the rest profile.  Scaling Q by 0.9 or 1.1 (a wrong
    coefficient) makes the Galilean error several times larger; dropping Q
    makes the run blow up."""
    e1 = _moving_flat_error(1.0, axis, monkeypatch)
    assert e1 < 0.03
    assert _moving_flat_error(0.9, axis, monkeypatch) > 3 * e1
    assert _moving_flat_error(1.1, axis, monkeypatch) > 3 * e1


def test_shear_wave_decay_gives_nu():
    """omega_1 from tau = rho nu / p_m + 1/2 (Sec. II B) makes a transverse
    shear wave in a uniform fluid decay at rate nu k^2 (after the initial
    layer; a density other than 1 exercises the rho / p_m factor)."""
    n, nu, U, rho = 64, 0.15, 1e-4, 1.5
    p = lbm.Params(1, 1, n, T=eos.temperature(0.8), nu=nu)
    rho0 = torch.full((n, 1, 1), rho, dtype=DT)
    z = torch.arange(n, dtype=DT)
    k = 2 * math.pi / n
    u0 = torch.zeros((3, n, 1, 1), dtype=DT)
    u0[0] = (U * torch.sin(k * z)).view(n, 1, 1)
    cx = torch.tensor([c[0] for c in C], dtype=DT)
    amp = lambda f: float((torch.einsum("i,i...->...", cx, f)[:, 0, 0] * torch.sin(k * z)).sum() * 2 / n / rho)
    f = lbm.run(lbm.init(rho0, p, u0), p, 50)
    a50 = amp(f)
    a200 = amp(lbm.run(f, p, 150))
    rate = math.log(a200 / a50) / 150
    assert abs(rate / (-nu * k * k) - 1) < 2e-3


# ---------------------------------------------------------------------------
# Moving walls (the moving-wall droplet test of Sec. III B)
# ---------------------------------------------------------------------------
def _moving_params(nx, ny, nz, wall_u):
    T = 0.7 * eos.critical_point(eos.PAPER["a"], eos.PAPER["b"], 1.0)[1]
    return lbm.Params(nx, ny, nz, walls_z=True, T=T, omega=[1.0, 1.0, 1.0, 0.5] + [1.0] * 7,
                      wall_u=tuple(wall_u)), T


@pytest.mark.parametrize("phase", ["liquid", "vapour"])
def test_moving_walls_leave_a_comoving_fluid_unchanged(phase):
    """A uniform fluid moving with both walls is a fixed point of the step:
    the reflected populations take exactly the equilibrium's odd part at the
    wall velocity (any error in sign, factor, wall side or the p_m structure
    of the correction breaks this at the first step)."""
    U = (0.1, -0.03)
    p, T = _moving_params(3, 4, 9, (U[0], U[1], U[0], U[1]))
    rl, rv = eos.maxwell(p.a, p.b, p.R, T)
    r = rl if phase == "liquid" else rv
    rho = torch.full((9, 4, 3), r, dtype=torch.float64)
    u0 = torch.zeros((3, 9, 4, 3), dtype=torch.float64)
    u0[0], u0[1] = U
    f = lbm.init(rho, p, u0)
    f1 = lbm.step(f, p)
    assert float((f1 - f).abs().max() / f.abs().max()) < 1e-13


def test_moving_walls_couette_profile_is_linear():
    """Walls at -U (bottom) and +U (top) in a uniform liquid: the steady
    velocity is linear between the walls located half a link beyond the
    first and last fluid planes, u_x(z) = -U + 2U (z - 1/2)/(nz - 2), with
    no slip; the mass is conserved."""
    U = 1e-3
    nz = 6  # four fluid planes: the start-up transient decays by ~20x per 100 steps
    p, T = _moving_params(1, 1, nz, (-U, 0.0, U, 0.0))
    rl, _ = eos.maxwell(p.a, p.b, p.R, T)
    f = lbm.init(torch.full((nz, 1, 1), rl, dtype=torch.float64), p)
    m0 = float(lbm.aux_fields(f, p)["rho"][1:-1].sum())
    for _ in range(500):
        f = lbm.step(f, p)
    A = lbm.aux_fields(f, p)
    z = torch.arange(1, nz - 1, dtype=torch.float64)
    exact = -U + 2 * U * (z - 0.5) / (nz - 2)
    ux = A["u"][0][1:-1, 0, 0]
    assert float((ux - exact).abs().max()) < 1e-6 * U
    assert float(A["u"][1].abs().max()) < 1e-15 and float(A["u"][2][1:-1].abs().max()) < 1e-13
    assert abs(float(A["rho"][1:-1].sum()) - m0) < 1e-12 * m0


def test_moving_wall_correction_reduces_to_the_ideal_gas_form():
    """With p_m = rho c_s^2 the bracket f^eq_o - f^eq_i at the wall velocity
    is, to first order in u_w, the textbook 2 w_o rho c_o . u_w / c_s^2."""
    rho = torch.tensor([[[2.3]]], dtype=torch.float64)
    pm = rho / 3.0
    eps = 1e-6
    uw = torch.zeros((3, 1, 1, 1), dtype=torch.float64)
    uw[0], uw[1] = eps, -0.5 * eps
    feq = lbm.populations_from_central(lbm.equilibrium_central(rho, pm), uw)
    for o, c in enumerate(C):
        i = OPP[o]
        got = float(feq[o] - feq[i])
        want = 2.0 * float(W_EXACT[o]) * 2.3 * (c[0] * eps - 0.5 * c[1] * eps) * 3.0
        assert abs(got - want) < 1e-9 * eps + 1e-6 * abs(want)


def test_mass_conservation_with_moving_walls():
    """A droplet between walls moving in opposite directions keeps its mass
    to round-off (the corrections of the reflected populations cancel)."""
    nz, ny, nx = 12, 10, 11
    p, T = _moving_params(nx, ny, nz, (0.05, 0.02, -0.04, 0.0))
    rl, rv = eos.maxwell(p.a, p.b, p.R, T)
    rho = torch.tensor(phys.tanh_droplet((nz, ny, nx), (nx / 2, ny / 2, 0.5), 4.5, rl, rv), dtype=DT)
    f = lbm.init(rho, p)
    m0 = float(lbm.aux_fields(f, p)["rho"][1:-1].sum())
    for _ in range(8):
        f = lbm.step(f, p)
    m1 = float(lbm.aux_fields(f, p)["rho"][1:-1].sum())
    assert abs(m1 - m0) < 1e-12 * m0
