"""Pin P9 in three dimensions: a droplet density field solved by Newton's
method so that mu0(rho) - kappa lap_h rho is the same constant at every
node (oracle.phys.static_equilibrium_3d, with the mass of a tanh droplet)
is an exact fixed point of the step for any relaxation rates: with u = 0
the force (1/3 - rho) grad mu and the Q terms vanish and the moving
populations are uniform (1 + mu*) w_i.  One oracle step must leave it
unchanged to rounding; a wrong stencil weight, a sign in the force or an
ignored term of the collision would move it."""
import functools

import numpy as np
import torch

from oracle import eos, lbm, phys

A, B, R = eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"]


@functools.lru_cache(maxsize=None)
def _droplet(n=16, tr=0.7, radius=5.0):
    T = eos.temperature(tr)
    rl, rv = eos.maxwell(A, B, R, T)
    rho0 = phys.tanh_droplet((n, n, n), (n / 2, n / 2, n / 2), radius, rl, rv)
    r, mu = phys.static_equilibrium_3d(rho0, A, B, R, T, 0.02)
    return T, rl, rv, rho0, r, mu


def test_newton_droplet_solves_the_discrete_equilibrium():
    T, rl, rv, rho0, r, mu = _droplet()
    # a droplet (not the uniform state of the same mass), mass kept
    assert r.max() - r.min() > 0.8 * (rl - rv)
    assert abs(r.sum() - rho0.sum()) < 1e-12 * rho0.sum()
    # residual with the oracle's own stencil (torch.roll), not the sparse
    # matrix the solver used
    p = lbm.Params(16, 16, 16, T=T)
    rt = torch.tensor(r)
    res = lbm.mu_bulk(rt, p) - p.kappa * lbm.lap_h(rt) - mu
    assert float(res.abs().max()) < 1e-13
    # cubic symmetry of the centred droplet
    assert np.allclose(r, r.transpose(1, 0, 2), atol=1e-12)
    # mirror x -> 16 - x about the centre node 8 (periodic)
    assert np.allclose(r, np.roll(np.flip(r, axis=2), 1, axis=2), atol=1e-12)


def test_newton_droplet_is_a_fixed_point_of_the_step():
    T, rl, rv, rho0, r, mu = _droplet()
    g = np.random.Generator(np.random.PCG64(31))
    for nu, om in ((0.15, [1.0] * 11), (0.03, list(g.uniform(0.5, 1.6, 11)))):
        p = lbm.Params(16, 16, 16, T=T, nu=nu, omega=om)
        f = lbm.init(torch.tensor(r), p)
        f1 = lbm.step(f, p)
        e = float((f1 - f).abs().max() / f.abs().max())
        assert e < 1e-13, (nu, e)
        A_ = lbm.aux_fields(f, p)
        assert float(A_["u"].abs().max()) < 1e-14
        assert float((A_["mu"] - mu).abs().max()) < 1e-13


def test_tanh_droplet_is_not_a_fixed_point():
    # the same check on the initial tanh profile fails: the pin can fail
    T, rl, rv, rho0, r, mu = _droplet()
    p = lbm.Params(16, 16, 16, T=T)
    f = lbm.init(torch.tensor(rho0), p)
    e = float((lbm.step(f, p) - f).abs().max() / f.abs().max())
    assert e > 1e-6
