"""Linear stability of the step next to a halfway bounce-back wall (oracle,
CPU).  Documents a property of the method as read here: with every
higher-order rate at 1, a wall bounding the 0.7 T_c vapour has an unstable
mode (tangential velocity alternating in x along the first fluid layer);
omega_3 = 0.5 removes it; the same vapour without walls is neutrally
stable.  With moving walls (the momentum-corrected bounce-back of the
moving-wall test, Sec. III B) the same holds around the vapour moving with
the walls and around the sheared vapour between walls moving in opposite
directions: the wall mode at omega_3 = 1, neutral at omega_3 = 1/2.  In the
uniform phases the step leaves the Nyquist mode in x (alternating density
and momentum, on which the central-difference force vanishes) undamped:
eigenvalue -1."""
import numpy as np
import torch

from oracle import eos, lattice, lbm


def spectral_radius(walls, omega3, tr=0.7, nu=0.15):
    om = [1.0] * 11
    om[3] = omega3
    nx, ny, nz = 2, 1, 6
    p = lbm.Params(nx, ny, nz, walls_z=walls, T=eos.temperature(tr), omega=om, nu=nu)
    rl, rv = p.coexistence()
    f0 = lbm.init(torch.full((nz, ny, nx), rv, dtype=torch.float64), p)
    keep = torch.ones_like(f0, dtype=torch.bool)
    if walls:
        keep[:, 0] = False
        keep[:, -1] = False
    idx = keep.reshape(-1).nonzero().squeeze(1)

    def F(v):
        f = f0.reshape(-1).index_put((idx,), v)
        return lbm.step(f.reshape(f0.shape), p).reshape(-1)[idx]

    J = torch.autograd.functional.jacobian(F, f0.reshape(-1)[idx], vectorize=True)
    return float(np.abs(np.linalg.eigvals(J.numpy())).max())


def test_wall_vapour_mode():
    assert spectral_radius(True, 1.0) > 1.15
    assert abs(spectral_radius(True, 0.5) - 1.0) < 1e-9
    assert abs(spectral_radius(False, 1.0) - 1.0) < 1e-9
    assert abs(spectral_radius(True, 0.5, nu=0.03) - 1.0) < 1e-3
    assert abs(spectral_radius(True, 1.0, tr=0.8) - 1.0) < 1e-9


def moving_wall_radius(omega3, U, Ut, base_steps, nx=2, nz=6, tr=0.7, nu=0.15):
    """Spectral radius of the linearised step around the 0.7 T_c vapour
    between walls moving at U (bottom) and Ut (top), started from the linear
    Couette profile and stepped base_steps times towards its steady state
    (with U = Ut the vapour moving with the walls is a fixed point)."""
    om = [1.0] * 11
    om[3] = omega3
    p = lbm.Params(nx, 1, nz, walls_z=True, T=eos.temperature(tr), omega=om, nu=nu, wall_u=(U, 0.0, Ut, 0.0))
    rl, rv = p.coexistence()
    u = torch.zeros((3, nz, 1, nx), dtype=torch.float64)
    z = torch.arange(nz, dtype=torch.float64)
    u[0] = (U + (Ut - U) * (z - 0.5) / (nz - 2)).reshape(nz, 1, 1)
    f = lbm.init(torch.full((nz, 1, nx), rv, dtype=torch.float64), p, u)
    for _ in range(base_steps):
        f = lbm.step(f, p)
    keep = torch.ones_like(f, dtype=torch.bool)
    keep[:, 0] = False
    keep[:, -1] = False
    idx = keep.reshape(-1).nonzero().squeeze(1)

    def F(v):
        return lbm.step(f.reshape(-1).index_put((idx,), v).reshape(f.shape), p).reshape(-1)[idx]

    J = torch.autograd.functional.jacobian(F, f.reshape(-1)[idx], vectorize=True)
    return float(np.abs(np.linalg.eigvals(J.numpy())).max())


def test_moving_wall_vapour_modes():
    assert moving_wall_radius(1.0, 0.1, 0.1, 0) > 1.15
    assert abs(moving_wall_radius(0.5, 0.1, 0.1, 0) - 1.0) < 1e-9
    assert abs(moving_wall_radius(0.5, 0.1, -0.1, 300) - 1.0) < 1e-9


def test_nyquist_mode_is_undamped():
    """The uniform 0.7 T_c liquid moving at u_x = 0.1 (periodic, no walls):
    the step has an eigenvalue -1 whose mode alternates density and x-momentum
    from node to node (the wavenumber pi in x), on which the central-difference
    gradient of the force vanishes; nothing damps it."""
    om = [1.0] * 11
    om[3] = 0.5
    nx = 2
    p = lbm.Params(nx, 1, 1, walls_z=False, T=eos.temperature(0.7), omega=om, nu=0.15)
    rl, rv = p.coexistence()
    u = torch.zeros((3, 1, 1, nx), dtype=torch.float64)
    u[0] = 0.1
    f = lbm.init(torch.full((1, 1, nx), rl, dtype=torch.float64), p, u)
    J = torch.autograd.functional.jacobian(lambda v: lbm.step(v.reshape(f.shape), p).reshape(-1), f.reshape(-1),
                                           vectorize=True).numpy()
    ev, V = np.linalg.eig(J)
    assert np.abs(ev).max() < 1 + 1e-12
    k = int(np.argmin(np.abs(ev + 1)))
    assert abs(ev[k] + 1) < 1e-12
    v = np.real(V[:, k]).reshape(f.shape)
    drho = v[:, 0, 0, :].sum(0)
    cx = np.array([lattice.C_T[i][0] for i in range(27)], dtype=float)
    djx = (cx[:, None] * v[:, 0, 0, :]).sum(0)
    assert abs(drho[0] + drho[1]) < 1e-12 * abs(drho[0]) and abs(drho[0]) > 1e-3
    assert abs(djx[0] + djx[1]) < 1e-12 * abs(djx[0]) and abs(djx[0]) > 1e-3
