"""Linear stability of the step next to a halfway bounce-back wall (oracle,
CPU).  Documents a property of the method as read here: with every
higher-order rate at 1, a wall bounding the 0.7 T_c vapour has an unstable
mode (tangential velocity alternating in x along the first fluid layer);
omega_3 = 0.5 removes it; the same vapour without walls is neutrally
stable."""
import numpy as np
import torch

from oracle import eos, lbm


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

    J = torch.autograd.functional.jacobian(F, f0.reshape(-1)[idx])
    return float(np.abs(np.linalg.eigvals(J.numpy())).max())


def test_wall_vapour_mode():
    assert spectral_radius(True, 1.0) > 1.15
    assert abs(spectral_radius(True, 0.5) - 1.0) < 1e-9
    assert abs(spectral_radius(False, 1.0) - 1.0) < 1e-9
    assert abs(spectral_radius(True, 0.5, nu=0.03) - 1.0) < 1e-3
    assert abs(spectral_radius(True, 1.0, tr=0.8) - 1.0) < 1e-9
