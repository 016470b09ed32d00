"""Shared helpers of the GPU tests (parity metrics, oracle wrappers)."""
import sys

import numpy as np
import torch

from oracle import eos, lbm
from paper_2504_03819_amd import inputs, lbfe

DT = torch.float64
A_, B_, R_ = eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(gpu, ora):
    """max |gpu - ora| / max |ora| (absolute when the oracle field is 0)."""
    g = torch.as_tensor(gpu).detach().double().cpu()
    o = torch.as_tensor(ora).detach().double().cpu()
    d = float((g - o).abs().max())
    s = float(o.abs().max())
    return d / s if s > 0 else d


def oracle_params(sim_or_params):
    p = sim_or_params.params if hasattr(sim_or_params, "params") else sim_or_params
    solid = getattr(sim_or_params, "solid", None)
    return lbm.Params(int(p.nx), int(p.ny), int(p.nz), walls_z=bool(p.walls_z), a=p.a, b=p.b, R=p.R, T=p.T,
                      kappa=p.kappa, nu=p.nu, omega=list(p.omega), corr4=bool(p.corr4), rho_l=p.rho_l,
                      rho_v=p.rho_v, wet_mode=int(p.wet_mode), wet_value=p.wet_value,
                      wall_u=tuple(float(v) for v in p.wall_u),
                      solid=None if solid is None else solid.cpu() != 0)


def make_sim(**kw):
    return lbfe.Simulation(device="cuda:0", **kw)


def droplet_rho(shape, T, radius=None, center=None, noise=1e-3, seed=0, walls=False):
    rl, rv = eos.maxwell(A_, B_, R_, T)
    nz, ny, nx = shape
    radius = radius or min(shape) / 3.5
    center = center or (nx / 2, ny / 2, 0.5 if walls else nz / 2)
    rho = inputs.sphere(shape, center, radius, rl, rv)
    if noise:
        rho = rho + inputs.uniform_noise(shape, noise, seed)
    if walls:
        rho[0] = rv
        rho[-1] = rv
    return rho


def oracle_fields(f, p):
    A = lbm.aux_fields(f, p)
    Q = torch.stack(A["Q"][:3])
    return {"rho": A["rho"], "u": A["u"], "mu": A["mu"], "F": A["F"], "Q": Q}


def gpu_fields(sim):
    out = sim.fields()
    out["Q"] = sim.field(lbfe.FIELD_Q)
    return {k: v.cpu() for k, v in out.items()}


def fluid_slice(p):
    return slice(1, -1) if p.walls_z else slice(None)


def _window_step(f_win, p_win):
    return lbm.step(f_win, p_win)


def sampled_windows(sim, f_t, f_t1, centres, tol, label):
    """Oracle steps of 17^3 windows of f(t) (device tensors, indexed on the
    device) around the sample centres, compared on the central 5^3 with
    f(t+1).  In the bulk a node's update depends on f(t) within 4 nodes (3
    stencil hops plus streaming); next to a wall within 6 in x and y, since
    the wall density and the wall chemical potential each average the first
    fluid layer over x+-1, y+-1.  Next to a wall the window starts (ends) at
    the real solid plane and the first (last) five fluid planes are compared;
    the oracle also treats the window's far z-face as solid, which stays
    more than 6 planes away."""
    p = oracle_params(sim)
    nz, ny, nx = sim.shape
    worst = 0.0
    mid = slice(6, 11)
    for (cz, cy, cx) in centres:
        iy = np.arange(cy - 8, cy + 9) % ny
        ix = np.arange(cx - 8, cx + 9) % nx
        if p.walls_z and cz < 9:
            iz, cmp_z, walls = np.arange(0, 17), slice(1, 6), True
        elif p.walls_z and cz > nz - 10:
            iz, cmp_z, walls = np.arange(nz - 17, nz), slice(11, 16), True
        else:
            iz, cmp_z, walls = np.arange(cz - 8, cz + 9) % nz, mid, False
        dev = f_t.device
        tz, ty, tx = (torch.as_tensor(v, device=dev) for v in (iz, iy, ix))
        win = f_t.index_select(1, tz).index_select(2, ty).index_select(3, tx).double().cpu()
        pw = lbm.Params(17, 17, 17, walls_z=walls, T=p.T, kappa=p.kappa, nu=p.nu, omega=p.omega, corr4=p.corr4,
                        rho_l=p.rho_l, rho_v=p.rho_v, wet_mode=p.wet_mode, wet_value=p.wet_value,
                        wall_u=p.wall_u)
        fo = _window_step(win, pw)[:, cmp_z, mid, mid]
        fg = f_t1.index_select(1, tz[cmp_z]).index_select(2, ty[mid]).index_select(3, tx[mid]).double().cpu()
        e = float((fg - fo).abs().max() / fo.abs().max())
        worst = max(worst, e)
    say(f"{label}: sampled windows, max rel err {worst:.2e}")
    assert worst < tol
