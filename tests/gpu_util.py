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
