"""torch.autograd.Function over the hand-written discrete adjoint.

    rho_T = LBFEFunction.apply(rho0, kappa, wet_value, cfg)

runs `cfg.steps` time steps from the initial density rho0 (float64 tensor
on the GPU, shape (nz, ny, nx)) and returns the final density field.  Its
backward pass seeds lambda(T) = dL/drho_T, sweeps the adjoint steps in
reverse, recomputing the forward states segment by segment from checkpoints
taken every `cfg.checkpoint_every` steps (uniform checkpointing: memory is
T/K checkpoints plus K states of one segment), and returns dL/drho0,
dL/dkappa and dL/d(wet_value).  The recomputation is bitwise identical to
the forward pass, so the gradients do not depend on K.

kappa and wet_value are 0-d tensors; their values configure the library
context (the HIP library needs them as parameters), their gradients come
from the adjoint's accumulators.  All arithmetic runs in liblbfe.so.
"""
from dataclasses import dataclass, field

import torch

from . import lbfe


@dataclass
class StepConfig:
    nx: int
    ny: int
    nz: int
    steps: int
    checkpoint_every: int = 200
    T: float = 0.05
    nu: float = 0.15
    walls_z: int = 0
    wet_mode: int = lbfe.WET_NEUTRAL
    precision: str = "fp64"
    corr4: int = 1
    omega: list = field(default_factory=lambda: [1.0] * 11)
    u0: object = None          # optional (3, nz, ny, nx) initial velocity
    device: str = "cuda"
    stats: dict = field(default_factory=dict)   # filled with timing/memory info

    def make(self, kappa, wet_value):
        return lbfe.Simulation(device=self.device, nx=self.nx, ny=self.ny, nz=self.nz, T=self.T, nu=self.nu,
                               kappa=float(kappa), walls_z=self.walls_z, wet_mode=self.wet_mode,
                               wet_value=float(wet_value), precision=self.precision, corr4=self.corr4,
                               omega=self.omega, adjoint=1, check_every=max(1, self.checkpoint_every))


class LBFEFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, kappa, wet_value, cfg):
        sim = cfg.make(kappa.item(), wet_value.item())
        sim.init_density(rho0.detach(), cfg.u0)
        K = max(1, int(cfg.checkpoint_every))
        checkpoints = {}
        for s in range(0, cfg.steps, K):
            checkpoints[s] = sim.get_state().clone()
            sim.step(min(K, cfg.steps - s))
        rho_T = sim.fields()["rho"]
        ctx.sim, ctx.cfg, ctx.checkpoints = sim, cfg, checkpoints
        ctx.save_for_backward(rho0)
        return rho_T

    @staticmethod
    def backward(ctx, grad_rho):
        sim, cfg = ctx.sim, ctx.cfg
        (rho0,) = ctx.saved_tensors
        K = max(1, int(cfg.checkpoint_every))
        sim.adjoint_seed(grad_rho.detach().to(torch.float64))
        starts = sorted(ctx.checkpoints, reverse=True)
        for s0 in starts:
            s1 = min(s0 + K, cfg.steps)
            sim.set_state(ctx.checkpoints[s0], s0)
            states = [sim.get_state().clone()]
            for _ in range(s0 + 1, s1):
                sim.step(1)
                states.append(sim.get_state().clone())
            for t in range(s1 - 1, s0 - 1, -1):
                sim.adjoint_step(states[t - s0])
            del states
        g_rho0 = sim.adjoint_init_density(rho0.detach(), cfg.u0)
        g = sim.adjoint_grads()
        dev = grad_rho.device
        g_kappa = torch.tensor(g["kappa"], dtype=torch.float64, device=dev)
        g_wet = torch.tensor(g["wet_value"], dtype=torch.float64, device=dev)
        cfg.stats["dL_dnu"] = g["nu"]
        ctx.sim = None
        ctx.checkpoints = None
        return g_rho0, g_kappa, g_wet, None


def simulate(rho0, kappa, wet_value, cfg):
    """Differentiable final density field (see LBFEFunction)."""
    if not isinstance(kappa, torch.Tensor):
        kappa = torch.tensor(float(kappa), dtype=torch.float64)
    if not isinstance(wet_value, torch.Tensor):
        wet_value = torch.tensor(float(wet_value), dtype=torch.float64)
    return LBFEFunction.apply(rho0, kappa, wet_value, cfg)
