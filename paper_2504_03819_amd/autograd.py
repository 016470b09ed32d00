"""torch.autograd.Function over the hand-written discrete adjoint.

    rho_T = LBFEFunction.apply(rho0, kappa, wet_value, cfg)

runs `cfg.steps` time steps from the initial density rho0 (float64 tensor
on the GPU, shape (nz, ny, nx)) and returns the final density field.  Its
backward pass seeds lambda(T) = dL/drho_T, sweeps the adjoint steps in
reverse and returns dL/drho0, dL/dkappa and dL/d(wet_value).  The forward
states are recomputed either segment by segment from checkpoints taken every
`cfg.checkpoint_every` steps (uniform: memory is T/K checkpoints plus K
states of one segment, each with the record of its forward auxiliary fields
when `cfg.keep_aux`) or by the binomial schedule of reverse_binomial
(memory: `cfg.snapshots` states).  The recomputation is bitwise identical to
the forward pass, so the gradients do not depend on the schedule.

kappa and wet_value are 0-d tensors; their values configure the library
context (the HIP library needs them as parameters), their gradients come
from the adjoint's accumulators.  All arithmetic runs in liblbfe.so.
"""
from dataclasses import dataclass, field
from math import comb

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
    wall_u: tuple = (0.0, 0.0, 0.0, 0.0)  # moving walls: (ux, uy) bottom, top
    solid: object = None       # optional solid voxel mask (nz, ny, nx), nonzero = solid
    u0: object = None          # optional (3, nz, ny, nx) initial velocity
    device: str = "cuda"
    stats: dict = field(default_factory=dict)   # filled with timing/memory info
    # "uniform": a checkpoint every checkpoint_every steps and the states of
    # one segment held during its reversal; "binomial": at most `snapshots`
    # stored states besides the initial one, placed by the binomial
    # (revolve) schedule, for runs whose states do not all fit in memory
    checkpoint: str = "uniform"
    snapshots: int = 8
    # uniform schedule: keep the forward auxiliary fields of every recomputed
    # state of a segment (lbfe_step_aux), so the adjoint steps skip their
    # recomputation; costs one aux record per state held
    keep_aux: bool = True

    def make(self, kappa, wet_value):
        return lbfe.Simulation(device=self.device, nx=self.nx, ny=self.ny, nz=self.nz, T=self.T, nu=self.nu,
                               kappa=float(kappa), walls_z=self.walls_z, wet_mode=self.wet_mode,
                               wet_value=float(wet_value), precision=self.precision, corr4=self.corr4,
                               omega=self.omega, wall_u=tuple(self.wall_u), adjoint=1,
                               check_every=max(1, self.checkpoint_every), solid=self.solid)


def reverse_binomial(sim, state_a, a, b, snapshots, stats=None):
    """Run the adjoint steps b-1, ..., a (lambda(b) must be seeded) from the
    stored state f(a), holding at most `snapshots` further states at once.
    With t = b - a steps and s snapshots, r is the least number of forward
    sweeps with C(s + r, s) >= t; the next snapshot is placed after m steps,
    where the right part (t - m steps) is reversible with s - 1 snapshots and
    r sweeps and the left part (m steps) with s snapshots and r - 1 sweeps
    (C(s + r, s) = C(s - 1 + r, s - 1) + C(s + r - 1, s)).  Every recomputed
    state is bitwise the one of the forward run, so the gradients do not
    depend on the schedule."""
    if stats is None:
        stats = {}
    stats.setdefault("recompute_steps", 0)
    stats.setdefault("max_held", 0)

    cur = [None]  # the stored state the simulation currently holds, if any

    def load(st, lo):
        if cur[0] is not st:
            sim.set_state(st, lo)
            cur[0] = st

    def rev(st, lo, hi, s, held):
        stats["max_held"] = max(stats["max_held"], held)
        t = hi - lo
        if t == 1:
            sim.adjoint_step(st)
            return
        if s == 0:  # no memory left: recompute from lo for every step
            for k in range(hi - 1, lo - 1, -1):
                if k == lo:
                    sim.adjoint_step(st)
                else:
                    load(st, lo)
                    sim.step(k - lo)
                    cur[0] = None
                    stats["recompute_steps"] += k - lo
                    sim.adjoint_step(None)  # f(k) is the simulation's current state
            return
        r = 1
        while comb(s + r, s) < t:
            r += 1
        m = min(t - 1, comb(s + r - 1, s))
        m = max(m, t - comb(s - 1 + r, s - 1), 1)
        load(st, lo)
        sim.step(m)
        stats["recompute_steps"] += m
        st_m = sim.get_state()
        cur[0] = st_m  # (an adjoint step only reads the state)
        rev(st_m, lo + m, hi, s - 1, held + 1)
        del st_m
        rev(st, lo, lo + m, s, held)

    rev(state_a, a, b, int(snapshots), 0)
    return stats


class LBFEFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, kappa, wet_value, cfg):
        sim = cfg.make(kappa.item(), wet_value.item())
        sim.init_density(rho0.detach(), cfg.u0)
        K = max(1, int(cfg.checkpoint_every))
        checkpoints = {}
        if cfg.checkpoint == "binomial":
            checkpoints[0] = sim.get_state()
            sim.step(cfg.steps)
        else:
            for s in range(0, cfg.steps, K):
                checkpoints[s] = sim.get_state()
                sim.step(min(K, cfg.steps - s))
        rho_T = sim.fields()["rho"]
        ctx.sim, ctx.cfg, ctx.checkpoints = sim, cfg, checkpoints
        ctx.param_devices = (kappa.device, wet_value.device)
        ctx.save_for_backward(rho0)
        return rho_T

    @staticmethod
    def backward(ctx, grad_rho):
        sim, cfg = ctx.sim, ctx.cfg
        (rho0,) = ctx.saved_tensors
        K = max(1, int(cfg.checkpoint_every))
        sim.adjoint_seed(grad_rho.detach().to(torch.float64))
        if cfg.checkpoint == "binomial":
            if cfg.steps > 0:
                reverse_binomial(sim, ctx.checkpoints[0], 0, cfg.steps, cfg.snapshots, cfg.stats)
        else:
            for s0 in sorted(ctx.checkpoints, reverse=True):
                s1 = min(s0 + K, cfg.steps)
                sim.set_state(ctx.checkpoints[s0], s0)
                # states[k] = f(s0 + k) for the states that are stepped from
                # (with the record of their fields if kept); the segment's
                # last state stays in the simulation
                states, recs = [ctx.checkpoints[s0]], []
                for t in range(s0, s1 - 1):
                    if cfg.keep_aux:
                        recs.append(sim.aux_record())
                        sim.step_aux(recs[-1])
                    else:
                        sim.step(1)
                    if t + 1 < s1 - 1:
                        states.append(sim.get_state())
                sim.adjoint_step(None)  # f(s1 - 1)
                for t in range(s1 - 2, s0 - 1, -1):
                    if cfg.keep_aux:
                        sim.adjoint_step_aux(states[t - s0], recs[t - s0])
                    else:
                        sim.adjoint_step(states[t - s0])
                del states, recs
        g_rho0 = sim.adjoint_init_density(rho0.detach(), cfg.u0)
        g = sim.adjoint_grads()
        # each gradient on the device and in the dtype of its input
        g_rho0 = g_rho0.to(device=rho0.device, dtype=rho0.dtype)
        g_kappa = torch.tensor(g["kappa"], dtype=torch.float64, device=ctx.param_devices[0])
        g_wet = torch.tensor(g["wet_value"], dtype=torch.float64, device=ctx.param_devices[1])
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
