"""Benchmark of the D3Q27 free-energy LB step on one MI355X.

Workload (default): the largest single-GPU configuration, the two-droplet
head-on collision, a periodic 512^3 box at 0.85 T_c with two droplets of
radius 64 whose centres are 160 lattice units apart along x, approaching at
-+0.04, stepped in FP64 (the headline line) and, as extra fields, in the
FP32 and FP16-deviation (rest population in FP32) storage forms and on the
moment-state path in FP64 and FP32 (`fp64_state`, `fp32_state`: 16 numbers
per node, 32 S algorithmic bytes).

Prints ONE JSON line.  `value` is whole-job MLUPS (fluid nodes x steps /
s / 1e6) of the FP64 form, measured with HIP events around K steps on the
library's stream, inputs resident in HBM.  `roofline` describes the dominant
kernel (the collide-stream kernel of the step path the library chose), with
the bandwidth a plain 4 GiB device copy attains beside it and the whole
step's fraction on the same algorithmic bytes; `cpu_baseline` times the CPU
oracle on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
POP_BYTES = {"fp64": 8, "fp32": 4, "fp16dev": 2, "fp16dev_f0fp32": 2, "fp64_state": 8, "fp32_state": 4}
METRIC = "MLUPS and % of HBM peak, D3Q27 fused step FP64 vs FP32/FP16-store; adjoint MLUPS"
COUNTERS = os.path.join(ROOT, "profiles", "collide_counters.json")


def alg_bytes_per_node(form):
    """Method state read once and written once: 27 populations each way
    (FP16 with f0 in FP32: 26 halves + 1 float); in the moment-state forms
    (`*_state`, every rate but omega_1 at 1) the 16 post-collision numbers
    each way."""
    if form == "fp16dev_f0fp32":
        return 2 * (26 * 2 + 4)
    if form.endswith("_state"):
        return 32 * POP_BYTES[form]
    return 54 * POP_BYTES[form]


def form_params(form):
    """Simulation keywords of a bench form: a storage form, with `_state`
    the moment-state step path."""
    if form.endswith("_state"):
        return dict(precision=form[:-len("_state")], step_path=3)
    return dict(precision=form)


def kernel_source_hash():
    """Hash of every source the library is built from (the counter file is
    ignored once any of them changes)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_03819_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "lbfe.h"), "rb").read())
    return h.hexdigest()[:16]


# storage forms outside their stated tolerances for long runs (the all-FP16
# form rounds the rest population, which carries the density contrast: mass
# drifts by 5.9e-2 per 1000 steps and long runs leave the EOS domain)
INVALID_FORMS = {"fp16dev": "all-FP16 storage: mass drift 5.9e-2 per 1000 steps, diverges in long runs"}
STEP_KERNELS = ("k_moments", "k_chain", "k_collide", "k_fused", "k_wall_rho", "k_wall_move", "k_mstate")
ADJ_COUNTERS = os.path.join(ROOT, "profiles", "adjoint_counters.json")
# kernels of one adjoint step with the forward fields kept (the seed, the
# read-out and the initialiser's adjoint are not part of a step)
ADJ_STEP_KERNELS = ("k_adj_collide", "k_adj_phimu", "k_adj_rho", "k_adj_wall", "k_adj_pack", "k_adj_reduce")
PATH_NAMES = {1: "two-pass", 2: "fused", 3: "state"}
DOMINANT = {"two-pass": "k_collide (collide + push-stream)",
            "fused": "k_fused (collide + stream + next-step moments)",
            "state": "k_mstate<kCollide> (rebuild from the 16-number state, gather, collide, new state)"}


def workload(name, lbfe, torch):
    from paper_2504_03819_amd import inputs
    if name == "moving":
        T = 0.85 * 8 * (9 / 392) / (27 * (2 / 21))
        rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
        rho, u = inputs.moving_droplet(rl, rv)
        desc = "moving droplet 128^3 periodic, r=24, W=5, u0=(0.05,0.02,0), T=0.85Tc"
        return dict(nx=128, ny=128, nz=128, T=T), rho, u, desc
    if name == "spinodal":
        T = 0.8 * 8 * (9 / 392) / (27 * (2 / 21))
        rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
        rho, u = inputs.spinodal(rl, rv)
        desc = "spinodal decomposition 256^3 periodic, mean density +-1% noise, T=0.8Tc"
        return dict(nx=256, ny=256, nz=256, T=T), rho, u, desc
    if name == "stationary":
        T = 0.9 * 8 * (9 / 392) / (27 * (2 / 21))
        rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
        rho, u = inputs.stationary_droplet(rl, rv)
        desc = "stationary droplet 32^3 periodic, r=8, noise 1e-6, T=0.9Tc"
        return dict(nx=32, ny=32, nz=32, T=T), rho, u, desc
    if name == "wetting":
        T = 0.7 * 8 * (9 / 392) / (27 * (2 / 21))
        rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
        rho, u = inputs.sessile_droplet(rl, rv)
        desc = "sessile droplet 192x192x96, walls z=0,95, r=32, phi=1.0, T=0.7Tc, omega3=0.5"
        return dict(nx=192, ny=192, nz=96, T=T, walls_z=1, wet_mode=1, wet_value=1.0,
                    omega=[1.0, 1.0, 1.0, 0.5] + [1.0] * 7), rho, u, desc
    if name == "moving_walls":
        T = 0.8 * 8 * (9 / 392) / (27 * (2 / 21))
        rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
        rho = inputs.sphere((128, 128, 128), (64, 64, 64), 30.0, rl, rv)
        desc = "droplet 128^3 r=30 between walls moving at U=0.1 (x), T=0.8Tc"
        return dict(nx=128, ny=128, nz=128, T=T, walls_z=1, wall_u=(0.1, 0.0, 0.1, 0.0)), rho, None, desc
    if name == "collision":
        T = 0.85 * 8 * (9 / 392) / (27 * (2 / 21))
        rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
        rho, u = inputs.head_on_collision(rl, rv)
        desc = "head-on collision 512^3 periodic, two r=64 droplets 160 apart at +-0.04, T=0.85Tc"
        return dict(nx=512, ny=512, nz=512, T=T), rho, u, desc
    if name == "pillars":
        T = 0.7 * 8 * (9 / 392) / (27 * (2 / 21))
        rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
        shape = (96, 192, 192)
        mask = inputs.mask_pillars(shape, plate=2, pitch=12, width=4, height=6)
        rho = inputs.sphere(shape, (96.0, 96.0, 8.0), 32.0, rl, rv)
        rho[mask.astype(bool)] = rv
        desc = ("droplet r=32 on a pillared substrate 192x192x96 (solid mask: plate 2, pillars 4x4x6 at pitch 12, "
                "solid top layer), drho=0.9, T=0.7Tc, omega3=0.5")
        return dict(nx=192, ny=192, nz=96, T=T, wet_mode=2, wet_value=0.9, solid=mask,
                    omega=[1.0, 1.0, 1.0, 0.5] + [1.0] * 7), rho, None, desc
    raise SystemExit(f"unknown workload {name}")


def time_form(lbfe, torch, geom, rho, u, form, steps, warmup, timed_steps):
    sim = lbfe.Simulation(device="cuda:0", **form_params(form), **geom)
    nfluid = sim.params.nx * sim.params.ny * (sim.params.nz - (2 if sim.params.walls_z else 0))
    if geom.get("solid") is not None:
        nfluid = int((geom["solid"] == 0).sum())
    sim.init_density(torch.tensor(rho), None if u is None else torch.tensor(u))
    sim.step(warmup)
    torch.cuda.synchronize()
    stream = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kms = sim.step_timed(timed_steps)
    kavg = {k: v / timed_steps for k, v in kms.items()}
    path = PATH_NAMES[sim.params.step_path]
    mlups = nfluid * steps / (ms / 1e3) / 1e6
    b_alg = alg_bytes_per_node(form)
    out = {
        "mlups": mlups,
        "ms_per_step": ms / steps,
        "step_alg_GBps": mlups * 1e6 * b_alg / 1e9,
        "step_alg_frac": mlups * 1e6 * b_alg / 1e9 / HBM_PEAK_GBS,
        "kernel_ms": {k: round(v, 5) for k, v in kavg.items()},
        "collide_alg_GBps": nfluid * b_alg / (kavg["collide_stream"] / 1e3) / 1e9,
        "nfluid": nfluid,
        "step_path": path,
    }
    if form in INVALID_FORMS:
        out["valid"] = False
        out["invalid_because"] = INVALID_FORMS[form]
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def time_adjoint(lbfe, torch, steps=20, form="fp32"):
    """Adjoint of the wetting workload (192x192x96, walls, FP32): K forward
    states are stored with the records of their forward auxiliary fields
    (as the checkpointed recomputation leaves them), then K adjoint steps are
    timed with the records, and again with the fields evaluated inside each
    adjoint step; the forward recompute step that a checkpointed run adds is
    timed separately."""
    geom, rho, u, desc = workload("wetting", lbfe, torch)
    sim = lbfe.Simulation(device="cuda:0", precision=form, adjoint=1, **geom)
    nfluid = sim.params.nx * sim.params.ny * (sim.params.nz - 2)
    sim.init_density(torch.tensor(rho))
    sim.step(50)
    states, recs = [], []
    for _ in range(steps):
        states.append(sim.get_state().clone())
        recs.append(sim.aux_record())
        sim.step_aux(recs[-1])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    seed = torch.ones(sim.shape, dtype=torch.float64, device="cuda:0")
    sim.adjoint_seed(seed)
    torch.cuda.synchronize()
    ev[0].record(sim.stream)
    for t in range(steps - 1, -1, -1):  # forward fields kept by the recompute steps
        sim.adjoint_step_aux(states[t], recs[t])
    ev[1].record(sim.stream)
    sim.adjoint_seed(seed)
    ev[2].record(sim.stream)
    for t in range(steps - 1, -1, -1):  # forward fields evaluated again
        sim.adjoint_step(states[t])
    ev[3].record(sim.stream)
    sim.set_state(states[0], 0)
    ev[4].record(sim.stream)
    for t in range(steps):
        sim.step_aux(recs[t])
    ev[5].record(sim.stream)
    torch.cuda.synchronize()
    adj_ms = ev[0].elapsed_time(ev[1]) / steps
    adj_re_ms = ev[2].elapsed_time(ev[3]) / steps
    fwd_ms = ev[4].elapsed_time(ev[5]) / steps
    b_alg = 81 * POP_BYTES[form]
    out = {"workload": desc + ", adjoint, " + form, "mlups_adjoint": nfluid / (adj_ms / 1e3) / 1e6,
           "mlups_adjoint_with_recompute": nfluid / ((adj_ms + fwd_ms) / 1e3) / 1e6,
           "ms_per_adjoint_step": adj_ms, "ms_per_adjoint_step_fields_recomputed": adj_re_ms,
           "ms_per_forward_recompute": fwd_ms, "alg_bytes_per_node": b_alg,
           "alg_frac": nfluid * b_alg / (adj_ms / 1e3) / 1e9 / HBM_PEAK_GBS, "steps": steps}
    sim.close()
    del states
    torch.cuda.empty_cache()
    return out


def spinodal_stats(lbfe, torch, steps=20000, chunk=500,
                   forms=("fp64", "fp32", "fp16dev_f0fp32", "fp16dev")):
    """Precision forms on the 256^3 spinodal workload, all run side by side
    from the same initial density: the step at which max|rho - rho_FP64|
    first exceeds 1e-2 (rho_l - rho_v) (checked every `chunk` steps), and at
    the end, per form, the liquid volume fraction, the peak of the spherically
    averaged structure factor (wavenumber index k* and wavelength 256/k*),
    and the two peaks of the density histogram against the Maxwell pair."""
    geom, rho, u, desc = workload("spinodal", lbfe, torch)
    sims = {f: lbfe.Simulation(device="cuda:0", precision=f, check_every=chunk, **geom) for f in forms}
    for sim in sims.values():
        sim.init_density(torch.tensor(rho))
    ref = sims[forms[0]]
    rl, rv = ref.rho_l, ref.rho_v
    cross = {f: None for f in forms[1:]}
    t = 0
    while t < steps:
        for sim in sims.values():
            sim.step(chunk)
        t += chunk
        r0 = ref.fields()["rho"]
        for f in cross:
            if cross[f] is None:
                e = float((sims[f].fields()["rho"] - r0).abs().max()) / (rl - rv)
                if e > 1e-2:
                    cross[f] = t
        if t % 2000 == 0:
            print(f"[bench] spinodal statistics: step {t}", file=sys.stderr, flush=True)
    n = geom["nx"]
    k = torch.fft.fftfreq(n, d=1.0 / n, device="cuda:0").double()
    kr = torch.fft.rfftfreq(n, d=1.0 / n, device="cuda:0").double()
    kk = torch.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + kr[None, None, :] ** 2)
    shell = torch.round(kk).long().flatten()
    out = {"workload": desc + ", precision forms side by side", "steps": steps, "check_every": chunk,
           "rho_l": rl, "rho_v": rv, "forms": {}}
    mid = 0.5 * (rl + rv)
    for f, sim in sims.items():
        r = sim.fields()["rho"]
        P = torch.fft.rfftn(r - r.mean()).abs() ** 2
        sk = torch.zeros(int(shell.max()) + 1, dtype=torch.float64, device="cuda:0").index_add_(0, shell, P.flatten())
        cnt = torch.zeros_like(sk).index_add_(0, shell, torch.ones_like(P.flatten()))
        sk = sk / cnt.clamp(min=1)
        kpk = int(torch.argmax(sk[1:n // 2]).item()) + 1
        hist = torch.histc(r.float(), bins=800, min=0.0, max=float(1.2 * rl))
        centres = (torch.arange(800, device="cuda:0").double() + 0.5) * (1.2 * rl / 800)
        lo_mask, hi_mask = centres < mid, centres >= mid
        pk_v = float(centres[lo_mask][torch.argmax(hist[lo_mask])])
        pk_l = float(centres[hi_mask][torch.argmax(hist[hi_mask])])
        out["forms"][f] = {"liquid_fraction": float((r > mid).double().mean()), "k_peak": kpk,
                           "wavelength": n / kpk, "hist_peak_vapour": pk_v, "hist_peak_liquid": pk_l,
                           "step_pointwise_error_above_1e-2": cross.get(f)}
    for sim in sims.values():
        sim.close()
    torch.cuda.empty_cache()
    return out


def wetting_adjoint(lbfe, torch, steps=4000, every=200, neutral=0, phi=1.3):
    """The wetting workload's gradients at full size: 192x192x96, walls,
    phi wetting, omega3 = 1/2, 0.7 T_c, `steps` steps.  Loss L = sum over
    fluid nodes of (rho_T - rho_tgt)^2 with rho_tgt the final density of a
    run at phi + 0.05 plus seeded noise of 1e-3 (rho_l - rho_v).  dL/dkappa,
    dL/dphi and dL/drho0 at three nodes (liquid, interface, vapour) from the
    hand-written adjoint (uniform checkpoints every `every` steps, FP32 and
    FP64), against central differences of the FP64 forward.  neutral = 1:
    the same with neutral wetting (no contact-line window, so the step is
    smooth in the state), dL/dkappa and dL/drho0 only."""
    from paper_2504_03819_amd import autograd as lag, inputs
    geom, rho, u, desc = workload("wetting", lbfe, torch)
    T, om = geom["T"], geom["omega"]
    rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
    kappa = 0.02
    dev = "cuda:0"
    mode = lbfe.WET_NEUTRAL if neutral else lbfe.WET_PHI

    def forward64(k=kappa, w=phi, r0=None):
        sim = lbfe.Simulation(device=dev, nx=192, ny=192, nz=96, T=T, walls_z=1, wet_mode=mode,
                              wet_value=w, kappa=k, omega=om, check_every=steps)
        sim.init_density(torch.tensor(rho if r0 is None else r0))
        sim.step(steps)
        out = sim.fields()["rho"]
        sim.close()
        return out

    tgt = forward64(k=kappa * 1.05 if neutral else kappa, w=phi if neutral else phi + 0.05) + torch.tensor(1e-3 * (rl - rv) * inputs.uniform_noise(rho.shape, 1.0, 21),
                                                  device=dev)

    def loss(rT):
        return ((rT - tgt)[1:-1] ** 2).sum()

    nodes = [(48, 96, 96), (33, 96, 96), (80, 96, 96)]  # (z, y, x): liquid, near the interface, vapour
    res = {"workload": desc + f", {steps} steps, " + ("neutral wetting, loss against a kappa x 1.05 run plus noise"
                                                       if neutral else "loss against a phi + 0.05 run plus noise"),
           "phi": phi,
           "checkpoint_every": every, "nodes_zyx": nodes}
    for form in ("fp32", "fp64"):
        cfg = lag.StepConfig(nx=192, ny=192, nz=96, steps=steps, checkpoint_every=every, T=T, walls_z=1,
                             wet_mode=mode, precision=form, omega=om, device=dev,
                             keep_aux=form == "fp32")  # the FP64 segment without records fits in HBM
        r0 = torch.tensor(rho, device=dev, requires_grad=True)
        kap = torch.tensor(kappa, dtype=torch.float64, requires_grad=True)
        wet = torch.tensor(phi, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.time()
        L = loss(lag.simulate(r0, kap, wet, cfg))
        L.backward()
        torch.cuda.synchronize()
        res[form] = {"loss": float(L), "dL_dkappa": float(kap.grad), "dL_dphi": float(wet.grad),
                     "dL_drho0": [float(r0.grad[z, y, x]) for z, y, x in nodes], "seconds": time.time() - t0}
        del r0, L
        torch.cuda.empty_cache()
        print(f"[bench] wetting adjoint {form} done", file=sys.stderr, flush=True)
    hk, hp, hr = 2e-6, 1e-4, 1e-4
    fd = {"dL_dkappa": (float(loss(forward64(k=kappa + hk))) - float(loss(forward64(k=kappa - hk)))) / (2 * hk),
          "dL_dphi": 0.0 if neutral else
          (float(loss(forward64(w=phi + hp))) - float(loss(forward64(w=phi - hp)))) / (2 * hp)}
    d0 = []
    for z, y, x in nodes:
        rp, rm = rho.copy(), rho.copy()
        rp[z, y, x] += hr
        rm[z, y, x] -= hr
        d0.append((float(loss(forward64(r0=rp))) - float(loss(forward64(r0=rm)))) / (2 * hr))
    fd["dL_drho0"] = d0
    res["central_differences_fp64"] = fd
    for form in ("fp32", "fp64"):
        g = res[form]
        res[form]["rel_err_vs_fd"] = {
            "kappa": abs(g["dL_dkappa"] - fd["dL_dkappa"]) / abs(fd["dL_dkappa"]),
            "phi": abs(g["dL_dphi"] - fd["dL_dphi"]) / abs(fd["dL_dphi"]) if fd["dL_dphi"] else None,
            "rho0": [abs(a - b) / abs(b) for a, b in zip(g["dL_drho0"], d0)]}
    return res


def wetting_fd_table(lbfe, torch, steps=4000, every=200):
    """The wetting workload's gradient check at the five target angles (30,
    60, 90, 120, 150 deg: phi 1.62, 1.28, 1.0 and drho 0.9, 1.5 on the
    192x192x96 box, walls, 0.7 T_c, omega3 = 1/2): dL/dkappa, dL/d(wet) and
    dL/drho0 at three nodes from the hand-written adjoint (FP32 and FP64),
    against central differences of the FP64 forward.  The wetting rule of
    Eq. (38) switches branches where a wall node's average density crosses a
    window edge or the limiter binds; a difference quotient is the adjoint's
    derivative only if both probes take the same branches at every step.  So
    each probe records, per step, a fingerprint of its active set (which wall
    nodes are in the window and which are clamped), and a difference is
    reported only where the +h and -h fingerprints agree at every step;
    elsewhere the number of steps whose active sets differ is reported."""
    import numpy as np
    from paper_2504_03819_amd import autograd as lag, inputs
    geom, rho, u, desc = workload("wetting", lbfe, torch)
    T, om = geom["T"], geom["omega"]
    rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
    lo, hi = 0.05 * rl + 0.95 * rv, 0.95 * rl + 0.05 * rv
    kappa, dev = 0.02, "cuda:0"
    nx, ny, nz = 192, 192, 96
    g = np.random.Generator(np.random.PCG64(41))
    wts = torch.tensor(g.uniform(0.5, 1.5, (4, ny, nx)), device=dev)
    w1 = torch.tensor([1 / 6, 2 / 3, 1 / 6], dtype=torch.float64, device=dev)

    def fingerprint(r, mode, value):
        out = 0.0
        for k, z in enumerate((1, nz - 2)):
            pl = r[z]
            ave = sum(w1[a] * w1[b] * torch.roll(pl, shifts=(1 - a, 1 - b), dims=(0, 1))
                      for a in range(3) for b in range(3))
            win = (ave >= lo) & (ave <= hi)
            v = value * ave if mode == lbfe.WET_PHI else ave - value
            clamp = win & ((v < lo) | (v > hi))
            out += float((wts[2 * k] * win).sum() + (wts[2 * k + 1] * clamp).sum())
        return out

    def forward64(mode, value, k=kappa, r0=None, record=False):
        sim = lbfe.Simulation(device=dev, nx=nx, ny=ny, nz=nz, T=T, walls_z=1, wet_mode=mode, wet_value=value,
                              kappa=k, omega=om, check_every=steps)
        sim.init_density(torch.tensor(rho if r0 is None else r0))
        fp = []
        if record:
            for _ in range(steps):
                fp.append(fingerprint(sim.field(lbfe.FIELD_RHO), mode, value))
                sim.step(1)
        else:
            sim.step(steps)
        out = sim.fields()["rho"]
        sim.close()
        return out, fp

    cases = [(30, lbfe.WET_PHI, 1.62), (60, lbfe.WET_PHI, 1.28), (90, lbfe.WET_PHI, 1.0), (120, lbfe.WET_DELTA, 0.9),
             (150, lbfe.WET_DELTA, 1.5)]
    nodes = [(48, 96, 96), (33, 96, 96), (80, 96, 96)]
    res = {"workload": desc + f", {steps} steps, checkpoints every {every}", "nodes_zyx": nodes, "cases": []}
    for angle, mode, value in cases:
        dv = 0.05 if mode == lbfe.WET_PHI else 0.1
        tgt = forward64(mode, value + dv)[0] + torch.tensor(
            1e-3 * (rl - rv) * inputs.uniform_noise(rho.shape, 1.0, 21), device=dev)

        def loss(rT):
            return float(((rT - tgt)[1:-1] ** 2).sum())

        row = {"target_angle": angle, "mode": int(mode), "value": value}
        for form in ("fp32", "fp64"):
            cfg = lag.StepConfig(nx=nx, ny=ny, nz=nz, steps=steps, checkpoint_every=every, T=T, walls_z=1,
                                 wet_mode=mode, precision=form, omega=om, device=dev, keep_aux=form == "fp32")
            r0 = torch.tensor(rho, device=dev, requires_grad=True)
            kap = torch.tensor(kappa, dtype=torch.float64, requires_grad=True)
            wet = torch.tensor(value, dtype=torch.float64, requires_grad=True)
            L = ((lag.simulate(r0, kap, wet, cfg) - tgt)[1:-1] ** 2).sum()
            L.backward()
            row[form] = {"dL_dkappa": float(kap.grad), "dL_dwet": float(wet.grad),
                         "dL_drho0": [float(r0.grad[z, y, x]) for z, y, x in nodes]}
            del r0, L
            torch.cuda.empty_cache()

        def central(h, **kw):
            (rp, fpp), (rm, fpm) = (forward64(record=True, **{k: v(s) for k, v in kw.items()}) for s in (1, -1))
            crossings = sum(1 for a, b in zip(fpp, fpm) if a != b)
            return (loss(rp) - loss(rm)) / (2 * h), crossings

        fd = {}
        hk, hw, hr = 2e-6, 1e-5, 1e-4
        fd["kappa"] = central(hk, mode=lambda s: mode, value=lambda s: value, k=lambda s: kappa + s * hk)
        fd["wet"] = central(hw, mode=lambda s: mode, value=lambda s: value + s * hw)
        fd["rho0"] = []
        for z, y, x in nodes:
            def r0_of(sgn, z=z, y=y, x=x):
                r = rho.copy()
                r[z, y, x] += sgn * hr
                return r
            fd["rho0"].append(central(hr, mode=lambda s: mode, value=lambda s: value, r0=r0_of))
        row["fd_fp64"] = {"kappa": fd["kappa"][0], "wet": fd["wet"][0], "rho0": [v[0] for v in fd["rho0"]]}
        row["active_set_crossings"] = {"kappa": fd["kappa"][1], "wet": fd["wet"][1], "rho0": [v[1] for v in fd["rho0"]]}
        for form in ("fp32", "fp64"):
            gr = row[form]
            rel = {"kappa": abs(gr["dL_dkappa"] - fd["kappa"][0]) / abs(fd["kappa"][0]),
                   "wet": abs(gr["dL_dwet"] - fd["wet"][0]) / abs(fd["wet"][0]) if fd["wet"][0] else None,
                   "rho0": [abs(a - b[0]) / abs(b[0]) for a, b in zip(gr["dL_drho0"], fd["rho0"])]}
            row[form]["rel_err_vs_fd"] = rel
        res["cases"].append(row)
        print(f"[bench] fd table: {angle} deg done", file=sys.stderr, flush=True)
    return res


def wetting_angles(lbfe, torch, steps=40000, every=10000, form="fp64", cases=None, dump=None):
    """The wetting test of Sec. III C on the paper's geometry: Nx x Ny x Nz =
    128 x 256 x 256, solid planes z = 0 and 255 (halfway bounce-back), a
    droplet of radius 30 centred on the wall plane z = 0.5, 0.7 T_c, the
    third-order rate omega_3 = 1/2 (the wall reading of the oracle), and the
    three printed cases: neutral (phi = 1), phi = 1.6 and drho = 1.8.
    Reports the contact angle (oracle measurement) every `every` steps, the
    spread of mu over the fluid, and the mass drift; with `dump` a directory,
    the central x-z and y-z density planes of every report go to an .npz
    file there."""
    from oracle import phys
    from paper_2504_03819_amd import inputs
    T = 0.7 * 8 * (9 / 392) / (27 * (2 / 21))
    nx, ny, nz = 128, 256, 256
    cases = cases or [("neutral", lbfe.WET_PHI, 1.0, 89.9), ("phi 1.6", lbfe.WET_PHI, 1.6, 33.5),
                      ("drho 1.8", lbfe.WET_DELTA, 1.8, 153.4)]
    out = {"workload": "sessile droplet 128x256x256 (Nx x Ny x Nz), walls z=0,255, r=30 at z=0.5, T=0.7Tc, "
                       f"omega3=0.5, {form}", "steps": steps, "cases": {}}
    for label, mode, value, paper in cases:
        sim = lbfe.Simulation(device="cuda:0", nx=nx, ny=ny, nz=nz, T=T, walls_z=1, wet_mode=mode, wet_value=value,
                              omega=[1.0, 1.0, 1.0, 0.5] + [1.0] * 7, precision=form, check_every=every)
        rl, rv = sim.rho_l, sim.rho_v
        rho = inputs.sphere((nz, ny, nx), (nx / 2, ny / 2, 0.5), 30.0, rl, rv)
        rho[0] = rho[-1] = rv
        sim.init_density(torch.tensor(rho))
        m0 = sim.reduce()[0]
        traj = []
        done = 0
        while done < steps:
            sim.step(every)
            done += every
            f = sim.fields()
            r = f["rho"].cpu().numpy()
            mu = f["mu"][1:-1].cpu().numpy()
            th, zc, Rf = phys.contact_angle(r, rl, rv)
            traj.append({"step": done, "theta": round(th, 3), "cap_radius": round(Rf, 2),
                         "mu_spread": float(mu.max() - mu.min()), "rho_max": float(r.max())})
            if dump:
                import numpy as np
                os.makedirs(dump, exist_ok=True)
                np.savez_compressed(os.path.join(dump, f"wet_{label.replace(' ', '_')}_{done}.npz"),
                                    xz=r[:, ny // 2, :], yz=r[:, :, nx // 2], rho_l=rl, rho_v=rv)
            print(f"[bench] wetting {label}: step {done} theta {th:.2f}", file=sys.stderr, flush=True)
        out["cases"][label] = {"mode": int(mode), "value": value, "paper_theta": paper, "trajectory": traj,
                               "mass_drift": (sim.reduce()[0] - m0) / m0}
        sim.close()
        torch.cuda.empty_cache()
    return out


def time_collision_adjoint(lbfe, torch, forward=5000, adjoint=500, snapshots=8, form="fp32"):
    """512^3 head-on collision in a storage form (FP32 by default; the
    adjoint runs in the form's compute precision): `forward` steps, then the adjoint of
    the last `adjoint` steps from the stored state f(T - adjoint) with the
    binomial checkpoint schedule (`snapshots` states held), loss
    L = sum (rho_T - rho_0)^2.  Reports forward and backward times, the
    recomputed steps and the peak device memory."""
    from paper_2504_03819_amd.autograd import reverse_binomial
    n = 512
    T = 0.85 * 8 * (9 / 392) / (27 * (2 / 21))
    rl, rv = lbfe.coexistence(9 / 392, 2 / 21, 1.0, T)
    from paper_2504_03819_amd import inputs
    rho0, u0 = inputs.head_on_collision(rl, rv)
    torch.cuda.reset_peak_memory_stats()
    sim = lbfe.Simulation(device="cuda:0", nx=n, ny=n, nz=n, T=T, precision=form, adjoint=1, check_every=500)
    r0 = torch.tensor(rho0, device="cuda:0")
    sim.init_density(r0, torch.tensor(u0))
    del rho0, u0
    t0 = forward - adjoint
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record(sim.stream)
    done = 0
    while done < t0:
        k = min(500, t0 - done)
        sim.step(k)
        done += k
        print(f"[bench] collision forward step {done}", file=sys.stderr, flush=True)
    state = sim.get_state()
    sim.step(adjoint)
    e[1].record(sim.stream)
    rho_T = sim.fields()["rho"]
    e[2].record(sim.stream)
    sim.adjoint_seed(2.0 * (rho_T - r0))
    del rho_T
    print("[bench] collision adjoint", file=sys.stderr, flush=True)
    stats = reverse_binomial(sim, state, t0, forward, snapshots)
    e[3].record(sim.stream)
    torch.cuda.synchronize()
    fwd_ms = e[0].elapsed_time(e[1]) / forward
    bwd_ms = e[2].elapsed_time(e[3])
    adj_ms = (bwd_ms - stats["recompute_steps"] * fwd_ms) / adjoint
    g = sim.adjoint_grads()
    nodes = n ** 3
    out = {"workload": f"head-on collision 512^3 {form}, two r=64 droplets 160 apart at +-0.04, T=0.85Tc",
           "forward_steps": forward, "adjoint_steps": adjoint, "snapshots": snapshots,
           "recompute_steps": stats["recompute_steps"], "ms_per_forward_step": fwd_ms,
           "mlups_forward": nodes / (fwd_ms / 1e3) / 1e6, "backward_s": bwd_ms / 1e3,
           "ms_per_adjoint_step_excl_recompute": adj_ms, "mlups_adjoint": nodes / (adj_ms / 1e3) / 1e6,
           "peak_device_GB": torch.cuda.max_memory_allocated() / 1e9, "dL_dkappa": g["kappa"]}
    sim.close()
    return out


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rho, u, geom, seconds_target=20.0, box=128):
    """The CPU oracle as it stands, timed on a bounded sample of the
    workload: grids above box^3 are sampled by a periodic box^3 sub-box cut
    from the centre of the initial fields (the oracle's cost per node does
    not depend on the box size or the values, so its MLUPS carries over to
    the full grid); about 10-30 s of CPU work."""
    import torch
    from oracle import lbm
    nx, ny, nz = geom["nx"], geom["ny"], geom["nz"]
    sample = "full grid"
    if nx * ny * nz > box ** 3 and not geom.get("walls_z") and geom.get("solid") is None:
        cz, cy, cx = nz // 2, ny // 2, nx // 2
        h = box // 2
        rho = rho[cz - h:cz + h, cy - h:cy + h, cx - h:cx + h].copy()
        u = None if u is None else u[:, cz - h:cz + h, cy - h:cy + h, cx - h:cx + h].copy()
        nx = ny = nz = box
        sample = f"periodic {box}^3 sub-box cut from the centre of the {geom['nx']}x{geom['ny']}x{geom['nz']} initial fields"
    p = lbm.Params(nx, ny, nz, walls_z=bool(geom.get("walls_z", 0)), T=geom["T"],
                   wet_mode=geom.get("wet_mode", 0), wet_value=geom.get("wet_value", 1.0))
    f = lbm.init(torch.tensor(rho), p, None if u is None else torch.tensor(u))
    steps, t0 = 0, time.time()
    while True:
        f = lbm.step(f, p)
        steps += 1
        if time.time() - t0 > seconds_target or steps >= 50:
            break
    dt = time.time() - t0
    nfluid = nx * ny * (nz - (2 if geom.get("walls_z") else 0))
    return {"value": nfluid * steps / dt / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(),
            "kind": "oracle", "cpu_model": host_cpu_model(),
            "sample": f"{steps} steps of the {sample} ({dt:.1f} s); MLUPS per fluid-node update, "
                      f"extrapolated to the full grid" if sample != "full grid"
                      else f"{steps} full-size steps of the same workload ({dt:.1f} s)"}


def copy_calibration(torch, gib=1):
    """A plain device copy of known size (read gib GiB, write gib GiB): its
    FETCH_SIZE / WRITE_SIZE counters calibrate the collide kernel's."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def copy_bandwidth(torch, gib=4, reps=10):
    """Attainable HBM bandwidth: a streaming copy of gib GiB through torch's
    vectorised elementwise kernel (b = 1 * a; read + write bytes over the
    mean time of `reps` copies, HIP events).  The runtime's own
    device-to-device copy is slower on this GPU (4.6-5.2 TB/s against
    6.0-6.2), so it is not used as the reference."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (ms / 1e3) / 1e9


def _read_counter_csv(path, counter):
    """Per-kernel list of one counter's values (KiB per dispatch) from a
    rocprofv3 counter_collection.csv."""
    import csv
    vals = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter:
                continue
            vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return vals


def summarize_counters(fetch_csv, write_csv, form, workload_name, out_path):
    """Calibrated HBM bytes per launch of every step kernel from two rocprofv3
    --pmc passes (FETCH_SIZE, then WRITE_SIZE) of
    `bench.py --copy-calib --forms <form> --no-cpu-baseline --no-adjoint`;
    the dominant kernel is the fused collide-stream kernel if the run has
    one, else the moment-state collide pass, else the two-pass
    collide-stream kernel."""
    fetch_all = _read_counter_csv(fetch_csv, "FETCH_SIZE")
    write_all = _read_counter_csv(write_csv, "WRITE_SIZE")
    copy_k = [k for k in fetch_all if "copybuffer" in k.lower()]
    dom = [k for k in fetch_all if "k_fused" in k] or [k for k in fetch_all if re.search(r"k_mstate<\d+, 2,", k)] \
        or [k for k in fetch_all if "k_collide" in k]
    if not copy_k or not dom:
        raise SystemExit(f"kernels not found: {sorted(fetch_all)}")
    # the 1 GiB copies are the largest copy dispatches of the run
    gib_kib = (1 << 30) / 1024.0
    f_fac = gib_kib / max(max(fetch_all[k]) for k in copy_k)
    w_fac = gib_kib / max(max(write_all[k]) for k in copy_k if k in write_all)
    fetch = {k: sum(v) / len(v) for k, v in fetch_all.items()}
    write = {k: sum(v) / len(v) for k, v in write_all.items()}
    launches = {k: len(v) for k, v in fetch_all.items()}
    res = {"form": form, "workload": workload_name, "source_hash": kernel_source_hash(),
           "dominant_kernel": re.sub(r"^void |lbfe::\(anonymous namespace\)::|\(lbfe::KP.*$", "", dom[0]),
           "fetch_kib_per_launch": fetch[dom[0]], "write_kib_per_launch": write[dom[0]],
           "copy_fetch_factor": f_fac, "copy_write_factor": w_fac,
           "bytes_per_launch": (fetch[dom[0]] * f_fac + write[dom[0]] * w_fac) * 1024.0,
           "kernels": {"fetch_kib": fetch, "write_kib": write, "launches": launches}}
    json.dump(res, open(out_path, "w"), indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "kernels"}))


def step_kernels(c):
    """The kernels of one step in a counter summary: the step-path kernels
    launched as often as the dominant kernel (once per step); kernels that
    ran fewer times (the initial refresh of the moments, the initialiser)
    are not part of a step."""
    launches = c["kernels"]["launches"]
    dom = [k for k in launches if re.sub(r"^void |lbfe::\(anonymous namespace\)::|\(lbfe::KP.*$", "", k)
           == c["dominant_kernel"]]
    n = launches[dom[0]]
    return {k for k, m in launches.items() if m == n and any(s in k for s in STEP_KERNELS)}


def summarize_adjoint_counters(fetch_csv, write_csv, out_path):
    """Calibrated HBM bytes per adjoint step from two rocprofv3 --pmc passes
    (FETCH_SIZE, then WRITE_SIZE) of `bench.py --adjoint-only --copy-calib`:
    every dispatch of the adjoint-step kernels summed, over the number of
    collision-adjoint dispatches (one per adjoint step)."""
    import csv
    rows = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        with open(path) as fh:
            rows[counter] = [(r["Kernel_Name"], float(r["Counter_Value"])) for r in csv.DictReader(fh)
                             if r.get("Counter_Name") == counter]
    gib_kib = (1 << 30) / 1024.0
    fac = {}
    for counter, rs in rows.items():
        copies = [v for k, v in rs if "copybuffer" in k.lower()]
        if not copies:
            raise SystemExit(f"no copy dispatch in the {counter} pass")
        fac[counter] = gib_kib / max(copies)
    steps = sum(1 for k, _ in rows["FETCH_SIZE"] if "k_adj_collide" in k)
    if steps == 0:
        raise SystemExit("no collision-adjoint dispatch in the run")
    per_kernel = {}
    for counter, rs in rows.items():
        for k, v in rs:
            if any(s in k for s in ADJ_STEP_KERNELS):
                name = re.sub(r"^void |lbfe::\(anonymous namespace\)::|\(lbfe::KP.*$", "", k)
                d = per_kernel.setdefault(name, {"FETCH_SIZE": 0.0, "WRITE_SIZE": 0.0})
                d[counter] += v * fac[counter] * 1024.0 / steps
    res = {"source_hash": kernel_source_hash(), "adjoint_steps": steps,
           "copy_fetch_factor": fac["FETCH_SIZE"], "copy_write_factor": fac["WRITE_SIZE"],
           "bytes_per_adjoint_step": sum(d["FETCH_SIZE"] + d["WRITE_SIZE"] for d in per_kernel.values()),
           "kernels_bytes_per_step": per_kernel}
    json.dump(res, open(out_path, "w"), indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "kernels_bytes_per_step"}))


def adjoint_achieved(adj):
    """Counter-based HBM fraction of an adjoint step (the committed counter
    file, while it matches the sources) added to the adjoint leg."""
    if not os.path.exists(ADJ_COUNTERS):
        return
    c = json.load(open(ADJ_COUNTERS))
    if c.get("source_hash") != kernel_source_hash():
        return
    adj["traffic_per_step"] = c["bytes_per_adjoint_step"]
    adj["achieved_frac"] = c["bytes_per_adjoint_step"] / (adj["ms_per_adjoint_step"] / 1e3) / 1e9 / HBM_PEAK_GBS


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="collision")
    ap.add_argument("--forms", default="fp64,fp32,fp16dev_f0fp32,fp64_state,fp32_state",
                    help="storage forms; the first is the headline (fp16dev is reported with valid: false)")
    ap.add_argument("--timed-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--copy-calib", action="store_true", help="run a 1 GiB device copy first (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--counters-out", default=COUNTERS,
                    help="where --summarize-counters writes (the bench line reads profiles/collide_counters.json)")
    ap.add_argument("--summarize-adjoint-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--adjoint-only", action="store_true", help="time only the adjoint leg, print its JSON")
    ap.add_argument("--adjoint-steps", type=int, default=20)
    ap.add_argument("--adjoint-form", default="fp32", help="storage form of --collision-adjoint")
    ap.add_argument("--collision-adjoint", nargs=3, type=int, metavar=("FORWARD", "ADJOINT", "SNAPSHOTS"),
                    help="time the 512^3 collision with a binomial-checkpointed adjoint of its last steps")
    ap.add_argument("--wetting-adjoint", nargs=3, type=int, metavar=("STEPS", "CHECKPOINT_EVERY", "NEUTRAL"),
                    help="192x192x96 wetting gradients (FP32 and FP64 adjoint) against central differences")
    ap.add_argument("--wetting-angles", nargs=2, type=int, metavar=("STEPS", "EVERY"),
                    help="Sec. III C wetting on the paper's 128x256x256 geometry: contact angles of the printed cases")
    ap.add_argument("--wetting-cases", default="neutral,phi 1.6,drho 1.8")
    ap.add_argument("--wetting-fd-table", nargs=2, type=int, metavar=("STEPS", "CHECKPOINT_EVERY"),
                    help="adjoint vs central differences at the five target angles, with the active-set check")
    ap.add_argument("--dump-planes", default=None, help="directory for the central density planes (--wetting-angles)")
    ap.add_argument("--spinodal-stats", nargs=2, type=int, metavar=("STEPS", "CHECK_EVERY"),
                    help="256^3 spinodal in every storage form side by side: error onset and end statistics")
    args = ap.parse_args()
    if args.summarize_adjoint_counters:
        summarize_adjoint_counters(*args.summarize_adjoint_counters, out_path=ADJ_COUNTERS)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, form=args.forms.split(",")[0], workload_name=args.workload,
                           out_path=args.counters_out)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        sys.stderr.write("bench.py: runs on one GPU only; a multi-GPU (z-slab) decomposition "
                         "is designed but not built, so --gpus must be 1.\n")
        sys.exit(2)

    import torch
    from paper_2504_03819_amd import lbfe
    if not torch.cuda.is_available():
        sys.stderr.write("bench.py needs a GPU\n")
        sys.exit(1)
    if args.wetting_adjoint:
        print(json.dumps(wetting_adjoint(lbfe, torch, *args.wetting_adjoint)), flush=True)
        return
    if args.spinodal_stats:
        print(json.dumps(spinodal_stats(lbfe, torch, *args.spinodal_stats)), flush=True)
        return
    if args.wetting_fd_table:
        print(json.dumps(wetting_fd_table(lbfe, torch, *args.wetting_fd_table)), flush=True)
        return
    if args.wetting_angles:
        allc = {"neutral": ("neutral", lbfe.WET_PHI, 1.0, 89.9), "phi 1.6": ("phi 1.6", lbfe.WET_PHI, 1.6, 33.5),
                "drho 1.8": ("drho 1.8", lbfe.WET_DELTA, 1.8, 153.4)}
        cases = [allc[c] for c in args.wetting_cases.split(",")]
        print(json.dumps(wetting_angles(lbfe, torch, *args.wetting_angles, cases=cases, dump=args.dump_planes)),
              flush=True)
        return
    if args.collision_adjoint:
        print(json.dumps(time_collision_adjoint(lbfe, torch, *args.collision_adjoint, form=args.adjoint_form)),
              flush=True)
        return
    if args.adjoint_only:
        if args.copy_calib:
            copy_calibration(torch)
        adj = time_adjoint(lbfe, torch, steps=args.adjoint_steps)
        adjoint_achieved(adj)
        print(json.dumps(adj), flush=True)
        return
    geom, rho, u, desc = workload(args.workload, lbfe, torch)
    if args.copy_calib:
        copy_calibration(torch)
    forms = [f for f in args.forms.split(",") if f]
    results = {}
    for form in forms:
        print(f"[bench] {desc}: timing {form}", file=sys.stderr, flush=True)
        results[form] = time_form(lbfe, torch, geom, rho, u, form, args.steps, args.warmup, args.timed_steps)
    head = forms[0]
    r = results[head]
    dom = DOMINANT[r["step_path"]]
    roof = {
        "bound": "hbm",
        "kernel": dom,
        "achieved": round(r["collide_alg_GBps"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(r["collide_alg_GBps"] / HBM_PEAK_GBS, 4),
        "traffic": None,
        "alg_bytes_per_node": alg_bytes_per_node(head),
        "step_alg_GBps": round(r["step_alg_GBps"], 1),
        "step_alg_frac": round(r["step_alg_frac"], 4),
    }
    if os.path.exists(COUNTERS):
        c = json.load(open(COUNTERS))
        if c.get("source_hash") == kernel_source_hash() and c.get("workload") == args.workload \
                and c.get("form") == head:
            roof["traffic"] = c.get("bytes_per_launch")
            # achieved HBM fraction of the whole step: calibrated counter
            # bytes of every kernel of one step over the measured step time
            ff, wf = c["copy_fetch_factor"], c["copy_write_factor"]
            per_step = step_kernels(c)
            tb = sum(v * ff for k, v in c["kernels"]["fetch_kib"].items() if k in per_step)
            tb += sum(v * wf for k, v in c["kernels"]["write_kib"].items() if k in per_step)
            roof["step_traffic"] = tb * 1024.0
            roof["step_achieved_frac"] = round(tb * 1024.0 / (r["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    print("[bench] device copy bandwidth", file=sys.stderr, flush=True)
    cbw = copy_bandwidth(torch)
    roof["copy_GBps"] = round(cbw, 1)
    roof["frac_of_copy"] = round(r["collide_alg_GBps"] / cbw, 4)
    adj = None
    if not args.no_adjoint:
        print("[bench] timing the adjoint (wetting workload, FP32)", file=sys.stderr, flush=True)
        adj = time_adjoint(lbfe, torch, steps=args.adjoint_steps)
        adjoint_achieved(adj)
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(rho, u, geom)
    line = {
        "metric": METRIC,
        "value": round(r["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32"}.get(form_params(head)["precision"], "f16-store/f32"),
        "data": "synthetic",
        "config": {"workload": desc, "grid": [geom["nx"], geom["ny"], geom["nz"]], "form": head,
                   "step_path": r["step_path"], "nfluid": r["nfluid"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in results.items()},
        "adjoint": None if adj is None else {k: (round(v, 4) if isinstance(v, float) else v) for k, v in adj.items()},
        "source_hash": kernel_source_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
