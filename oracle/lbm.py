"""FP64 oracle of one time step of the chemical-potential-based free-energy
LB model on D3Q27 with central-moment MRT collision (arXiv:2504.03819,
Sec. II B) and the wetting boundary of Sec. III C.

State layout: f has shape (27, nz, ny, nx), direction order from
``oracle.lattice``.  With walls, z = 0 and z = nz-1 are solid planes whose
populations are kept at zero; all other nodes are fluid.  An arbitrary solid
voxel mask (``Params.solid``) generalises the planes: the halfway bounce-back
and the wetting boundary of Eqs. (36)-(38) are written in the paper for any
solid node x_s, and the flat walls are the case of a mask holding the two
planes.

Readings of points the paper leaves open (each also listed in the design
notes of the repository):
  * Discrete operators (the paper does not state them): the isotropic
    D3Q27 stencils  grad_h g = 3 sum_i w_i c_i g(x+c_i)  and
    lap_h g = 6 sum_i w_i [g(x+c_i) - g(x)].
  * All auxiliary fields of step t come from the post-streaming f(t).
  * The velocity in the central-moment shift and in the Q terms is the
    force-corrected u of Eq. (11); mu inside p_m is the full mu of Eq. (32).
  * omega_1 is evaluated per node from local rho and p_m.
  * Wall order: rho(fluid) -> rho_ave(x_s) -> rho(x_s) -> mu(fluid)
    -> mu(x_s) -> grad mu(fluid); u = 0 and hence phi = 0 at solid nodes;
    neighbours outside the domain count as solid (s_w = 0); window and
    limiter bounds are inclusive and use the Maxwell pair at T.
  * Initial populations: the generalized equilibrium of Eq. (20) at
    (rho0, u0, p_m(mu[rho0])).

The step is plain torch (CPU, float64) so that autograd can differentiate it.
"""
from dataclasses import dataclass, field
from itertools import product
from math import comb

import torch

from . import eos
from .lattice import C, OPP, Q, W_T

NEUTRAL, PHI, DELTA = 0, 1, 2
DT = torch.float64


@dataclass
class Params:
    nx: int
    ny: int
    nz: int
    walls_z: bool = False
    a: float = eos.PAPER["a"]
    b: float = eos.PAPER["b"]
    R: float = eos.PAPER["R"]
    T: float = 0.7 * eos.critical_point(eos.PAPER["a"], eos.PAPER["b"], eos.PAPER["R"])[1]
    kappa: float = eos.PAPER["kappa"]
    nu: float = eos.PAPER["nu"]
    # omega[0], omega[2..10]; omega[1] is derived from nu per node (Sec. II B)
    omega: list = field(default_factory=lambda: [1.0] * 11)
    corr4: bool = True
    rho_l: float = 0.0     # 0 -> Maxwell pair at T
    rho_v: float = 0.0
    wet_mode: int = NEUTRAL
    wet_value: float = 1.0
    # tangential velocities (ux, uy) of the bottom (z = 0) and top (z = nz-1)
    # walls; moving walls use the momentum-corrected halfway bounce-back
    wall_u: tuple = (0.0, 0.0, 0.0, 0.0)
    # optional solid voxel mask, bool (nz, ny, nx), True = solid; combined
    # with the wall planes when both are given
    solid: object = None

    def coexistence(self):
        if self.rho_l > 0 and self.rho_v > 0:
            return self.rho_l, self.rho_v
        return eos.maxwell(self.a, self.b, self.R, self.T)


# --------------------------------------------------------------------------
# neighbour access and discrete operators
# --------------------------------------------------------------------------
def at(g, c):
    """Value of field g (nz, ny, nx) at x + c, periodic index wrap.  With
    walls the wrap only ever reaches solid planes, which callers mask."""
    return torch.roll(g, shifts=(-c[2], -c[1], -c[0]), dims=(0, 1, 2))


def grad_h(g):
    """Isotropic gradient 3 * sum_i w_i c_i g(x + c_i); returns (3, nz, ny, nx)."""
    out = torch.zeros((3,) + tuple(g.shape), dtype=DT)
    for i, c in enumerate(C):
        if c == (0, 0, 0):
            continue
        gi = at(g, c)
        for a in range(3):
            if c[a] != 0:
                out[a] = out[a] + 3.0 * W_T[i] * c[a] * gi
    return out


def lap_h(g):
    """Isotropic Laplacian 6 * sum_i w_i (g(x + c_i) - g(x))."""
    out = torch.zeros_like(g)
    for i, c in enumerate(C):
        if c == (0, 0, 0):
            continue
        out = out + 6.0 * W_T[i] * (at(g, c) - g)
    return out


def has_solid(p: Params):
    return bool(p.walls_z) or p.solid is not None


def fluid_mask(p: Params):
    """Fluid indicator s (1 fluid, 0 solid) of the wall planes and the
    solid mask."""
    s = torch.ones((p.nz, p.ny, p.nx), dtype=DT)
    if p.walls_z:
        s[0] = 0.0
        s[-1] = 0.0
    if p.solid is not None:
        s = torch.where(torch.as_tensor(p.solid, dtype=torch.bool), torch.zeros_like(s), s)
    return s


def wall_average(g, s):
    """Eqs. (36)/(37): sum_i w_i s_w g(x+c_i) / sum_i w_i s_w, evaluated at
    every node (only used at solid nodes).  s is the fluid indicator; values
    of g at non-fluid nodes never enter.  A solid node without fluid
    neighbours (inside a thick solid) gets 0: no stencil of a fluid node
    reaches it."""
    num = torch.zeros_like(g)
    den = torch.zeros_like(g)
    for i, c in enumerate(C):
        fl = at(s, c) > 0
        num = num + torch.where(fl, W_T[i] * at(g, c), torch.zeros_like(g))
        den = den + torch.where(fl, torch.full_like(g, W_T[i]), torch.zeros_like(g))
    return torch.where(den > 0, num / torch.where(den > 0, den, torch.ones_like(den)), torch.zeros_like(g))


# --------------------------------------------------------------------------
# closure, Eq. (32)
# --------------------------------------------------------------------------
def mu_bulk(rho, p: Params):
    return p.R * p.T * (torch.log(rho / (1.0 - p.b * rho)) + 1.0 / (1.0 - p.b * rho)) - 2.0 * p.a * rho


# --------------------------------------------------------------------------
# moments: Eq. (18) raw moments, Eq. (19) central moments
# --------------------------------------------------------------------------
IDX = list(product(range(3), range(3), range(3)))   # (alpha, beta, gamma), gamma fastest


def moment_matrix():
    """M[(abc), i] = cx^a cy^b cz^c (Eq. (18))."""
    M = torch.zeros((27, 27), dtype=DT)
    for r, (a, b, g) in enumerate(IDX):
        for i, c in enumerate(C):
            M[r, i] = float(c[0] ** a * c[1] ** b * c[2] ** g)
    return M


M_RAW = moment_matrix()
M_INV = torch.linalg.inv(M_RAW)


def _shift(mom, u, sign):
    """Binomial change of origin of a (27, ...) moment array: with sign=-1
    raw -> central (Eq. (19) expanded via the binomial theorem applied to
    (c - u)^n), with sign=+1 central -> raw (c^n = ((c - u) + u)^n)."""
    ux, uy, uz = sign * u[0], sign * u[1], sign * u[2]
    out = []
    for (a, b, g) in IDX:
        acc = torch.zeros_like(mom[0])
        for (a2, b2, g2) in IDX:
            if a2 > a or b2 > b or g2 > g:
                continue
            coef = comb(a, a2) * comb(b, b2) * comb(g, g2)
            acc = acc + coef * ux ** (a - a2) * uy ** (b - b2) * uz ** (g - g2) * mom[IDX.index((a2, b2, g2))]
        out.append(acc)
    return torch.stack(out)


def raw_moments(f):
    return torch.einsum("ri,i...->r...", M_RAW, f)


def central_moments(f, u):
    """Eq. (19) computed through the raw moments of Eq. (18) (Sec. II B)."""
    return _shift(raw_moments(f), u, -1.0)


def populations_from_central(k, u):
    """Inverse of central_moments: CM -> RM -> f (Sec. II B, last paragraph)."""
    m = _shift(k, u, +1.0)
    return torch.einsum("ir,r...->i...", M_INV, m)


def central_moments_direct(f, u):
    """Eq. (19) summed literally over the 27 directions (brute force)."""
    out = []
    for (a, b, g) in IDX:
        acc = torch.zeros_like(f[0])
        for i, c in enumerate(C):
            acc = acc + f[i] * (c[0] - u[0]) ** a * (c[1] - u[1]) ** b * (c[2] - u[2]) ** g
        out.append(acc)
    return torch.stack(out)


def K(k, a, b, g):
    return k[IDX.index((a, b, g))]


# --------------------------------------------------------------------------
# equilibrium central moments, Eq. (20)
# --------------------------------------------------------------------------
def equilibrium_central(rho, pm):
    cs2 = 1.0 / 3.0
    rows = []
    for (a, b, g) in IDX:
        if (a, b, g) == (0, 0, 0):
            rows.append(rho)
        elif sorted((a, b, g)) == [0, 0, 2]:
            rows.append(pm)
        elif sorted((a, b, g)) == [0, 2, 2]:
            rows.append(pm * cs2)
        elif (a, b, g) == (2, 2, 2):
            rows.append(pm * cs2 * cs2)
        else:
            rows.append(torch.zeros_like(rho))
    return torch.stack(rows)


# --------------------------------------------------------------------------
# collision in central-moment space, Eqs. (21)-(26)
# --------------------------------------------------------------------------
def _solve_combos(rows, rhs):
    """Solve a small set of linear combination equations of the form
    sum_j rows[r][j] * x_j = rhs[r] for the unknown moments x_j."""
    A = torch.tensor(rows, dtype=DT)
    Ainv = torch.linalg.inv(A)
    return [sum(Ainv[j, r] * rhs[r] for r in range(len(rhs))) for j in range(len(rows))]


def collide(k, F, Qd, pm, w):
    """Post-collision central moments.  k: (27, ...) pre-collision CMs; F:
    (3, ...) force; Qd: (Q200, Q020, Q002, Q220, Q202, Q022) correction terms;
    pm: modified pressure; w: list of 11 rates, w[1] may be a field."""
    cs2 = 1.0 / 3.0
    Fx, Fy, Fz = F[0], F[1], F[2]
    Q200, Q020, Q002, Q220, Q202, Q022 = Qd
    out = {}
    kk = lambda a, b, g: K(k, a, b, g)
    # zeroth order: mass is conserved
    out[(0, 0, 0)] = kk(0, 0, 0)
    # first order, Eq. (21)
    for (idx, Fa) in (((1, 0, 0), Fx), ((0, 1, 0), Fy), ((0, 0, 1), Fz)):
        out[idx] = (1 - w[0]) * kk(*idx) + (1 - w[0] / 2) * Fa
    # second order, Eq. (22)
    for idx in ((1, 1, 0), (0, 1, 1), (1, 0, 1)):
        out[idx] = (1 - w[1]) * kk(*idx)
    k200, k020, k002 = kk(2, 0, 0), kk(0, 2, 0), kk(0, 0, 2)
    r1 = (1 - w[1]) * (k200 - k020) + (1 - w[1] / 2) * (Q200 - Q020)
    r2 = (1 - w[1]) * (k200 - k002) + (1 - w[1] / 2) * (Q200 - Q002)
    r3 = (1 - w[2]) * (k200 + k020 + k002) + 3 * w[2] * pm + (1 - w[2] / 2) * (Q200 + Q020 + Q002)
    x = _solve_combos([[1, -1, 0], [1, 0, -1], [1, 1, 1]], [r1, r2, r3])
    out[(2, 0, 0)], out[(0, 2, 0)], out[(0, 0, 2)] = x
    # third order, Eq. (23)
    for (ia, ib, Fa) in (((1, 2, 0), (1, 0, 2), Fx), ((2, 1, 0), (0, 1, 2), Fy), ((2, 0, 1), (0, 2, 1), Fz)):
        rp = (1 - w[3]) * (kk(*ia) + kk(*ib)) + 2 * (1 - w[3] / 2) * Fa * cs2
        rm = (1 - w[4]) * (kk(*ia) - kk(*ib))
        x = _solve_combos([[1, 1], [1, -1]], [rp, rm])
        out[ia], out[ib] = x
    out[(1, 1, 1)] = (1 - w[5]) * kk(1, 1, 1)
    # fourth order, Eq. (24)
    k220, k202, k022 = kk(2, 2, 0), kk(2, 0, 2), kk(0, 2, 2)
    r1 = (1 - w[6]) * (k220 - 2 * k202 + k022) + (1 - w[6] / 2) * (Q220 - 2 * Q202 + Q022)
    r2 = (1 - w[6]) * (k220 + k202 - 2 * k022) + (1 - w[6] / 2) * (Q220 + Q202 - 2 * Q022)
    r3 = (1 - w[7]) * (k220 + k202 + k022) + 3 * w[7] * pm * cs2 + (1 - w[7] / 2) * (Q220 + Q202 + Q022)
    x = _solve_combos([[1, -2, 1], [1, 1, -2], [1, 1, 1]], [r1, r2, r3])
    out[(2, 2, 0)], out[(2, 0, 2)], out[(0, 2, 2)] = x
    for idx in ((2, 1, 1), (1, 2, 1), (1, 1, 2)):
        out[idx] = (1 - w[8]) * kk(*idx)
    # fifth order, Eq. (25)
    for (idx, Fa) in (((1, 2, 2), Fx), ((2, 1, 2), Fy), ((2, 2, 1), Fz)):
        out[idx] = (1 - w[9]) * kk(*idx) + (1 - w[9] / 2) * Fa * cs2 * cs2
    # sixth order, Eq. (26)
    out[(2, 2, 2)] = (1 - w[10]) * kk(2, 2, 2) + w[10] * pm * cs2 * cs2
    return torch.stack([out[idx] for idx in IDX])


# --------------------------------------------------------------------------
# the step
# --------------------------------------------------------------------------
def wall_density(rho_f, s, p: Params):
    """Eqs. (37)-(38) with the contact-line window and limiter.  rho_f holds
    fluid densities (values at solid nodes are ignored).  Returns rho with
    solid nodes filled in."""
    rl, rv = p.coexistence()
    lo, hi = 0.05 * rl + 0.95 * rv, 0.95 * rl + 0.05 * rv
    rave = wall_average(rho_f, s)
    inwin = (rave >= lo) & (rave <= hi)
    if p.wet_mode == PHI:
        mod = torch.clamp(p.wet_value * rave, lo, hi)
    elif p.wet_mode == DELTA:
        mod = torch.clamp(rave - p.wet_value, lo, hi)
    else:
        mod = rave
    rho_s = torch.where(inwin, mod, rave)
    return torch.where(s > 0, rho_f, rho_s)


def aux_fields(f, p: Params):
    """Steps S1-S6 on the post-streaming state f(t): returns a dict with rho,
    j, mu, G (grad mu), F, u, pm, phi, Q (6 terms), omega1.  Solid nodes
    carry rho(x_s), mu(x_s) and zero u, F, phi, Q."""
    s = fluid_mask(p)
    fluid = s > 0
    rho_f = f.sum(0)
    j = torch.einsum("ia,i...->a...", torch.tensor(C, dtype=DT), f)
    # S2: density at solid nodes
    rho = wall_density(rho_f, s, p) if has_solid(p) else rho_f
    # S3: chemical potential, Eq. (32), then Eq. (36) at solid nodes (a
    # solid node inside a thick solid keeps rho = 0; mu0 is taken at a
    # harmless density there and never used)
    rho_m = torch.where(fluid, rho, torch.where(rho > 0, rho, torch.ones_like(rho)))
    mu = mu_bulk(rho_m, p) - p.kappa * lap_h(rho)
    if has_solid(p):
        mu = torch.where(fluid, mu, wall_average(mu, s))
    # S4: Eq. (11)-(12)
    pm = (1.0 + mu) / 3.0
    G = grad_h(mu)
    F = (1.0 / 3.0 - rho) * G * s
    rho_safe = torch.where(fluid, rho, torch.ones_like(rho))
    u = (j + 0.5 * F) / rho_safe * s
    # S5: Eq. (27)-(28)
    phi = (pm - rho / 3.0) * u * s
    Q200 = -3.0 * grad_h(phi[0])[0] * s
    Q020 = -3.0 * grad_h(phi[1])[1] * s
    Q002 = -3.0 * grad_h(phi[2])[2] * s
    if p.corr4:
        Q220 = (Q200 + Q020) / 3.0
        Q202 = (Q200 + Q002) / 3.0
        Q022 = (Q020 + Q002) / 3.0
    else:
        Q220 = Q202 = Q022 = torch.zeros_like(Q200)
    # S6: omega_1 from nu, tau = rho nu / p_m + 1/2
    om1 = 1.0 / (rho * p.nu / pm + 0.5)
    return dict(rho=rho, j=j, mu=mu, G=G, F=F, u=u, pm=pm, phi=phi,
                Q=(Q200, Q020, Q002, Q220, Q202, Q022), omega1=om1, s=s)


def stream(fs, p: Params, rho=None, pm=None):
    """Eq. (10): f_i(x, t+1) = f*_i(x - c_i); with walls the halfway
    bounce-back f_i(x, t+1) = f*_opp(i)(x) when x - c_i is solid.

    Moving walls (the moving-wall droplet test of Sec. III B, whose scheme
    the paper cites without writing it out): the reflected population takes
    the odd part of the model's own equilibrium at the wall velocity u_w,
        f_i(x, t+1) = f*_o(x) - [f^eq_o - f^eq_i](rho(x), p_m(x), u_w),
    o = opp(i), with f^eq the generalized equilibrium of Eq. (20) at the
    fluid node's rho and p_m.  A fluid moving with the wall is then left
    unchanged by the wall; for p_m = rho c_s^2 the bracket is, to first order
    in u_w, the familiar 2 w_o rho c_o . u_w / c_s^2."""
    s = fluid_mask(p)
    moving = p.walls_z and any(v != 0.0 for v in p.wall_u)
    if moving and p.solid is not None:
        raise ValueError("moving walls are defined for the wall planes only")
    if moving:
        shape = tuple(fs.shape[1:])

        def feq_at(ux, uy):
            uw = torch.zeros((3,) + shape, dtype=DT)
            uw[0] = ux
            uw[1] = uy
            return populations_from_central(equilibrium_central(rho, pm), uw)

        feq_b = feq_at(p.wall_u[0], p.wall_u[1])  # bottom wall (z = 0)
        feq_t = feq_at(p.wall_u[2], p.wall_u[3])  # top wall (z = nz-1)
    out = []
    for i, c in enumerate(C):
        pulled = at(fs[i], (-c[0], -c[1], -c[2]))
        if has_solid(p):
            src_fluid = at(s, (-c[0], -c[1], -c[2])) > 0
            back = fs[OPP[i]]
            if moving and c[2] != 0:
                # x - c_i is solid only across a z wall: c_z > 0 reflects at
                # the bottom wall, c_z < 0 at the top wall
                fe = feq_b if c[2] > 0 else feq_t
                back = back - (fe[OPP[i]] - fe[i])
            pulled = torch.where(src_fluid, pulled, back)
            pulled = pulled * s
        out.append(pulled)
    return torch.stack(out)


def step(f, p: Params, return_aux=False):
    """One time step t -> t+1 (S1-S10)."""
    A = aux_fields(f, p)
    w = list(p.omega)
    w[1] = A["omega1"]
    k = central_moments(f, A["u"])
    ks = collide(k, A["F"], A["Q"], A["pm"], w)
    fs = populations_from_central(ks, A["u"])
    fn = stream(fs, p, A["rho"], A["pm"])
    return (fn, A) if return_aux else fn


def init(rho0, p: Params, u0=None):
    """Initial populations: Eq. (20) equilibrium CMs at (rho0, u0, p_m) with
    p_m from mu[rho0] (wall densities from Eqs. (37)-(38) first)."""
    s = fluid_mask(p)
    fluid = s > 0
    rho0 = rho0.to(DT)
    rho = wall_density(rho0, s, p) if has_solid(p) else rho0
    rho_m = torch.where(fluid, rho, torch.where(rho > 0, rho, torch.ones_like(rho)))
    mu = mu_bulk(rho_m, p) - p.kappa * lap_h(rho)
    pm = (1.0 + mu) / 3.0
    if u0 is None:
        u0 = torch.zeros((3,) + tuple(rho0.shape), dtype=DT)
    rho_safe = torch.where(s > 0, rho0, torch.ones_like(rho0))
    keq = equilibrium_central(rho_safe, pm)
    f = populations_from_central(keq, u0.to(DT) * s)
    return f * s


def run(f, p: Params, nsteps):
    for _ in range(nsteps):
        f = step(f, p)
    return f
