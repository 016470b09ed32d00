"""Measurement helpers for the paper's validation cases (Sec. III):
surface tension (Eq. (33)), discrete static equilibria found by Newton's
method, the Young-Laplace prediction, equimolar radius and contact angle.
Plain numpy/scipy float64."""
import math

import numpy as np

from . import eos


# --------------------------------------------------------------------------
# flat interface, Sec. III A
# --------------------------------------------------------------------------
def surface_tension(rho_z, kappa):
    """Eq. (33) on the lattice: kappa * sum over z in [0, Nz/2) of the squared
    central difference (rho_{z+1} - rho_{z-1}) / 2 (periodic wrap)."""
    r = np.asarray(rho_z, dtype=np.float64)
    n = r.size
    d = (np.roll(r, -1) - np.roll(r, 1)) / 2.0
    return kappa * float(np.sum(d[: n // 2] ** 2))


def _mu0_vec(r, a, b, R, T):
    return R * T * (np.log(r / (1.0 - b * r)) + 1.0 / (1.0 - b * r)) - 2.0 * a * r


def _dmu0_vec(r, a, b, R, T):
    return R * T / (r * (1.0 - b * r) ** 2) - 2.0 * a


def tanh_profile_1d(nz, rho_l, rho_v, width=5.0, z1=None, z2=None):
    """Liquid slab between z1 and z2 (default Nz/4 and 3Nz/4), tanh walls."""
    z = np.arange(nz, dtype=np.float64)
    z1 = 0.25 * nz if z1 is None else z1
    z2 = 0.75 * nz if z2 is None else z2
    return rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(2 * (z - z1) / width) - np.tanh(2 * (z - z2) / width))


def flat_equilibrium(rho_init, a, b, R, T, kappa, tol=1e-15, maxit=100):
    """Discrete flat-interface equilibrium on a periodic 1-D lattice:
    mu0(rho_z) - kappa (rho_{z+1} - 2 rho_z + rho_{z-1}) = mu*, with the total
    mass of rho_init conserved.  For fields uniform in x and y the isotropic
    D3Q27 Laplacian reduces to this 3-point form.  Returns (rho, mu*)."""
    r = np.array(rho_init, dtype=np.float64)
    n = r.size
    mass = r.sum()
    mu_s = float(np.mean(_mu0_vec(r, a, b, R, T)))
    L = -2.0 * np.eye(n) + np.roll(np.eye(n), 1, axis=1) + np.roll(np.eye(n), -1, axis=1)
    for _ in range(maxit):
        res = np.concatenate([_mu0_vec(r, a, b, R, T) - kappa * (L @ r) - mu_s, [r.sum() - mass]])
        J = np.zeros((n + 1, n + 1))
        J[:n, :n] = np.diag(_dmu0_vec(r, a, b, R, T)) - kappa * L
        J[:n, n] = -1.0
        J[n, :n] = 1.0
        d = np.linalg.solve(J, -res)
        r, mu_s, done = _damped_update(r, mu_s, d, lambda rr, mm: _flat_residual(rr, mm, L, mass, a, b, R, T, kappa),
                                       res, b, tol)
        if done:
            break
    return r, mu_s


def _flat_residual(r, mu_s, L, mass, a, b, R, T, kappa):
    return np.concatenate([_mu0_vec(r, a, b, R, T) - kappa * (L @ r) - mu_s, [r.sum() - mass]])


def _damped_update(r, mu_s, d, resid, res0, b, tol):
    """Newton update with backtracking: halve the step until the density
    stays inside (0, 1/b) and the residual norm does not grow."""
    n = r.size
    lam = 1.0
    n0 = np.linalg.norm(res0)
    while lam > 1e-6:
        rn = r + lam * d[:n]
        mn = mu_s + lam * d[n]
        if np.all(rn > 0) and np.all(b * rn < 1):
            if np.linalg.norm(resid(rn, mn)) <= n0 or lam < 1e-3:
                break
        lam *= 0.5
    done = lam == 1.0 and np.max(np.abs(d)) < tol * max(1.0, np.max(np.abs(rn)))
    return rn, mn, done


def wall_flat_equilibrium(rho_init, a, b, R, T, kappa, rho_wall, drho_wall, tol=1e-15, maxit=100):
    """Discrete equilibrium of a film uniform in x, y between two solid planes
    (fluid nodes z = 1..n-2 given in rho_init of length n-2).  rho_wall(r1) and
    drho_wall(r1) give the solid-node density (Eqs. (37)-(38)) and its
    derivative as a function of the adjacent fluid density (for a uniform
    layer the weighted average of Eq. (37) equals that density)."""
    r = np.array(rho_init, dtype=np.float64)
    n = r.size
    mass = r.sum()
    mu_s = float(np.mean(_mu0_vec(r, a, b, R, T)))
    for _ in range(maxit):
        full = np.concatenate([[rho_wall(r[0])], r, [rho_wall(r[-1])]])
        lap = full[2:] - 2 * full[1:-1] + full[:-2]
        res = np.concatenate([_mu0_vec(r, a, b, R, T) - kappa * lap - mu_s, [r.sum() - mass]])
        J = np.zeros((n + 1, n + 1))
        for z in range(n):
            J[z, z] = _dmu0_vec(r[z], a, b, R, T) + 2 * kappa
            if z > 0:
                J[z, z - 1] = -kappa
            if z < n - 1:
                J[z, z + 1] = -kappa
        J[0, 0] -= kappa * drho_wall(r[0])
        J[n - 1, n - 1] -= kappa * drho_wall(r[-1])
        J[:n, n] = -1.0
        J[n, :n] = 1.0
        d = np.linalg.solve(J, -res)

        def resid(rr, mm):
            full = np.concatenate([[rho_wall(rr[0])], rr, [rho_wall(rr[-1])]])
            lp = full[2:] - 2 * full[1:-1] + full[:-2]
            return np.concatenate([_mu0_vec(rr, a, b, R, T) - kappa * lp - mm, [rr.sum() - mass]])

        r, mu_s, done = _damped_update(r, mu_s, d, resid, res, b, tol)
        if done:
            break
    return r, mu_s


# --------------------------------------------------------------------------
# droplets, Sec. III B
# --------------------------------------------------------------------------
def young_laplace(sigma, radius, a, b, R, T, guess=None):
    """Inside/outside densities of a droplet of radius R from equal chemical
    potential and the Laplace pressure jump p0(in) - p0(out) = 2 sigma / R."""
    rl, rv = guess if guess is not None else eos.maxwell(a, b, R, T)
    dp = 2.0 * sigma / radius
    for _ in range(100):
        f1 = eos.mu0(rl, a, b, R, T) - eos.mu0(rv, a, b, R, T)
        f2 = eos.p0(rl, a, b, R, T) - eos.p0(rv, a, b, R, T) - dp
        j11, j12 = eos.dmu0(rl, a, b, R, T), -eos.dmu0(rv, a, b, R, T)
        j21, j22 = rl * j11, rv * j12
        det = j11 * j22 - j12 * j21
        dl = (f1 * j22 - f2 * j12) / det
        dv = (j11 * f2 - j21 * f1) / det
        rl, rv = rl - dl, rv - dv
        if abs(dl) + abs(dv) < 1e-15 * rl:
            break
    return rl, rv


def _lap_h_matrix(shape):
    """The isotropic D3Q27 Laplacian of the step (reading R4: lap_h g =
    6 sum_i w_i (g(x + c_i) - g(x)), weights of Eq. (17)) as a sparse matrix
    on a periodic (nz, ny, nx) grid, nodes in C order."""
    import scipy.sparse as sp
    from .lattice import C, W_EXACT
    nz, ny, nx = shape
    n = nz * ny * nx
    idx = np.arange(n).reshape(shape)
    rows, cols, vals = [], [], []
    for (cx, cy, cz), w in zip(C, W_EXACT):
        if (cx, cy, cz) == (0, 0, 0):
            continue
        nb = np.roll(idx, shift=(-cz, -cy, -cx), axis=(0, 1, 2))  # index of x + c_i
        rows += [idx.ravel(), idx.ravel()]
        cols += [nb.ravel(), idx.ravel()]
        vals += [np.full(n, 6.0 * float(w)), np.full(n, -6.0 * float(w))]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def static_equilibrium_3d(rho_init, a, b, R, T, kappa, tol=1e-14, maxit=60):
    """Discrete static equilibrium in 3-D (pins P9/P11): the density field of
    a periodic box with mu0(rho) - kappa lap_h rho = mu* at every node and the
    mass of rho_init, by Newton's method on the sparse system (unknowns rho
    and mu*).  With u = 0 such a field makes F = 0, Q = 0 and the moving
    populations uniform, so it is a fixed point of the step for any rates.
    Returns (rho, mu*)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    r = np.array(rho_init, dtype=np.float64)
    shape = r.shape
    r = r.ravel()
    n = r.size
    mass = r.sum()
    L = _lap_h_matrix(shape)
    mu_s = float(np.mean(_mu0_vec(r, a, b, R, T) - kappa * (L @ r)))
    def resid(rr, mm):
        return np.concatenate([_mu0_vec(rr, a, b, R, T) - kappa * (L @ rr) - mm, [rr.sum() - mass]])

    for _ in range(maxit):
        res = resid(r, mu_s)
        # converged: mu0 - kappa lap_h rho - mu* at rounding level, mass to
        # the rounding of its sum
        if np.max(np.abs(res[:n])) < tol and abs(res[n]) < 1e-13 * mass:
            break
        # bordered Newton system [[J, -1], [1^T, 0]] (d_rho, d_mu) = -res,
        # solved through one sparse LU of J = diag(mu0') - kappa lap_h
        lu = spla.splu(sp.csc_matrix(sp.diags(_dmu0_vec(r, a, b, R, T)) - kappa * L))
        y1 = lu.solve(-res[:n])
        y2 = lu.solve(np.ones(n))
        dmu = (-res[n] - y1.sum()) / y2.sum()
        d = np.concatenate([y1 + dmu * y2, [dmu]])
        r, mu_s, done = _damped_update(r, mu_s, d, resid, res, b, tol)
        if done:
            break
    return r.reshape(shape), mu_s


def equimolar_radius(rho, rho_in, rho_out):
    """R = (3V / 4 pi)^(1/3), V = sum (rho - rho_out) / (rho_in - rho_out)."""
    V = float(np.sum((np.asarray(rho) - rho_out) / (rho_in - rho_out)))
    return (3.0 * V / (4.0 * math.pi)) ** (1.0 / 3.0)


def tanh_droplet(shape, center, radius, rho_l, rho_v, width=5.0):
    """Eqs. (34)-(35) on a (nz, ny, nx) grid, centre given as (x0, y0, z0)."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r0 = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    return (rho_l + rho_v) / 2 - (rho_l - rho_v) / 2 * np.tanh(2 * (r0 - radius) / width)


def contact_angle(rho, rho_l, rho_v, z_wall=0.5, zmin_offset=3.0):
    """Contact angle of a sessile droplet resting on the bottom wall of a
    (nz, ny, nx) density field.  Points of the rho = (rho_l + rho_v)/2
    isosurface are located by linear interpolation along x and along z in
    the central x-z plane and along y and z in the central y-z plane; a
    least-squares circle fit (horizontal coordinates relative to the plane
    centre N/2, where the droplet is placed) to the points with
    z > z_wall + zmin_offset
    gives centre height z_c and radius R; cos(theta) = (z_wall - z_c) / R."""
    rho = np.asarray(rho)
    nz, ny, nx = rho.shape
    level = 0.5 * (rho_l + rho_v)
    pts = []
    for plane, along in ((rho[:, ny // 2, :], "x"), (rho[:, :, nx // 2], "y")):
        nzp, nh = plane.shape
        # crossings along the horizontal axis
        for z in range(nzp):
            row = plane[z]
            for h in range(nh - 1):
                a, b = row[h] - level, row[h + 1] - level
                if a == 0 or a * b < 0:
                    t = a / (a - b)
                    pts.append((h + t - nh / 2.0, z))
        # crossings along z
        for h in range(nh):
            col = plane[:, h]
            for z in range(nzp - 1):
                a, b = col[z] - level, col[z + 1] - level
                if a == 0 or a * b < 0:
                    t = a / (a - b)
                    pts.append((h - nh / 2.0, z + t))
    P = np.array(pts, dtype=np.float64).reshape(-1, 2)
    P = P[P[:, 1] > z_wall + zmin_offset]
    if len(P) < 3:
        return float("nan"), float("nan"), float("nan")
    # algebraic circle fit in the (h, z) plane:  h^2 + z^2 + D h + E z + F = 0
    A = np.column_stack([P[:, 0], P[:, 1], np.ones(len(P))])
    rhs = -(P[:, 0] ** 2 + P[:, 1] ** 2)
    D, E, Fc = np.linalg.lstsq(A, rhs, rcond=None)[0]
    hc, zc = -D / 2, -E / 2
    Rf = math.sqrt(hc * hc + zc * zc - Fc)
    cos_t = max(-1.0, min(1.0, (z_wall - zc) / Rf))
    return math.degrees(math.acos(cos_t)), zc, Rf
