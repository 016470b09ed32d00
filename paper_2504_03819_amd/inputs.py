"""Seeded synthetic initial fields for the paper's test problems.

Only input construction lives here (geometry, noise, velocities): no part of
the time step.  Coexistence densities are arguments.  Both the GPU path and
the CPU oracle consume these arrays.  All arrays are float64 numpy with
shape (nz, ny, nx) for scalars and (3, nz, ny, nx) for vectors.
"""
import numpy as np


def _grid(shape):
    nz, ny, nx = shape
    return np.ogrid[0:nz, 0:ny, 0:nx]


def sphere(shape, center, radius, rho_l, rho_v, width=5.0):
    """Eqs. (34)-(35): tanh profile of width W around a sphere of radius r
    centred at (x0, y0, z0)."""
    z, y, x = _grid(shape)
    r0 = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (r0 - radius) / width)


def indicator(shape, center, radius, width=5.0):
    """Smooth 0..1 indicator of one sphere (same tanh profile)."""
    z, y, x = _grid(shape)
    r0 = np.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
    return 0.5 - 0.5 * np.tanh(2.0 * (r0 - radius) / width)


def flat_slab(shape, rho_l, rho_v, width=5.0, axis=0):
    """Liquid slab between 0.25 N and 0.75 N along `axis` (0 = z), Sec. III A."""
    n = shape[axis]
    c = np.arange(n, dtype=np.float64)
    prof = rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(2 * (c - 0.25 * n) / width) - np.tanh(2 * (c - 0.75 * n) / width))
    view = [1, 1, 1]
    view[axis] = n
    return np.broadcast_to(prof.reshape(view), shape).copy()


def uniform_noise(shape, amplitude, seed):
    """i.i.d. U(-amplitude, amplitude) from numpy PCG64 with a fixed seed."""
    g = np.random.Generator(np.random.PCG64(seed))
    return g.uniform(-amplitude, amplitude, size=shape)


# --------------------------------------------------------------------------
# the five benchmark problems
# --------------------------------------------------------------------------
def stationary_droplet(rho_l, rho_v, n=32, radius=8.0, noise=1e-6, seed=1):
    """Droplet of radius 8 centred in a periodic 32^3 box, tanh width 5,
    zero velocity, seeded uniform density noise of amplitude 1e-6."""
    shape = (n, n, n)
    rho = sphere(shape, (n / 2, n / 2, n / 2), radius, rho_l, rho_v)
    if noise:
        rho = rho + uniform_noise(shape, noise, seed)
    return rho, None


def moving_droplet(rho_l, rho_v, n=128, radius=24.0, velocity=(0.05, 0.02, 0.0)):
    """Droplet of radius 24 centred in a periodic 128^3 box with a uniform
    initial velocity everywhere (Galilean-invariance test)."""
    shape = (n, n, n)
    rho = sphere(shape, (n / 2, n / 2, n / 2), radius, rho_l, rho_v)
    u = np.empty((3,) + shape)
    for a in range(3):
        u[a] = velocity[a]
    return rho, u


def spinodal(rho_l, rho_v, n=256, rel_noise=0.01, seed=3):
    """Mean of the coexistence pair times (1 + U(-1%, 1%)) i.i.d. per node,
    zero velocity."""
    shape = (n, n, n)
    mean = 0.5 * (rho_l + rho_v)
    return mean * (1.0 + uniform_noise(shape, rel_noise, seed)), None


def sessile_droplet(rho_l, rho_v, nx=192, ny=192, nz=96, radius=32.0, z_wall=0.5):
    """Hemispherical droplet of radius 32 on the bottom wall (solid planes at
    z = 0 and z = nz-1; the halfway bounce-back wall plane is z = 0.5)."""
    shape = (nz, ny, nx)
    rho = sphere(shape, (nx / 2, ny / 2, z_wall), radius, rho_l, rho_v)
    rho[0] = rho_v
    rho[-1] = rho_v
    return rho, None


def head_on_collision(rho_l, rho_v, n=512, radius=64.0, gap_centres=160.0, speed=0.04):
    """Two droplets of radius 64 whose centres are 160 apart along x,
    approaching with +-0.04 (velocity carried by each droplet's indicator)."""
    shape = (n, n, n)
    c1 = (n / 2 - gap_centres / 2, n / 2, n / 2)
    c2 = (n / 2 + gap_centres / 2, n / 2, n / 2)
    chi1 = indicator(shape, c1, radius)
    chi2 = indicator(shape, c2, radius)
    rho = rho_v + (rho_l - rho_v) * (chi1 + chi2)
    u = np.zeros((3,) + shape)
    u[0] = speed * chi1 - speed * chi2
    return rho, u


def perturb_populations(f, amplitude, seed):
    """Add seeded uniform noise to a (27, ...) population array (used to
    leave the equilibrium manifold in parity checks)."""
    return f + uniform_noise(f.shape, amplitude, seed)


# ---------------------------------------------------------------------------
# solid voxel masks (uint8, 1 = solid, shape (nz, ny, nx))
# ---------------------------------------------------------------------------
def mask_planes(shape):
    """The two flat walls z = 0 and z = nz-1 as a mask."""
    m = np.zeros(shape, dtype=np.uint8)
    m[0] = 1
    m[-1] = 1
    return m


def mask_obstacles(shape, seed=11):
    """A periodic box with assorted solids: a ball, a pillar through the
    whole height, a thick block (with solid nodes that touch no fluid) and a
    few seeded single voxels.  Sizes scale with the box; at least 8^3."""
    nz, ny, nx = shape
    z, y, x = _grid(shape)
    m = np.zeros(shape, dtype=np.uint8)
    r = max(1.5, min(shape) / 6.0)
    m[(x - 0.3 * nx) ** 2 + (y - 0.35 * ny) ** 2 + (z - 0.4 * nz) ** 2 <= r * r] = 1
    m[:, int(0.7 * ny):int(0.7 * ny) + 2, int(0.75 * nx) % nx] = 1
    bz, by, bx = max(3, nz // 4), max(3, ny // 4), max(3, nx // 4)
    m[nz - bz:, :by, nx - bx:] = 1
    g = np.random.Generator(np.random.PCG64(seed))
    for _ in range(3):
        m[g.integers(nz), g.integers(ny), g.integers(nx)] = 1
    return m


def mask_pillars(shape, plate=2, pitch=12, width=4, height=6):
    """A patterned substrate: a solid plate of `plate` layers at the bottom,
    square pillars of `width` x `width` and `height` layers on a square
    lattice of `pitch`, and a flat solid top layer."""
    nz, ny, nx = shape
    m = np.zeros(shape, dtype=np.uint8)
    m[:plate] = 1
    m[-1] = 1
    z, y, x = _grid(shape)
    pill = ((x % pitch) < width) & ((y % pitch) < width) & (z < plate + height)
    m[np.broadcast_to(pill, shape)] = 1
    return m
