"""Phase-space form of the generalized equilibrium, Eqs. (13)-(16).

The Hermite polynomials H_{i,abc} are only referenced (to an appendix of an
earlier paper).  Reading used here: tensor products of the 1-D Hermite
polynomials, H_{i,abc} = H_a(c_ix) H_b(c_iy) H_c(c_iz) with H_0 = 1,
H_1(c) = c, H_2(c) = c^2 - c_s^2.  The equations are transcribed term by
term from the paper; this module exists only to pin the central-moment
route (Eq. (20)) of ``oracle.lbm`` against the phase-space definition.
"""
import torch

from .lattice import C, W_T

CS2 = 1.0 / 3.0


def _H1d(n, c):
    return {0: 1.0, 1: c, 2: c * c - CS2}[n]


def hermite(a, b, g):
    """H_{i,abc} for all 27 directions as a float64 tensor."""
    return torch.tensor([_H1d(a, c[0]) * _H1d(b, c[1]) * _H1d(g, c[2]) for c in C], dtype=torch.float64)


def _bcast(t, like):
    return t.reshape((27,) + (1,) * like.dim())


def g_eq6(rho, u):
    """Eq. (14).  rho: (...), u: (3, ...) -> (27, ...)."""
    ux, uy, uz = u[0], u[1], u[2]
    H = lambda a, b, g: _bcast(hermite(a, b, g), rho)
    c2, c4, c6, c8, c10, c12 = CS2, CS2 ** 2, CS2 ** 3, CS2 ** 4, CS2 ** 5, CS2 ** 6
    t1 = (ux * H(1, 0, 0) + uy * H(0, 1, 0) + uz * H(0, 0, 1)) / c2
    t2 = (ux ** 2 * H(2, 0, 0) + uy ** 2 * H(0, 2, 0) + uz ** 2 * H(0, 0, 2)
          + 2 * (ux * uy * H(1, 1, 0) + uy * uz * H(0, 1, 1) + ux * uz * H(1, 0, 1))) / (2 * c4)
    t3 = (ux ** 2 * uy * H(2, 1, 0) + ux ** 2 * uz * H(2, 0, 1) + ux * uy ** 2 * H(1, 2, 0)
          + ux * uz ** 2 * H(1, 0, 2) + uy * uz ** 2 * H(0, 1, 2) + uy ** 2 * uz * H(0, 2, 1)
          + 2 * ux * uy * uz * H(1, 1, 1)) / (2 * c6)
    t4 = (ux ** 2 * uy ** 2 * H(2, 2, 0) + ux ** 2 * uz ** 2 * H(2, 0, 2) + uy ** 2 * uz ** 2 * H(0, 2, 2)
          + 2 * (ux * uy * uz ** 2 * H(1, 1, 2) + ux * uy ** 2 * uz * H(1, 2, 1)
                 + ux ** 2 * uy * uz * H(2, 1, 1))) / (4 * c8)
    t5 = (ux ** 2 * uy * uz ** 2 * H(2, 1, 2) + ux ** 2 * uy ** 2 * uz * H(2, 2, 1)
          + ux * uy ** 2 * uz ** 2 * H(1, 2, 2)) / (4 * c10)
    t6 = ux ** 2 * uy ** 2 * uz ** 2 * H(2, 2, 2) / (8 * c12)
    return rho * _bcast(W_T, rho) * (1 + t1 + t2 + t3 + t4 + t5 + t6)


def E_iso(like):
    """Eq. (16): isotropic operator."""
    H = lambda a, b, g: _bcast(hermite(a, b, g), like)
    c4, c6, c8 = CS2 ** 2, CS2 ** 3, CS2 ** 4
    return _bcast(W_T, like) * ((H(2, 0, 0) + H(0, 2, 0) + H(0, 0, 2)) / (2 * c4)
                                - (H(2, 2, 0) + H(0, 2, 2) + H(2, 0, 2)) / (4 * c6)
                                + H(2, 2, 2) / (8 * c8))


def Phi(u, like):
    """Eq. (15): correction operator."""
    ux, uy, uz = u[0], u[1], u[2]
    H = lambda a, b, g: _bcast(hermite(a, b, g), like)
    c2, c6, c8, c10, c12 = CS2, CS2 ** 3, CS2 ** 4, CS2 ** 5, CS2 ** 6
    s1 = (ux * (H(1, 2, 0) + H(1, 0, 2)) + uy * (H(2, 1, 0) + H(0, 1, 2)) + uz * (H(2, 0, 1) + H(0, 2, 1))) / (2 * c6)
    s2 = ((ux ** 2 + uy ** 2) * H(2, 2, 0) + (uy ** 2 + uz ** 2) * H(0, 2, 2) + (ux ** 2 + uz ** 2) * H(2, 0, 2)
          + 2 * (uy * uz * H(2, 1, 1) + ux * uz * H(1, 2, 1) + ux * uy * H(1, 1, 2))) / (4 * c8)
    s3 = (ux * (uy ** 2 + uz ** 2 - c2) * H(1, 2, 2) + uy * (ux ** 2 + uz ** 2 - c2) * H(2, 1, 2)
          + uz * (ux ** 2 + uy ** 2 - c2) * H(2, 2, 1)) / (4 * c10)
    s4 = ((ux ** 2 * uy ** 2 + uy ** 2 * uz ** 2 + ux ** 2 * uz ** 2 - c2 * (ux ** 2 + uy ** 2 + uz ** 2))
          * H(2, 2, 2)) / (8 * c12)
    return E_iso(like) + _bcast(W_T, like) * (s1 + s2 + s3 + s4)


def f_eq(rho, u, pm):
    """Eq. (13): f^eq = g^{eq,6} + (p_m - rho c_s^2) Phi."""
    return g_eq6(rho, u) + (pm - rho * CS2) * Phi(u, rho)
