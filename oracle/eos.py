"""van der Waals closure of Sec. III, Eqs. (29)-(32), and the Maxwell
equal-area coexistence densities used in Sec. III (plain float64 math)."""
import math


def critical_point(a, b, R):
    """Eq. (30): rho_c = 1/(3b), T_c = 8a/(27Rb), p_c = a/(27 b^2)."""
    return 1.0 / (3.0 * b), 8.0 * a / (27.0 * R * b), a / (27.0 * b * b)


def p0(rho, a, b, R, T):
    """Eq. (29)."""
    return rho * R * T / (1.0 - b * rho) - a * rho * rho


def psi(rho, a, b, R, T):
    """Eq. (31): bulk free-energy density."""
    return rho * R * T * math.log(rho / (1.0 - b * rho)) - a * rho * rho


def mu0(rho, a, b, R, T):
    """Bulk part of Eq. (32): d psi / d rho."""
    return R * T * (math.log(rho / (1.0 - b * rho)) + 1.0 / (1.0 - b * rho)) - 2.0 * a * rho


def dmu0(rho, a, b, R, T):
    """d mu0 / d rho = RT / (rho (1 - b rho)^2) - 2a."""
    return R * T / (rho * (1.0 - b * rho) ** 2) - 2.0 * a


def maxwell(a, b, R, T, guess=None, tol=1e-14, maxit=200):
    """Coexistence pair (rho_l, rho_v) from equal chemical potential and equal
    pressure, mu0(l) = mu0(v), p0(l) = p0(v) (the equal-area rule, Sec. III).
    Newton on the 2x2 system; the default start is the spinodal-bracketing
    pair (0.9/b, 0.05/b) which converges for 0.5 < T/Tc < 0.99."""
    rl, rv = guess if guess is not None else (0.75 / b, 0.03 / b)
    for _ in range(maxit):
        f1 = mu0(rl, a, b, R, T) - mu0(rv, a, b, R, T)
        f2 = p0(rl, a, b, R, T) - p0(rv, a, b, R, T)
        # dp0/drho = rho * dmu0/drho (Gibbs-Duhem)
        j11, j12 = dmu0(rl, a, b, R, T), -dmu0(rv, a, b, R, T)
        j21, j22 = rl * dmu0(rl, a, b, R, T), -rv * dmu0(rv, a, b, R, T)
        det = j11 * j22 - j12 * j21
        dl = (f1 * j22 - f2 * j12) / det
        dv = (j11 * f2 - j21 * f1) / det
        step = 1.0
        while True:
            nl, nv = rl - step * dl, rv - step * dv
            if 0 < nv < nl < 1.0 / b:
                break
            step *= 0.5
        rl, rv = nl, nv
        if abs(dl) + abs(dv) < tol * rl:
            break
    return rl, rv


# Paper defaults (Sec. III): a = 9/392, b = 2/21, R = 1, kappa = 0.02,
# T = 0.7 Tc, nu = 0.15.
PAPER = dict(a=9.0 / 392.0, b=2.0 / 21.0, R=1.0, kappa=0.02, nu=0.15)


def temperature(tr, a=PAPER["a"], b=PAPER["b"], R=PAPER["R"]):
    return tr * critical_point(a, b, R)[1]
