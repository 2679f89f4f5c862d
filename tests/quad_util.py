"""Independent numerical references (quadrature) for the pins.

Nothing here is shared with the oracle or the HIP library: each function is a
direct numerical evaluation of a formula of the paper or of a textbook result.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, special


def voigt_scipy(a, x):
    """H(a, x) = Re w(x + i a) from scipy's Faddeeva function."""
    return special.wofz(np.asarray(x, dtype=np.float64) + 1j * a).real


def upar_cdf_table(x0, a, n=6000):
    """CDF of p(u | x0) ~ exp(-u^2)/(a^2 + (x0 - u)^2) (Sec. 2.1.1) on a grid
    dense near the Lorentz peak at u = x0; returns (u, F)."""
    # grid: uniform in atan((u - x0)/a) near the peak, uniform in u elsewhere
    th = np.linspace(-np.arctan(1.0 / a), np.arctan(1.0 / a), n)
    core = x0 + a * np.tan(th)
    lo = min(-7.0, x0 - 8.0)
    hi = max(7.0, x0 + 8.0)
    outer = np.concatenate([np.linspace(lo, x0 - 1.0, n), np.linspace(x0 + 1.0, hi, n),
                            np.linspace(x0 - 1.0, x0 + 1.0, 2 * n)])
    u = np.unique(np.concatenate([core, outer]))
    f = np.exp(-u * u) / (a * a + (x0 - u) ** 2)
    # trapezoid in the variable that makes each piece smooth: use exact Lorentz
    # integral for the 1/(a^2+d^2) factor with exp(-u^2) linear on each interval
    d0, d1 = u[:-1] - x0, u[1:] - x0
    g0, g1 = np.exp(-u[:-1] ** 2), np.exp(-u[1:] ** 2)
    # int_{d0}^{d1} (g0 + (g1-g0) t) / (a^2 + d^2) dd with t = (d-d0)/(d1-d0)
    at = (np.arctan(d1 / a) - np.arctan(d0 / a)) / a
    lg = 0.5 * np.log((a * a + d1 * d1) / (a * a + d0 * d0))
    h = d1 - d0
    slope = (g1 - g0) / h
    seg = g0 * at + slope * (lg - d0 * at)
    F = np.concatenate([[0.0], np.cumsum(seg)])
    return u, F / F[-1], F[-1]


def riia_channel_probs(x0, a, g, edges):
    """Channel integrals of the R_IIA kernel (eq. riia-kernel): probability that
    x_out = x0 + u (g - 1) + N(0, (1 - g^2)/2) falls in each [e_k, e_k+1)."""
    u, F, _ = upar_cdf_table(x0, a)
    dF = np.diff(F)
    um = 0.5 * (u[1:] + u[:-1])
    s = np.sqrt(max(0.0, 1.0 - g * g) / 2.0)
    centre = x0 + um * (g - 1.0)
    edges = np.asarray(edges, dtype=np.float64)
    if s < 1e-12:
        cdf_e = np.array([np.sum(dF[centre < e]) for e in edges])
    else:
        cdf_e = np.array([np.sum(dF * special.ndtr((e - centre) / s)) for e in edges])
    return np.diff(cdf_e)


def neufeld_slab_profile(x, a, tau0):
    """Harrington / Neufeld slab escape profile in the line-centre convention:
    J(x) ~ x^2 / cosh(sqrt(pi^3/54) |x|^3 / (a tau0)) (normalised to unit area)."""
    c = np.sqrt(np.pi ** 3 / 54.0)
    f = lambda t: t * t / np.cosh(c * np.abs(t) ** 3 / (a * tau0))
    norm = 2.0 * integrate.quad(f, 0, 50 * (a * tau0) ** (1 / 3), limit=400)[0]
    return f(np.asarray(x)) / norm


def neufeld_mean_abs_x(a, tau0):
    c = np.sqrt(np.pi ** 3 / 54.0)
    f = lambda t: t * t / np.cosh(c * t ** 3 / (a * tau0))
    up = 50 * (a * tau0) ** (1 / 3)
    return integrate.quad(lambda t: t * f(t), 0, up, limit=400)[0] / integrate.quad(f, 0, up, limit=400)[0]


def thin_sphere_J_ratio(rho):
    """Mean intensity inside a uniformly emitting, optically thin sphere,
    J(rho)/J(0) = 1/2 [1 + (1 - rho^2)/(2 rho) ln((1 + rho)/(1 - rho))]."""
    rho = np.asarray(rho, dtype=np.float64)
    return 0.5 * (1.0 + (1.0 - rho ** 2) / (2.0 * rho) * np.log((1.0 + rho) / (1.0 - rho)))


def box_chord_no_scatter_prob(kappas, bounds_x, src, nth=400, nph=800):
    """(1/4 pi) int exp(-sum_i kappa_i l_i(n)) dOmega for a point source inside
    the box [-1,1]^3 split in x at bounds_x (cells i between consecutive bounds),
    l_i the chord length of the ray in cell i (plain ray geometry)."""
    mu = np.cos((np.arange(nth) + 0.5) * np.pi / nth)
    wmu = np.sin((np.arange(nth) + 0.5) * np.pi / nth) * np.pi / nth
    ph = (np.arange(nph) + 0.5) * 2 * np.pi / nph
    M, P = np.meshgrid(mu, ph, indexing="ij")
    st = np.sqrt(1 - M * M)
    n = np.stack([st * np.cos(P), st * np.sin(P), M])
    s = np.asarray(src, dtype=np.float64)
    # exit distance from the box
    t_exit = np.full(M.shape, np.inf)
    for d in range(3):
        nd = n[d]
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(nd > 0, (1 - s[d]) / nd, np.where(nd < 0, (-1 - s[d]) / nd, np.inf))
        t_exit = np.minimum(t_exit, t)
    tau = np.zeros(M.shape)
    for i, k in enumerate(kappas):
        x0, x1 = bounds_x[i], bounds_x[i + 1]
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = np.where(n[0] != 0, (x0 - s[0]) / n[0], -np.inf)
            tb = np.where(n[0] != 0, (x1 - s[0]) / n[0], np.inf)
        lo = np.minimum(ta, tb)
        hi = np.maximum(ta, tb)
        inside_always = (n[0] == 0) & (s[0] >= x0) & (s[0] < x1)
        lo = np.where(inside_always, -np.inf, lo)
        hi = np.where(inside_always, np.inf, hi)
        seg = np.clip(np.minimum(hi, t_exit) - np.maximum(lo, 0.0), 0.0, None)
        tau += k * seg
    w = wmu[:, None] * (2 * np.pi / nph)
    return float(np.sum(np.exp(-tau) * w) / (4 * np.pi))


def voigt_profile_cdf(a, x, span=60.0, step=5e-4):
    """CDF of the normalised Voigt profile H(a, x)/sqrt(pi) from scipy's own
    voigt_profile (Gaussian of variance 1/2 with a Lorentzian of half-width a),
    integrated by the trapezoid rule on [-span, span] with the Lorentz tails
    beyond added in closed form (a / (pi |x|) to leading order)."""
    t = np.arange(-span, span + step / 2, step)
    f = special.voigt_profile(t, np.sqrt(0.5), a)
    F = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * step)])
    tail = np.arctan(a / span) / np.pi  # Cauchy mass beyond |x| = span (Gaussian part negligible)
    F = tail + F * (1.0 - 2.0 * tail) / F[-1]
    x = np.asarray(x, dtype=np.float64)
    out = np.interp(x, t, F)
    out = np.where(x < -span, np.arctan(a / -np.minimum(x, -span)) / np.pi, out)
    out = np.where(x > span, 1.0 - np.arctan(a / np.maximum(x, span)) / np.pi, out)
    return out


def gauss_half_cdf(x):
    """CDF of the thermal profile exp(-x^2)/sqrt(pi) (a Gaussian of variance 1/2)."""
    return 0.5 * (1.0 + special.erf(np.asarray(x, dtype=np.float64)))
