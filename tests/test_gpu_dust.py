"""Grey (dust) absorption inside the Monte Carlo walk on the GPU, through the C
ABI: the absorption-only slab against its closed form, the dusty slab of
Sec. 3.2 against the analytic escape fraction and against the FP64 oracle."""
from __future__ import annotations

import numpy as np
import pytest
from scipy import special

import oracle
from paper_2608_09340_amd import workloads as W
from stats_util import chi2_two_sample

pytestmark = pytest.mark.gpu


def _fesc_ref(a, tau0, tau_a):
    """Neufeld (1990) escape fraction in the form of Verhamme, Schaerer &
    Maselli (2006), zeta = 0.525."""
    return 1.0 / np.cosh(np.sqrt(3.0) / (0.525 * np.pi ** (5.0 / 12.0)) * np.sqrt((a * tau0) ** (1 / 3) * tau_a))


@pytest.mark.parametrize("tau_a", [0.05, 0.5, 2.0])
def test_pure_absorber_slab_is_E2(gpu_ctx, tau_a):
    """No line opacity, grey absorption depth tau_a from the midplane to each
    face: a midplane photon with an isotropic direction leaves with
    probability E2(tau_a) (the exponential integral), every other one is
    absorbed; nothing scatters."""
    from paper_2608_09340_amd import krt
    p = W.dusty_slab(1.0, 1e-2, tau_a, nz=8)
    p["grid"]["k0"][:] = 0.0
    T = krt.Transport(p, ctx=gpu_ctx)
    N = 400_000
    r = T.run(N, seed=2)
    c = r["counters"]
    assert r["rc"] == 0 and c["scatterings"] == 0 and c["escaped"] + c["destroyed"] == N
    ref = special.expn(2, tau_a)
    assert abs(c["escaped"] / N - ref) < 4.5 * np.sqrt(ref * (1 - ref) / N), (c["escaped"] / N, ref)


@pytest.mark.parametrize("tau_a", [0.005, 0.036, 0.11, 0.3, 0.6, 1.2])
def test_dusty_slab_escape_fraction(gpu_ctx, tau_a):
    """Sec. 3.2: slab of depth tau0 = 1e5 in the analytic solution's (mean
    depth) convention, a = 0.015, central plane of line-centre photons, grey
    absorption depth tau_a (the escape fraction spans about 0.9 to 1e-3 over
    these depths, nearly three decades as in the paper); 2e5 packets per
    point, as in the paper.  The escaped fraction follows the analytic curve
    within the 12% the paper reports for its own code, plus 4 binomial
    standard errors."""
    from paper_2608_09340_amd import krt
    a, tau0 = 0.015, 1e5
    T = krt.Transport(W.dusty_slab(tau0, a, tau_a), ctx=gpu_ctx)
    N = 200_000
    r = T.run(N, seed=0)
    c = r["counters"]
    assert r["rc"] == 0 and c["escaped"] + c["destroyed"] == N
    f, ref = c["escaped"] / N, _fesc_ref(a, tau0, tau_a)
    print(f"tau_a {tau_a}: (a tau0)^(1/3) tau_a {(a * tau0) ** (1 / 3) * tau_a:.3f} f_esc {f:.4f} analytic {ref:.4f}")
    assert abs(f - ref) < 0.12 * ref + 4 * np.sqrt(ref * (1 - ref) / N), (f, ref)


def test_dusty_slab_vs_oracle(gpu_ctx):
    """The same slab at tau_a = 0.036: GPU escape fraction against the oracle's
    (binomial z < 4) and the escaped spectra (chi^2/dof < 1.3, every |z| < 4)."""
    from paper_2608_09340_amd import krt
    p = W.dusty_slab(1e5, 0.015, 0.036)
    T = krt.Transport(p, ctx=gpu_ctx)
    N = 200_000
    g = T.run(N, seed=0)
    no = 1500
    o = oracle.mc_run(p, no, seed=0, packet_offset=1 << 32)
    fg, fo = g["counters"]["escaped"] / N, o["counters"]["escaped"] / no
    se = np.sqrt(fo * (1 - fo) / no + fg * (1 - fg) / N)
    assert abs(fg - fo) < 4 * se, (fg, fo)
    chi2, dof, zmax = chi2_two_sample(g["spec_raw"], o["spec"], min_count=20)
    assert chi2 / dof < 1.3 and zmax < 4.0, (chi2 / dof, dof, zmax)
