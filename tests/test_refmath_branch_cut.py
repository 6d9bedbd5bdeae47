"""Pins of the no-wall reference (App. A, the infinite-phi_UV limit): the characteristic function
of eq. eq_appendix_characteristic_function_infinite_UV and the branch-cut integral for P(N).

* chi(0) = 1, and its first derivative at t = 0 gives the mean of N that the Green's-function
  moments of the backward operator give independently (eq. eq:meanN:S:gen).  That solver closes
  the domain with a reflecting wall at phi_esc = 100 phi_in; the walled characteristic function
  with its wall there reproduces the solver's variance, and the no-wall variance exceeds it by
  less than 1e-3 relative (the rare runs beyond phi_esc only add to it).
* The density from the cut agrees with simulated runs of the oracle (no wall, direct sampling),
  bin by bin within the counting error; a prefactor 2 pi off (the printed 2 in place of 1/pi)
  fails this by a factor of six.
* Far in the tail P(N) N^{3/2} exp(v0 N/4) tends to a constant, the asymptote the paper states,
  with the 1/N approach of a branch point.
"""
import math

import numpy as np

import oracle as O
from oracle import refmath as R

MODEL = O.Model(m=1.0, phi_in=6.0, dN=1e-3)
V0 = MODEL.m ** 2 / (48 * math.pi ** 2)


def _mean_sd(chi):
    """Mean and standard deviation of N from chi(-i s) = E[exp(s N)] by central differences."""
    import mpmath as mp
    h = mp.mpf("1e-5")
    cp, cm = chi(-1j * h), chi(1j * h)
    mean = float(mp.re((cp - cm) / (2 * h)))
    second = float(mp.re((cp + cm - 2) / h ** 2))
    return mean, math.sqrt(second - mean ** 2)


def test_no_wall_chi_matches_green_function_moments():
    import mpmath as mp
    mp.mp.dps = 60
    assert abs(complex(R.char_function_no_wall(0, MODEL, dps=60)) - 1.0) < 1e-40
    mean, sd = _mean_sd(lambda t: R.char_function_no_wall(t, MODEL, dps=60))
    walled = O.Model(m=MODEL.m, phi_in=MODEL.phi_in, phi_uv=MODEL.esc(), dN=MODEL.dN)
    mean_w, sd_w = _mean_sd(lambda t: R.char_function(t, walled, dps=60))
    mo = R.moments(MODEL)
    print(f"no wall: mean {mean:.9f}, sd {sd:.9f}; wall at phi_esc: mean {mean_w:.9f}, sd {sd_w:.9f}; "
          f"Green's function: {mo.mean:.9f}, {mo.std:.9f}")
    assert abs(mean / mo.mean - 1) < 1e-6
    assert abs(sd_w / mo.std - 1) < 1e-6
    assert 0 < sd / sd_w - 1 < 1e-3


def test_branch_cut_density_matches_simulated_runs():
    n = 100_000
    m = O.Model(m=1.0, phi_in=6.0, dN=1e-3, k_max=100_000)
    tr = O.simulate(m, 0, n)
    N = tr.k[tr.status == O.ST_ENDED] * m.dN
    # the simulated end is tested at step points: move the reference's end by beta S sqrt(dN)
    S_end = m.m * m.phi_end / (2 * math.pi * math.sqrt(6))
    shifted = O.Model(m=m.m, phi_in=m.phi_in, phi_end=m.phi_end - R.BGK_BETA * S_end * math.sqrt(m.dN))
    for c, w in ((8.0, 0.5), (10.0, 0.5), (12.0, 0.5), (15.0, 1.0), (20.0, 2.0)):
        cnt = int(np.sum((N > c - w / 2) & (N <= c + w / 2)))
        p_mc = cnt / (n * w)
        sig = math.sqrt(cnt) / (n * w)
        # bin average by Simpson's rule where the bin is wide enough for its curvature to matter
        if w > 0.5:
            p_ref = (R.pdf_no_wall(c - w / 2, shifted) + 4 * R.pdf_no_wall(c, shifted)
                     + R.pdf_no_wall(c + w / 2, shifted)) / 6
        else:
            p_ref = R.pdf_no_wall(c, shifted)
        print(f"N = {c}: simulated {p_mc:.4e} +- {sig:.1e}, branch cut {p_ref:.4e}")
        assert cnt >= 100
        assert abs(p_mc - p_ref) < 4 * sig + 0.02 * p_ref


def test_branch_cut_density_approaches_the_paper_asymptote():
    Ns = (1e4, 2e4, 4e4, 8e4)
    c = [R.pdf_no_wall(x, MODEL) * x ** 1.5 * math.exp(V0 * x / 4) for x in Ns]
    r = [c[i + 1] / c[i] for i in range(3)]
    print("successive ratios of P N^1.5 exp(v0 N/4):", r)
    # each doubling of N halves the distance to the constant (a 1/N correction)
    for a, b in zip(r, r[1:]):
        assert 0.4 < (1 - b) / (1 - a) < 0.6
    assert abs(r[-1] - 1) < 0.02
