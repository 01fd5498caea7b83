"""Pins of the oracle's Friedmann quadrature (Eq. (2)) and step coefficients
(the kick and drift integrals of Eq. (9)) to closed forms.

For one-component universes the integrals t = int da/(aH),
K = int da/(a^2 H) and D = int da/(a^3 H) have elementary antiderivatives;
flat LCDM has t(a) = 2/(3 H0 sqrt(OL)) asinh(sqrt(OL/OM) a^{3/2}), and
Einstein-de Sitter gives a proportional to t^{2/3}.
"""
import math

import numpy as np
import pytest

import oracle

H0 = 1.7

CASES = {
    # name: (Om_R, Om_M, Om_K, Om_L, t(a1,a2), K(a1,a2), D(a1,a2))
    "matter": ((0, 1, 0, 0),
               lambda a1, a2: 2 * (a2 ** 1.5 - a1 ** 1.5) / (3 * H0),
               lambda a1, a2: 2 * (math.sqrt(a2) - math.sqrt(a1)) / H0,
               lambda a1, a2: 2 * (a1 ** -0.5 - a2 ** -0.5) / H0),
    "radiation": ((1, 0, 0, 0),
                  lambda a1, a2: (a2 ** 2 - a1 ** 2) / (2 * H0),
                  lambda a1, a2: (a2 - a1) / H0,
                  lambda a1, a2: math.log(a2 / a1) / H0),
    "curvature": ((0, 0, 1, 0),
                  lambda a1, a2: (a2 - a1) / H0,
                  lambda a1, a2: math.log(a2 / a1) / H0,
                  lambda a1, a2: (1 / a1 - 1 / a2) / H0),
    "lambda": ((0, 0, 0, 1),
               lambda a1, a2: math.log(a2 / a1) / H0,
               lambda a1, a2: (1 / a1 - 1 / a2) / H0,
               lambda a1, a2: (a1 ** -2 - a2 ** -2) / (2 * H0)),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("a1,a2", [(0.02, 1.0), (0.1, 0.1003), (0.5, 2.0), (1.0, 0.3)])
def test_single_component_closed_forms(name, a1, a2):
    om, t_f, k_f, d_f = CASES[name]
    for kind, f in (("time", t_f), ("kick", k_f), ("drift", d_f)):
        got = oracle.time_integral(kind, a1, a2, H0, *om)
        want = f(a1, a2)
        assert abs(got - want) <= 1e-13 * abs(want), (kind, got, want)


def test_hubble_rate_is_eq2():
    # sum of components: H^2 adds linearly in the four density terms
    a = 0.37
    h2 = sum(oracle.hubble(a, H0, *om) ** 2 for om in
             [(0.1, 0, 0, 0), (0, 0.4, 0, 0), (0, 0, 0, 0.7)])
    h2 -= oracle.hubble(a, H0, 0, 0, 0.2, 0) ** 2
    assert abs(oracle.hubble(a, H0, 0.1, 0.4, -0.2, 0.7) ** 2 - h2) < 1e-13 * h2
    # single components scale as a^-4, a^-3, a^-2, a^0
    for om, p in (((1, 0, 0, 0), -2), ((0, 1, 0, 0), -1.5), ((0, 0, 1, 0), -1), ((0, 0, 0, 1), 0)):
        assert abs(oracle.hubble(a, H0, *om) - H0 * a ** p) < 1e-15 * H0 * a ** p
    assert math.isnan(oracle.hubble(0.9, 1.0, 0, 1, -2, 0))


def test_flat_lcdm_time():
    OM, OL = 0.3, 0.7
    t = lambda a: 2 / (3 * H0 * math.sqrt(OL)) * math.asinh(math.sqrt(OL / OM) * a ** 1.5)
    for a1, a2 in ((1 / 51, 1.0), (0.2, 0.25), (0.5, 3.0)):
        got = oracle.time_integral("time", a1, a2, H0, 0, OM, 0, OL)
        assert abs(got - (t(a2) - t(a1))) <= 1e-13 * (t(a2) - t(a1))


def test_eds_a_proportional_to_t_two_thirds():
    # t(a) - t(0) = 2 a^{3/2} / (3 H0): a(t) = (3 H0 t / 2)^{2/3}
    h0 = math.sqrt(8 * math.pi / 3)
    for a in (0.1, 0.5, 1.0):
        t = oracle.time_integral("time", 1e-12, a, h0, 0, 1, 0, 0) + 2 * 1e-18 / (3 * h0)
        assert abs((1.5 * h0 * t) ** (2 / 3) - a) < 1e-13 * a


def test_step_coefficients_split_in_ln_a():
    cos = dict(H0=H0, Om_R=0.0, Om_M=0.3, Om_K=0.0, Om_L=0.7)
    a_b, a_e, n = 1 / 51, 1.0, 10
    delta = math.log(a_e / a_b) / n
    total_d = 0.0
    for step in range(n):
        k1, d, k2, dt = oracle.step_coefficients(cos, a_b, a_e, n, step)
        a0 = a_b * math.exp(step * delta)
        ah = a_b * math.exp((step + 0.5) * delta)
        a1 = a_e if step == n - 1 else a_b * math.exp((step + 1) * delta)
        args = (H0, 0.0, 0.3, 0.0, 0.7)
        assert k1 == pytest.approx(oracle.time_integral("kick", a0, ah, *args), rel=1e-14)
        assert k2 == pytest.approx(oracle.time_integral("kick", ah, a1, *args), rel=1e-14)
        assert d == pytest.approx(oracle.time_integral("drift", a0, a1, *args), rel=1e-14)
        assert dt == pytest.approx(oracle.time_integral("time", a0, a1, *args), rel=1e-14)
        total_d += d
    assert total_d == pytest.approx(oracle.time_integral("drift", a_b, a_e, H0, 0, 0.3, 0, 0.7),
                                    rel=1e-13)
    # static limit: a fixed, dt = span / n_steps
    k1, d, k2, dt = oracle.step_coefficients(dict(H0=0.0, Om_R=0, Om_M=0, Om_K=0, Om_L=0),
                                             0.5, 2.0, 4, 1)
    assert (k1, d, k2, dt) == (0.5 * 0.5 / 0.5, 0.5 / 0.25, 0.5 * 0.5 / 0.5, 0.5)
