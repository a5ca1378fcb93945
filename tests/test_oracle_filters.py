"""Pins of the oracle's filter functions against what the paper fixes.

Sec. 2.1 (eq:QU, eq:comp), Sec. 4.1 (eq:sch, eq:mexhat), Sec. 4.2 (B3 spline,
eq:splinewl, starlet U and Q), Sec. 4.3 (starlet compensated within 2 theta).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "b3_spline_values.txt")


def _golden_b3():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, b, c, d = (int(v) for v in line.split())
            rows.append((Fraction(a, b), Fraction(c, d)))
    return rows


def test_phi_matches_exact_values():
    for x, v in _golden_b3():
        assert O.phi_b3(float(x)) == pytest.approx(float(v), abs=1e-15)


def test_phi_textbook_values_and_support():
    # cubic B-spline: phi(0) = 2/3, phi(+-1) = 1/6, phi(+-2) = 0, zero beyond 2
    assert O.phi_b3(0.0) == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert O.phi_b3(1.0) == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert O.phi_b3(-1.0) == pytest.approx(1.0 / 6.0, abs=1e-15)
    assert O.phi_b3(2.0) == pytest.approx(0.0, abs=1e-15)
    x = np.linspace(2.0, 7.0, 101)
    assert np.all(np.abs(O.phi_b3(x)) < 1e-13)
    assert np.all(np.abs(O.phi_b3(-x)) < 1e-13)


def test_phi_partition_of_unity_and_unit_integral():
    # B-splines of integer knots sum to one over integer shifts
    x = np.linspace(-0.5, 0.5, 41)
    tot = sum(O.phi_b3(x - k) for k in range(-4, 5))
    assert np.max(np.abs(tot - 1.0)) < 1e-14
    xg, wg = np.polynomial.legendre.leggauss(8)
    integral = 0.0
    for lo in range(-2, 2):  # piecewise cubic between integers: exact quadrature
        integral += 0.5 * np.sum(wg * O.phi_b3(0.5 * xg + lo + 0.5))
    assert integral == pytest.approx(1.0, abs=1e-14)


def test_b3_taps_two_scale_relation_exact():
    # phi(x/2)/2 = sum_k h_k phi(x - k), checked in exact rationals on the
    # golden values (x on a 1/8 grid, so x/2 and x-k stay on the fixture grid)
    table = {x: v for x, v in _golden_b3()}
    h = [Fraction(int(round(v * 16)), 16) for v in O.b3_taps()]
    assert [float(v) for v in h] == list(O.b3_taps())
    for x in [Fraction(m, 8) for m in range(-16, 17) if m % 2 == 0]:
        lhs = table.get(x / 2, Fraction(0)) / 2
        rhs = sum(h[k + 2] * table.get(x - k, Fraction(0)) for k in range(-2, 3)
                  if abs(x - k) <= Fraction(5, 2))
        assert lhs == rhs, x


def test_starlet_U_is_axis_cut_of_separable_wavelet():
    eta = np.linspace(0.0, 2.6, 261)
    assert np.max(np.abs(O.starlet_U(eta) - O.starlet_U_from_phi(eta))) < 1e-13


def test_starlet_U_special_values():
    # U(0) = (2/3)(4 phi(0) - phi(0)) = 4/3; U(1/2) = (2/3)(4/6 - 23/48) = 1/8;
    # U(1) = (2/3)(0 - 1/6)... = -1/9; U = 0 beyond 2
    assert O.starlet_U(0.0) == pytest.approx(4.0 / 3.0, abs=1e-14)
    assert O.starlet_U(0.5) == pytest.approx(1.0 / 8.0, abs=1e-14)
    assert O.starlet_U(1.0) == pytest.approx(-1.0 / 9.0, abs=1e-14)
    assert np.all(np.abs(O.starlet_U(np.linspace(2.0, 4.0, 9))) < 1e-13)


def test_starlet_U_compensated_within_two_theta():
    # eq:comp at radius 2 theta (Sec. 4.3: the starlet U is compensated within 2 theta)
    xg, wg = np.polynomial.legendre.leggauss(10)
    tot = 0.0
    for lo in np.arange(0.0, 2.0, 0.5):  # piecewise cubic on half-integers
        t = 0.25 * xg + lo + 0.25
        tot += 0.25 * np.sum(wg * t * O.starlet_U(t))
    assert abs(tot) < 1e-14


def test_starlet_Q_matches_eq_QU():
    for eta in [0.05, 0.2, 0.3, 0.5, 0.7, 0.9, 1.0, 1.2, 1.5, 1.9]:
        q = O.Q_from_U(O.starlet_U, eta)
        assert O.starlet_Q(eta) == pytest.approx(q, abs=1e-12), eta


def test_starlet_Q_special_values_and_support():
    assert O.starlet_Q(0.0) == 0.0
    assert O.starlet_Q(0.5) == pytest.approx(19.0 / 40.0, abs=1e-13)
    assert O.starlet_Q(1.0) == pytest.approx(8.0 / 45.0, abs=1e-13)
    assert np.all(np.abs(O.starlet_Q(np.linspace(2.0, 5.0, 31))) < 1e-12)
    eta = np.linspace(0.0, 2.0, 20001)
    q = O.starlet_Q(eta)
    i = int(np.argmax(q))
    assert q[i] == pytest.approx(0.4827, abs=2e-4)
    assert eta[i] == pytest.approx(0.545, abs=5e-3)


@pytest.mark.parametrize("ell", [1, 2, 3])
def test_s98_Q_from_U_and_normalisations(ell):
    theta = 1.0
    U = lambda r: O.s98_U(r, theta, ell)  # noqa: E731
    for r in [0.1, 0.3, 0.5, 0.8, 0.99]:
        assert float(O.s98_Q(r, theta, ell)) == pytest.approx(O.Q_from_U(U, r), abs=1e-11)
    xg, wg = np.polynomial.legendre.leggauss(40)
    t = 0.5 * xg + 0.5
    # compensated within theta (eq:comp) and Q integrates to one over the plane
    assert abs(0.5 * np.sum(wg * t * U(t))) < 1e-14
    assert 0.5 * np.sum(wg * 2 * math.pi * t * O.s98_Q(t, theta, ell)) == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("b", [0.5, 4.0])
def test_jbj04_Q_from_U(b):
    theta = 3.0
    U = lambda r: O.jbj04_U(r, theta, b)  # noqa: E731
    for r in [0.5, 1.5, 3.0, 4.2, 6.0]:
        assert float(O.jbj04_Q(r, theta, b)) == pytest.approx(O.Q_from_U(U, r), abs=1e-12)
    # Q peaks at sqrt(1/b) theta; for b = 1/2 that is sqrt(2) theta (Sec. 4.1)
    r = np.linspace(0.0, 5 * theta, 200001)
    q = O.jbj04_Q(r, theta, b)
    assert r[int(np.argmax(q))] == pytest.approx(theta / math.sqrt(b), rel=1e-3)


def test_filter_Q_theta_scaling():
    th = 4.0
    Q = O.filter_Q_theta(O.FILTER_STARLET, th, 0.0)
    assert float(Q(2.0)) == pytest.approx(O.starlet_Q(0.5) / 16.0, abs=1e-15)
    assert O.natural_cut(O.FILTER_STARLET, th) == 8.0
    assert O.natural_cut(O.FILTER_S98, th) == 4.0
    assert O.natural_cut(O.FILTER_JBJ04, th) == 20.0
