"""Filter functions of the aperture-mass statistic and of the starlet (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows Sec. 2.1 (eq:mapdef, eq:shearmap, eq:QU, eq:comp) and Sec. 4
(eq:sch, eq:mexhat, eq:splinewl, the B3 spline, and the starlet U(eta), Q(eta)).

Pins (tests/test_oracle_filters.py):
  * phi_b3 values at the integers and half-integers, unit integral, support;
  * b3_taps from the two-scale relation of the B3 spline, in exact rationals;
  * printed starlet U(eta) equals the axis cut of the separable wavelet of
    eq:splinewl, (2/3)[4 phi(2 eta) - phi(eta)];
  * printed starlet Q(eta) equals eq:QU applied to U by quadrature, and
    vanishes for eta >= 2; U is compensated within 2 theta (eq:comp);
  * S98 Q from eq:QU of the S98 U; S98 compensation within theta;
    the S98 Q integrates to 1 over the plane;
  * JBJ04 Q from eq:QU of the JBJ04 U (A = 1).
"""

import math

import numpy as np

FILTER_STARLET = 0
FILTER_S98 = 1
FILTER_JBJ04 = 2


def phi_b3(x):
    """Cubic B-spline scaling function of the starlet (Sec. 4.2, B3 spline).

    phi(x) = (|x-2|^3 - 4|x-1|^3 + 6|x|^3 - 4|x+1|^3 + |x+2|^3) / 12,
    identically zero for |x| > 2.
    """
    x = np.asarray(x, dtype=np.float64)
    return (np.abs(x - 2) ** 3 - 4 * np.abs(x - 1) ** 3 + 6 * np.abs(x) ** 3
            - 4 * np.abs(x + 1) ** 3 + np.abs(x + 2) ** 3) / 12.0


def b3_taps():
    """Discrete low-pass filter of the a trous algorithm for the B3 spline.

    The paper prints only phi (Sec. 4.2); the filter bank of the fast
    transform is the h of the two-scale relation phi(x/2)/2 = sum_k h_k
    phi(x - k), which for the cubic B-spline is (1, 4, 6, 4, 1)/16.  The
    relation itself is checked in exact arithmetic by the tests.
    """
    return np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


def starlet_U(eta):
    """Starlet aperture-mass filter U(eta), eta = vartheta/theta, as printed
    in Sec. 4.2 (the evaluation of eq:splinewl)."""
    e = np.asarray(eta, dtype=np.float64)
    a = np.abs
    return (93.0 * a(e) ** 3
            - 64.0 * (a(0.5 - e) ** 3 + a(0.5 + e) ** 3)
            + 18.0 * (a(1.0 - e) ** 3 + a(1.0 + e) ** 3)
            - 0.5 * (a(2.0 - e) ** 3 + a(2.0 + e) ** 3)) / 9.0


def starlet_U_from_phi(eta):
    """Axis cut psi(eta, 0) of the separable starlet wavelet of eq:splinewl:
    psi(u, v) = 4 phi(2u) phi(2v) - phi(u) phi(v), so psi(eta, 0) =
    phi(0) [4 phi(2 eta) - phi(eta)] with phi(0) = 2/3."""
    e = np.asarray(eta, dtype=np.float64)
    return phi_b3(0.0) * (4.0 * phi_b3(2.0 * e) - phi_b3(e))


def starlet_Q(eta):
    """Starlet tangential-shear filter Q(eta) as printed in Sec. 4.2.

    The printed expression has a removable 1/eta^2 singularity at 0; Q(0) = 0
    (Q is the difference of the mean of U inside the radius and U at the
    radius, eq:QU, and both tend to U(0)).  For eta >= 2 the expression is
    identically zero because U is compensated within 2 theta (Sec. 4.3).
    """
    e = np.atleast_1d(np.asarray(eta, dtype=np.float64))
    out = np.zeros_like(e)
    nz = e != 0.0
    x = e[nz]
    a = np.abs
    num = (-279.0 * x ** 2 * a(x) ** 3
           + 8.0 * (1.0 + 6.0 * x + 24.0 * x ** 2) * a(0.5 - x) ** 3
           - 9.0 * (1.0 + 3.0 * x + 6.0 * x ** 2) * a(1.0 - x) ** 3
           - 9.0 * (1.0 - 3.0 * x + 6.0 * x ** 2) * a(1.0 + x) ** 3
           + (1.0 + 1.5 * x + 1.5 * x ** 2) * a(2.0 - x) ** 3
           + (1.0 - 1.5 * x + 1.5 * x ** 2) * a(2.0 + x) ** 3
           + 8.0 * (1.0 - 6.0 * x + 24.0 * x ** 2) * a(0.5 + x) ** 3)
    out[nz] = num / (45.0 * x ** 2)
    return out.reshape(np.shape(eta)) if np.ndim(eta) else float(out[0])


def Q_from_U(U, r, n_seg=16):
    """eq:QU: Q(r) = (2/r^2) int_0^r r' U(r') dr' - U(r), by 32-point
    Gauss-Legendre quadrature on ``n_seg`` equal pieces of [0, r], further
    split at the half-integer breakpoints of piecewise polynomials.

    ``U`` is a vectorised callable.  Used to pin the closed-form Q's.
    """
    r = float(r)
    if r == 0.0:
        return 0.0
    # The piecewise-cubic starlet U has its breakpoints at multiples of 1/2;
    # splitting there makes the quadrature exact to rounding for it.
    pts = set(np.linspace(0.0, r, n_seg + 1).tolist())
    pts |= {b for b in (0.5, 1.0, 1.5, 2.0, 2.5, 3.0) if b < r}
    pts = sorted(pts)
    xg, wg = np.polynomial.legendre.leggauss(32)
    total = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        t = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
        total += 0.5 * (hi - lo) * np.sum(wg * t * U(t))
    return 2.0 * total / r ** 2 - float(U(np.array([r]))[0])


def s98_U(vt, theta, ell):
    """Schneider et al. (1998) polynomial U filter with Heaviside cut, eq:sch."""
    vt = np.asarray(vt, dtype=np.float64)
    x2 = (vt / theta) ** 2
    val = ((ell + 2.0) ** 2 / (math.pi * theta ** 2)
           * (1.0 - x2) ** ell * (1.0 / (ell + 2.0) - x2))
    return np.where(vt <= theta, val, 0.0)


def s98_Q(vt, theta, ell):
    """Schneider et al. (1998) polynomial Q filter with Heaviside cut, eq:sch.
    The Heaviside step is 1 for vartheta <= theta (Sec. 4.1)."""
    vt = np.asarray(vt, dtype=np.float64)
    x2 = (vt / theta) ** 2
    val = ((1.0 + ell) * (2.0 + ell) / (math.pi * theta ** 2)
           * x2 * (1.0 - x2) ** ell)
    return np.where(vt <= theta, val, 0.0)


def jbj04_U(vt, theta, b, A=1.0):
    """Gaussian-type U filter of eq:mexhat (van Waerbeke 1998 with b = 4,
    Jarvis et al. 2004 with b = 1/2).  The normalisation A is left free by
    the paper; A = 1 here."""
    vt = np.asarray(vt, dtype=np.float64)
    x2 = b * (vt / theta) ** 2
    return A / theta ** 2 * (1.0 - x2) * np.exp(-x2)


def jbj04_Q(vt, theta, b, A=1.0):
    """Gaussian-type Q filter of eq:mexhat (A = 1)."""
    vt = np.asarray(vt, dtype=np.float64)
    x2 = b * (vt / theta) ** 2
    return A / theta ** 2 * x2 * np.exp(-x2)


def natural_cut(filt, theta):
    """Truncation radius used when the caller passes cut <= 0.

    starlet: 2 theta (Q vanishes beyond, Sec. 4.3); S98: theta (its Heaviside
    support, eq:sch); JBJ04: 5 theta (the truncation the paper calls
    essentially exact, Sec. 4.3).
    """
    if filt == FILTER_STARLET:
        return 2.0 * theta
    if filt == FILTER_S98:
        return float(theta)
    if filt == FILTER_JBJ04:
        return 5.0 * theta
    raise ValueError("unknown filter %r" % (filt,))


def filter_Q_theta(filt, theta, fparam):
    """Return the callable vartheta -> Q_theta(vartheta) in pixel units.

    The starlet filter is dimensionless in eta; it is scaled as
    Q_theta(vt) = Q(vt/theta)/theta^2 (pixel area 1), like the other two,
    whose printed forms already carry the 1/theta^2.
    """
    if filt == FILTER_STARLET:
        return lambda vt: starlet_Q(np.asarray(vt, dtype=np.float64) / theta) / theta ** 2
    if filt == FILTER_S98:
        return lambda vt: s98_Q(vt, theta, fparam)
    if filt == FILTER_JBJ04:
        return lambda vt: jbj04_Q(vt, theta, fparam)
    raise ValueError("unknown filter %r" % (filt,))
