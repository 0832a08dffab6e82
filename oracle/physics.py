"""Physical kernel of the Zheleznyak photoionization model, in FP64 (oracle side).

Lin & Zhuang, Sec. 2.1:
  eq. (1)  S_ph(x) = integral over the source chamber of I(y) g(|x-y|) / (4 pi |x-y|^2) dy
  eq. (2)  I = xi * p_q/(p+p_q) * (omega/alpha) * S_i
  eq. (3)  g(r) = (exp(-chi_min pO2 r) - exp(-chi_max pO2 r)) / (r ln(chi_max/chi_min))
with chi_min = 0.035 and chi_max = 2 cm^-1 Torr^-1.

Reading used throughout: the bare source handed in is S_i-like and the
prefactor P = p_q/(p+p_q) * (xi omega/alpha) multiplies the result; the
oxygen partial pressure is pO2 = o2_fraction * p.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class GasConstants:
    p_torr: float
    pO2: float
    a: float        # chi_min * pO2, cm^-1
    b: float        # chi_max * pO2, cm^-1
    L: float        # ln(chi_max / chi_min)
    P: float        # p_q/(p+p_q) * xi*omega/alpha


def gas_constants(gas: dict) -> GasConstants:
    """Constants of eqs. (2)-(3) from a gas description (Sec. 2.1; Sec. 4.1 parameters)."""
    p = float(gas["p_torr"])
    pO2 = float(gas["o2_fraction"]) * p
    a = float(gas["chi_min"]) * pO2
    b = float(gas["chi_max"]) * pO2
    L = float(np.log(float(gas["chi_max"]) / float(gas["chi_min"])))
    P = float(gas["pq_torr"]) / (p + float(gas["pq_torr"])) * float(gas["xi_omega_over_alpha"])
    return GasConstants(p, pO2, a, b, L, P)


def g_absorption(r, gc: GasConstants):
    """g(r) of eq. (3), written exactly as printed (difference of exponentials over r L)."""
    r = np.asarray(r, dtype=np.float64)
    return (np.exp(-gc.a * r) - np.exp(-gc.b * r)) / (r * gc.L)


def kernel_K(r, gc: GasConstants):
    """K(r) = g(r) / (4 pi r^2), the integrand weight of eq. (1) per unit source.

    Evaluated as exp(-a r) * (-expm1(-(b-a) r)) / (4 pi L r^3), which equals the
    printed difference of exponentials but has no cancellation when (b-a) r is small.
    """
    r = np.asarray(r, dtype=np.float64)
    return np.exp(-gc.a * r) * (-np.expm1(-(gc.b - gc.a) * r)) / (4.0 * np.pi * gc.L * r ** 3)


def _g_series_safe(r, gc: GasConstants):
    # same function as g_absorption, evaluated without cancellation near r = 0
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    small = r == 0.0
    rr = np.where(small, 1.0, r)
    out[:] = np.exp(-gc.a * rr) * (-np.expm1(-(gc.b - gc.a) * rr)) / (rr * gc.L)
    out[small] = (gc.b - gc.a) / gc.L
    return out


_GL16 = np.polynomial.legendre.leggauss(16)


def absorbed_fraction(R, gc: GasConstants, panels: int = 48):
    """A(R) = integral_0^R g(r) dr: fraction of emitted photons absorbed within radius R.

    Since integral over R^3 of K = integral_0^inf g = 1 (Frullani), A(R) is also the
    integral of K over the ball of radius R.  Computed by Gauss-Legendre (16 nodes) on
    geometrically graded panels [R 2^-k-1, R 2^-k], which resolve the exp(-b r)
    boundary layer near r = 0 for any R.
    """
    R = np.atleast_1d(np.asarray(R, dtype=np.float64))
    x, wq = _GL16
    edges = np.concatenate([[0.0], 0.5 ** np.arange(panels - 1, -1, -1, dtype=np.float64)])
    lo, hi = edges[:-1], edges[1:]                      # panels of [0, 1]
    # nodes on [0,1]: (panels*16,)
    t = (0.5 * (hi - lo)[:, None] * (x[None, :] + 1.0) + lo[:, None]).ravel()
    wt = (0.5 * (hi - lo)[:, None] * wq[None, :]).ravel()
    out = np.empty_like(R)
    for k, Rk in enumerate(R):
        out[k] = Rk * np.dot(wt, _g_series_safe(Rk * t, gc))
    return out


def cube_self_coefficient(h: float, gc: GasConstants, n_face: int = 64) -> float:
    """c_self(h): integral of K over a cube of side h centred on the evaluation point.

    The discrete kernel's diagonal (reading of the deferred discrete G of eq. (15)):
    with I constant over the own cell, that cell contributes I * integral_cell K.
    In spherical coordinates the radial integral of K r^2 is A(R)/(4 pi), so
      c_self = (1/4 pi) * integral over directions of A(R(direction)),
    and over the 6 faces (face z = h/2, point (u, v, h/2), rho^2 = u^2+v^2+h^2/4,
    solid angle element (h/2)/rho^3 du dv):
      c_self = (6 / 4 pi) * double integral over [-h/2, h/2]^2 of A(rho) (h/2) / rho^3.
    Gauss-Legendre tensor rule on the face (the integrand is smooth there).
    """
    x, wq = np.polynomial.legendre.leggauss(n_face)
    u = 0.5 * h * x
    wu = 0.5 * h * wq
    U, V = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu)
    rho = np.sqrt(U ** 2 + V ** 2 + 0.25 * h * h).ravel()
    A = absorbed_fraction(rho, gc)
    integrand = A * (0.5 * h) / rho ** 3
    return float(6.0 / (4.0 * np.pi) * np.dot(W.ravel(), integrand))
