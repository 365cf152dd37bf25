"""One-ray accuracy study of Sect. 3.4: short-characteristics formal solvers on the
sigmoid source function (Eqs. ssigmas, sigma) against the analytic intensity (Eq.
analyti), as the maximum true error E(Delta tau) over -12 <= z < 12.

TEST INFRASTRUCTURE.  Only the tests may import this module.

Methods (constant opacity, Delta z = Delta tau, unpolarised):
  linear     linear interpolation of S between M and O
  parabolic  quadratic Bezier with the control point of the parabola through M, O, P
             (BESSER stopped after step 4; the DELOPAR choice)
  besser     the BESSER control point (Sect. 3.2)
  bezier     quadratic Bezier whose control point uses the Fritsch-Butland weighted
             harmonic mean of the two slopes as the derivative at O (zero where the
             slopes differ in sign), with no overshoot test
  cbezier    as bezier, with c_M clipped to the range of y_M, y_O
The last node has no downwind point; it takes the chord midpoint as control point and
is left out of E.

Other readings of the Bezier solvers (solve_ray_reading), each on the nodes of
[-12, 12] with the analytic source at ghost nodes beyond both ends, so that every
interval takes its full rule and E covers every node:
  bezier_o   tangent at O from the Fritsch-Butland derivative (as bezier above)
  bezier_m   tangent at M: c = y_M + h y'_M / 2, y'_M from the triple around M
  bezier_mo  the mean of those two control points
and each with the clip of c_M to the range of y_M, y_O (prefix c).
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as orc

METHODS = ("linear", "parabolic", "besser", "bezier", "cbezier")
Z_MIN, Z_MAX = -12.0, 12.0


def sigmoid(a, d, z):
    return 1.0 / (1.0 + np.exp(-a * (z - d)))


def source(z):
    """Eq. ssigmas: S(z) = sigma(2, -5, z) sigma(-2, 5, z)."""
    return sigmoid(2.0, -5.0, z) * sigmoid(-2.0, 5.0, z)


def intensity(z):
    """Eq. analyti: analytic intensity towards +z with I(-inf) = 0."""
    z = np.asarray(z, dtype=np.float64)
    return (np.exp(15.0 - z) / (math.exp(20.0) - 1.0)
            * (math.exp(10.0) * np.arctan(np.exp(z - 5.0)) - np.arctan(np.exp(z + 5.0))))


def fritsch_butland(yM, yO, yP, hM, hP):
    """Weighted harmonic mean of the slopes d_M, d_P (Fritsch & Butland 1984):
    1/y' = alpha/d_M + (1 - alpha)/d_P with alpha = (1 + h_P/(h_M + h_P))/3, and y' = 0
    where the slopes differ in sign."""
    dM, dP = (yO - yM) / hM, (yP - yO) / hP
    if dM * dP <= 0.0:
        return 0.0
    alpha = (1.0 + hP / (hM + hP)) / 3.0
    return dM * dP / (alpha * dP + (1.0 - alpha) * dM)


def control_point(method, yM, yO, yP, hM, hP):
    if method == "besser":
        return orc.besser_cm(yM, yO, yP, hM, hP)
    if method == "parabolic":
        return orc.parabolic_cm(yM, yO, yP, hM, hP)
    c = yO - 0.5 * hM * fritsch_butland(yM, yO, yP, hM, hP)
    if method == "cbezier":
        c = min(max(c, min(yM, yO)), max(yM, yO))
    return c


def solve_ray(z, S, i0, method):
    """Intensity at the nodes z (increasing) along the ray, I(z[0]) = i0."""
    n = len(z)
    out = np.empty(n)
    out[0] = i0
    for k in range(1, n):
        h = z[k] - z[k - 1]
        e, psi_m, psi_o, om_m, om_o, om_c = orc.coefficients(h)
        if method == "linear":
            out[k] = e * out[k - 1] + psi_m * S[k - 1] + psi_o * S[k]
            continue
        if k < n - 1:
            c = control_point(method, S[k - 1], S[k], S[k + 1], h, z[k + 1] - z[k])
        else:
            c = 0.5 * (S[k - 1] + S[k])
        out[k] = e * out[k - 1] + om_m * S[k - 1] + om_o * S[k] + om_c * c
    return out


def max_true_error(nodes, method):
    """E for a uniform grid of `nodes` points on [-12, 12]."""
    z = np.linspace(Z_MIN, Z_MAX, nodes)
    ia = intensity(z)
    i = solve_ray(z, source(z), ia[0], method)
    return float(np.max(np.abs((i[:-1] - ia[:-1]) / ia[:-1])))


def error_table(node_counts=(9, 13, 17, 25, 33, 49, 97, 193, 385)):
    """{method: [(Delta tau, E), ...]}."""
    return {m: [((Z_MAX - Z_MIN) / (n - 1), max_true_error(n, m)) for n in node_counts]
            for m in METHODS}


def solve_ray_reading(nodes, reading):
    """E for `nodes` uniform points on [-12, 12] with one of the readings above."""
    z = np.linspace(Z_MIN, Z_MAX, nodes)
    h = z[1] - z[0]
    S = source(np.r_[z[0] - 2 * h, z[0] - h, z, z[-1] + h])   # S[k + 2] is the source at z[k]
    ia = intensity(z)
    out = np.empty(nodes)
    out[0] = ia[0]
    base = reading.lstrip("c")
    for k in range(1, nodes):
        yMM, yM, yO, yP = S[k], S[k + 1], S[k + 2], S[k + 3]
        e, psi_m, psi_o, om_m, om_o, om_c = orc.coefficients(h)
        cO = yO - 0.5 * h * fritsch_butland(yM, yO, yP, h, h)
        cM = yM + 0.5 * h * fritsch_butland(yMM, yM, yO, h, h)
        c = {"bezier_o": cO, "bezier_m": cM, "bezier_mo": 0.5 * (cO + cM)}[base]
        if reading.startswith("c"):
            c = min(max(c, min(yM, yO)), max(yM, yO))
        out[k] = e * out[k - 1] + om_m * yM + om_o * yO + om_c * c
    return float(np.max(np.abs((out - ia) / ia)))
