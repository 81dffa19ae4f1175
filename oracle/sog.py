"""The u-series sum-of-Gaussians decomposition of 1/r (paper Sec. 2.2).

Test infrastructure only (see ``oracle/__init__``).

* Weights and widths: w_l = (pi/2)^(-1/2) b^(-l) log(b) / sigma for l >= 1,
  w_0 = omega (pi/2)^(-1/2) log(b) / sigma, s_l = sqrt(2) b^l sigma
  (Sec. 2.2, the weights/widths display after eq. SOGField, and the w_0
  display after eq. 2.22).
* Far part F(r) = sum_{l=0}^{M} w_l exp(-r^2/s_l^2) (eq. SOGField); near part
  N(r) = 1/r - F(r) for r < r_c and 0 beyond (eq. SOGDEcomp).
* (r0, omega) solve r0 F^1(r0) = 1 and r0^2 dF^1/dr(r0) = -1 with sigma = 1
  (eq. 2.35z and the paragraph after it), and r_c = r0 sigma.  The residuals of
  Table 1 vanish only when F^1 is the untruncated series over l >= 0, so the
  solve uses the infinite series.
"""
import math

import numpy as np

# Table 1 (tabl:parameter): b, r0, omega, energy error, M(energy), force error, M(force).
TABLE1 = (
    (2.0, 1.9892536839080267, 0.9944464927622323, 3.12e-2, 16, 9.93e-3, 11),
    (1.62976708826776469, 2.7520026668023417, 1.0078069793438068, 2.33e-3, 31, 6.21e-4, 16),
    (1.48783512395703226, 3.7554672283554990, 0.9919117057598183, 2.29e-4, 46, 7.98e-5, 26),
    (1.32070036405934420, 4.3914554711638349, 1.0018891411481198, 1.18e-6, 76, 5.76e-7, 41),
    (1.21812525709410644, 5.6355288151271085, 1.0009014615603334, 7.14e-10, 166, 5.14e-10, 71),
    (1.14878150173321925, 7.2956245490719404, 1.0000368348358225, 1.30e-15, 271, 1.98e-14, 116),
)


def weights(b, sigma, omega, M):
    """w_l and s_l for l = 0..M (Sec. 2.2, weights/widths displays)."""
    ell = np.arange(M + 1, dtype=np.float64)
    w = math.sqrt(2.0 / math.pi) * math.log(b) / sigma * b ** (-ell)
    w[0] *= omega
    s = math.sqrt(2.0) * b ** ell * sigma
    return w, s


def far(r, w, s):
    """F(r) = sum_l w_l exp(-r^2/s_l^2) (eq. SOGField), vectorised over r."""
    r = np.asarray(r, dtype=np.float64)
    return np.sum(w * np.exp(-(r[..., None] ** 2) / s ** 2), axis=-1)


def far_dr(r, w, s):
    """dF/dr = sum_l w_l (-2 r / s_l^2) exp(-r^2/s_l^2)."""
    r = np.asarray(r, dtype=np.float64)
    rr = r[..., None]
    return np.sum(w * (-2.0 * rr / s ** 2) * np.exp(-(rr ** 2) / s ** 2), axis=-1)


def near(r, w, s, rc):
    """N(r) = (1/r - F(r)) 1_{r<rc} (eq. SOGDEcomp)."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < rc, 1.0 / r - far(r, w, s), 0.0)


def _infinite_terms(b, omega, r):
    """w_l, s_l for sigma = 1 and every l >= 0 whose weight is above 1e-40 of w_1.

    The omitted tail sum_{l>L} w_l exp(-r^2/s_l^2) is below the geometric sum
    of the omitted weights, i.e. below 1e-40 relative."""
    L = int(math.ceil(40.0 * math.log(10.0) / math.log(b))) + 2
    return weights(b, 1.0, omega, L)


def continuity_residuals(b, r0, omega):
    """(r0 F^1(r0) - 1, r0^2 dF^1/dr(r0) + 1) with the untruncated series (eq. 2.35z)."""
    w, s = _infinite_terms(b, omega, r0)
    f = far(r0, w, s)
    fp = far_dr(r0, w, s)
    return float(r0 * f - 1.0), float(r0 * r0 * fp + 1.0)


def solve_r0_omega(b, r0_guess, omega_guess, iters=60):
    """Newton's method on the two C^1-continuity equations (eqs. 2.20, 2.22).

    Returns (r0, omega).  The root is not unique (Sec. 2.3 says so); the one
    returned is the one Newton reaches from the guess."""
    r0, om = float(r0_guess), float(omega_guess)
    for _ in range(iters):
        g = np.array(continuity_residuals(b, r0, om))
        if np.max(np.abs(g)) < 1e-15:
            break
        h0, h1 = 1e-7 * r0, 1e-7
        J = np.empty((2, 2))
        J[:, 0] = (np.array(continuity_residuals(b, r0 + h0, om)) - np.array(continuity_residuals(b, r0 - h0, om))) / (2 * h0)
        J[:, 1] = (np.array(continuity_residuals(b, r0, om + h1)) - np.array(continuity_residuals(b, r0, om - h1))) / (2 * h1)
        d = np.linalg.solve(J, -g)
        r0 += d[0]
        om += d[1]
    return r0, om


def table_row_for_tol(tol):
    """Smallest-M Table 1 row whose printed energy and force errors are both below tol/2."""
    for row in TABLE1:
        if row[3] <= 0.5 * tol and row[5] <= 0.5 * tol:
            return row
    return TABLE1[-1]


class SOG:
    """A resolved decomposition: b, sigma, omega, r_c, M and the arrays w, s."""

    def __init__(self, b, r0, omega, rc, M):
        self.b, self.r0, self.omega, self.rc, self.M = float(b), float(r0), float(omega), float(rc), int(M)
        self.sigma = self.rc / self.r0
        self.w, self.s = weights(self.b, self.sigma, self.omega, self.M)

    def split_index(self, eta, Lz):
        """m = max{l : s_l <= eta Lz}; -1 when every Gaussian is long-range (Sec. 3.1 definition and remark)."""
        idx = np.nonzero(self.s <= eta * Lz)[0]
        return int(idx[-1]) if idx.size else -1

    def self_coeff(self):
        """Phi_self_i = q_i sum_{l=0}^{M} w_l (eq. phiNDR)."""
        return float(np.sum(self.w))
