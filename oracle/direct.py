"""SOG-direct: the exact value of each term of the SOG decomposition, with no
grids, windows, FFTs or polynomial interpolation.

Test infrastructure only (see ``oracle/__init__``).

For a target i (eqs. SOGdecomp, phiNDR, trun2, splitting/phisplit):

  Phi_i = Phi^N_i + Phi^mid_i + Phi^long_i - Phi^self_i

  Phi^N_i    = sum'_{j,n} q_j N(|r_ij + n o L|),  N(r) = (1/r - F(r)) 1_{r<r_c}
  Phi^mid_i  = sum_j q_j sum_n sum_{l<=m} w_l exp(-|r_ij + n o L|^2 / s_l^2)
  Phi^long_i = sum_j q_j sum_n sum_{l>m}  w_l exp(-|r_ij + n o L|^2 / s_l^2)
  Phi^self_i = q_i sum_{l=0}^{M} w_l

where n runs over the xy image lattice (n_z = 0) and the far sums include
j = i (the n = 0 self image is what Phi^self removes; the sign follows
eq. phisplit, the reading taken where eq. splitting prints +Phi^self).

Each Gaussian's xy-lattice sum is evaluated either as a real-space image sum
or, by the Poisson summation formula (App. A.5), in 2D Fourier space:

  sum_n exp(-|r + n o L|^2/s^2) = (pi s^2/A) exp(-z^2/s^2) sum_{k in K^2} exp(-s^2 k^2/4) cos(k . r_xy)

(the same identity that gives eq. trun2).  For a neutral system the k = 0
constant pi s^2/A multiplies sum_j q_j = 0, so the k = 0 term is evaluated as
(pi s^2/A) expm1(-z^2/s^2), which is mathematically identical and avoids
cancelling huge numbers for the very wide Gaussians.  Whichever of the two
forms is cheaper is used per Gaussian; both are truncated where the terms fall
below 1e-17 relative.  Gradients are the analytic derivatives with respect to
r_i.
"""
import math

import numpy as np

from .sog import SOG

_CUT = math.sqrt(math.log(1e17))  # exp(-CUT^2) = 1e-17


def _min_image(d, box):
    d = d.copy()
    d[:, 0] -= box[0] * np.round(d[:, 0] / box[0])
    d[:, 1] -= box[1] * np.round(d[:, 1] / box[1])
    return d


def gaussian_lattice_sum(d, qj, s, box, grad=True):
    """sum_j q_j sum_n exp(-|d_j + n o L|^2/s^2) and its gradient in d, for one target.

    d: (N,3) minimum-image displacements r_i - r_j, qj: (N,) charges.
    Chooses real space or the Poisson-summed Fourier form by estimated cost."""
    Lx, Ly, _ = box
    A = Lx * Ly
    R = _CUT * s  # real-space radius
    nxm, nym = int(math.ceil(R / Lx + 0.5)), int(math.ceil(R / Ly + 0.5))  # d is a minimum image, |d_x| <= Lx/2
    cost_real = (2 * nxm + 1) * (2 * nym + 1)
    K = 2.0 * _CUT / s  # Fourier radius
    mx, my = int(math.floor(K * Lx / (2 * math.pi))), int(math.floor(K * Ly / (2 * math.pi)))
    cost_four = (2 * mx + 1) * (my + 1)
    g = np.zeros(3)
    if cost_real <= cost_four:
        val = 0.0
        for nx in range(-nxm, nxm + 1):
            for ny in range(-nym, nym + 1):
                dd = d + np.array([nx * Lx, ny * Ly, 0.0])
                r2 = np.sum(dd * dd, axis=1)
                e = qj * np.exp(-r2 / (s * s))
                val += e.sum()
                if grad:
                    g += (-2.0 / (s * s)) * (e @ dd)
        return val, g
    z = d[:, 2]
    ez = np.exp(-(z * z) / (s * s))
    pref = math.pi * s * s / A
    # k = 0 term, written with expm1 (its constant part multiplies sum q_j = 0)
    val = pref * float(qj @ np.expm1(-(z * z) / (s * s)))
    if grad:
        g[2] += pref * float(qj @ ((-2.0 * z / (s * s)) * ez))
    # k != 0: half plane doubled
    for ny in range(0, my + 1):
        nxs = np.arange(-mx, mx + 1) if ny > 0 else np.arange(1, mx + 1)
        if nxs.size == 0:
            continue
        kx = 2 * math.pi * nxs / Lx
        ky = 2 * math.pi * ny / Ly
        ek = np.exp(-(s * s) * (kx * kx + ky * ky) / 4.0)
        keep = ek > 1e-17
        if not np.any(keep):
            continue
        kx, ek = kx[keep], ek[keep]
        ph = np.outer(kx, d[:, 0]) + ky * d[:, 1][None, :]
        c, sn = np.cos(ph), np.sin(ph)
        w = qj * ez
        val += 2.0 * pref * float(ek @ (c @ w))
        if grad:
            g[0] += 2.0 * pref * float((ek * kx) @ (-(sn @ w)))
            g[1] += 2.0 * pref * float(ek @ (-(sn @ w))) * ky
            g[2] += 2.0 * pref * float(ek @ (c @ (qj * ez * (-2.0 * z / (s * s)))))
    return val, g


def sog_direct(x, q, box, sog: SOG, m, targets):
    """Exact SOG terms for the given targets.

    x: (N,3) positions in [0,Lx)x[0,Ly)x[0,Lz] (only differences matter), q: (N,),
    sog: the decomposition, m: last mid-range index (-1: no mid range).
    Returns a dict of arrays over targets: phi_near, grad_near, phi_mid, grad_mid,
    phi_long, grad_long, phi_self, phi (total), grad (total)."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = tuple(float(v) for v in box)
    if abs(q.sum()) > 1e-10 * np.abs(q).sum():
        raise ValueError("SOG-direct needs a charge-neutral system")
    targets = np.asarray(targets)
    T = targets.size
    out = {k: np.zeros(T) for k in ("phi_near", "phi_mid", "phi_long", "phi_self")}
    for k in ("grad_near", "grad_mid", "grad_long"):
        out[k] = np.zeros((T, 3))
    w, s, rc = sog.w, sog.s, sog.rc
    for a, i in enumerate(targets):
        d = _min_image(x[i] - x, box)
        # near field: minimum image suffices because r_c <= min(Lx, Ly)/2 (Assumption ass:SOG)
        r = np.sqrt(np.sum(d * d, axis=1))
        nb = (r < rc) & (np.arange(x.shape[0]) != i)
        rn, dn, qn = r[nb], d[nb], q[nb]
        F = np.sum(w * np.exp(-(rn[:, None] ** 2) / s ** 2), axis=1)
        Fp = np.sum(w * (-2.0 * rn[:, None] / s ** 2) * np.exp(-(rn[:, None] ** 2) / s ** 2), axis=1)
        out["phi_near"][a] = qn @ (1.0 / rn - F)
        dN = -1.0 / rn ** 2 - Fp  # N'(r)
        out["grad_near"][a] = (qn * dN / rn) @ dn
        for ell in range(sog.M + 1):
            v, g = gaussian_lattice_sum(d, q, s[ell], box)
            key = "mid" if ell <= m else "long"
            out["phi_" + key][a] += w[ell] * v
            out["grad_" + key][a] += w[ell] * g
        out["phi_self"][a] = q[i] * np.sum(w)
    out["phi"] = out["phi_near"] + out["phi_mid"] + out["phi_long"] - out["phi_self"]
    out["grad"] = out["grad_near"] + out["grad_mid"] + out["grad_long"]
    return out
