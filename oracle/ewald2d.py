"""Ewald2D: the O(N^2) reference the paper measures every error against (Sec. 5).

Test infrastructure only (see ``oracle/__init__``).

The paper cites Parry (1975) for Ewald2D but does not print the formula.  This
module writes the standard form of the quasi-2D Ewald sum in Gaussian units
(Phi_i = sum_j sum'_n q_j / |r_ij + n o L|, eq. Phi) from the mathematics: the
Ewald screening splits 1/r into erfc(alpha r)/r plus erf(alpha r)/r, and the
smooth part is summed over the 2D reciprocal lattice with the z integral done
in closed form:

  Phi_i = sum_j sum'_n q_j erfc(alpha |r_ij+n|)/|r_ij+n|
        + (pi/A) sum_j q_j sum_{k != 0} cos(k.r_ij)/|k|
              [e^{|k| z_ij} erfc(|k|/(2 alpha) + alpha z_ij)
             + e^{-|k| z_ij} erfc(|k|/(2 alpha) - alpha z_ij)]
        - (2 pi/A) sum_j q_j [z_ij erf(alpha z_ij) + exp(-alpha^2 z_ij^2)/(alpha sqrt(pi))]
        - 2 alpha q_i / sqrt(pi),

valid for a charge-neutral cell (Prop. lem::summation).  The value does not
depend on alpha; the tests use that as one of the pins.  Each product
e^{+-kz} erfc(.) is evaluated through erfcx to avoid overflow.
"""
import math

import numpy as np
from scipy.special import erfc, erf, erfcx


def _pair_geometry(x, box, targets):
    x = np.asarray(x, dtype=np.float64)
    t = np.arange(x.shape[0]) if targets is None else np.asarray(targets)
    d = x[t][:, None, :] - x[None, :, :]  # r_i - r_j, (T, N, 3)
    L = np.asarray(box, dtype=np.float64)
    d[..., 0] -= L[0] * np.round(d[..., 0] / L[0])
    d[..., 1] -= L[1] * np.round(d[..., 1] / L[1])
    return t, d


def _exp_erfc(a, kz, E):
    """e^{kz} erfc(a) where a = k/(2 alpha) + alpha z and E = exp(-k^2/(4 alpha^2) - alpha^2 z^2).

    For a >= 0: erfc(a) e^{kz} = erfcx(a) e^{-a^2 + kz} = erfcx(a) E.
    For a <  0: erfc(a) = 2 - erfc(-a), so the product is 2 e^{kz} - erfcx(-a) E."""
    out = np.empty_like(a)
    pos = a >= 0
    out[pos] = erfcx(a[pos]) * E[pos]
    neg = ~pos
    out[neg] = 2.0 * np.exp(kz[neg]) - erfcx(-a[neg]) * E[neg]
    return out


def ewald2d(x, q, box, alpha=None, tol=1e-16, targets=None, forces=True):
    """Potentials Phi_i and gradients grad_i Phi_i (the gradient acts on r_i).

    x: (N,3) positions (any origin; only differences are used), q: (N,), box: (Lx,Ly,Lz).
    Returns dict(phi=(T,), grad=(T,3)) for the targets (all particles by default)."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    Lx, Ly, _ = (float(v) for v in box)
    A = Lx * Ly
    if abs(q.sum()) > 1e-10 * np.abs(q).sum():
        raise ValueError("Ewald2D needs a charge-neutral system")
    if alpha is None:
        alpha = 6.0 / min(Lx, Ly)
    t, d = _pair_geometry(x, box, targets)
    T = t.size
    phi = np.zeros(T)
    grad = np.zeros((T, 3))
    lt = math.log(1.0 / tol)

    # real space: images within the radius where erfc(alpha r) < tol
    rcut = math.sqrt(lt) / alpha + 1e-12
    nxm = int(math.ceil(rcut / Lx)) + 1
    nym = int(math.ceil(rcut / Ly)) + 1
    self_mask = (t[:, None] == np.arange(x.shape[0])[None, :])
    for nx in range(-nxm, nxm + 1):
        for ny in range(-nym, nym + 1):
            dd = d.copy()
            dd[..., 0] += nx * Lx
            dd[..., 1] += ny * Ly
            r = np.sqrt(np.sum(dd * dd, axis=-1))
            mask = r < rcut
            if nx == 0 and ny == 0:
                mask &= ~self_mask
            rr = np.where(mask, r, 1.0)
            val = np.where(mask, erfc(alpha * rr) / rr, 0.0)
            phi += val @ q
            if forces:
                # d/dr [erfc(alpha r)/r] = -erfc(alpha r)/r^2 - 2 alpha/sqrt(pi) e^{-alpha^2 r^2}/r
                dr = np.where(mask, -erfc(alpha * rr) / rr ** 2 - 2 * alpha / math.sqrt(math.pi) * np.exp(-(alpha * rr) ** 2) / rr, 0.0)
                coef = dr / rr * q[None, :]
                grad += np.einsum("tn,tnc->tc", coef, dd)

    # reciprocal space, k != 0: half plane (ky > 0, or ky == 0 and kx > 0), doubled
    kcut = 2.0 * alpha * math.sqrt(lt)
    mx = int(math.ceil(kcut * Lx / (2 * math.pi)))
    my = int(math.ceil(kcut * Ly / (2 * math.pi)))
    z = d[..., 2]
    for ny in range(0, my + 1):
        for nx in range(-mx, mx + 1):
            if ny == 0 and nx <= 0:
                continue
            kx, ky = 2 * math.pi * nx / Lx, 2 * math.pi * ny / Ly
            k = math.hypot(kx, ky)
            if k > kcut:
                continue
            E = np.exp(-k * k / (4 * alpha * alpha) - alpha * alpha * z * z)
            a = k / (2 * alpha) + alpha * z
            bm = k / (2 * alpha) - alpha * z
            f1 = _exp_erfc(a, k * z, E)
            f2 = _exp_erfc(bm, -k * z, E)
            ph = kx * d[..., 0] + ky * d[..., 1]
            c, s = np.cos(ph), np.sin(ph)
            pref = 2.0 * math.pi / A / k
            phi += pref * ((c * (f1 + f2)) @ q)
            if forces:
                grad[:, 0] += pref * ((-kx * s * (f1 + f2)) @ q)
                grad[:, 1] += pref * ((-ky * s * (f1 + f2)) @ q)
                # d/dz of the bracket = k (e^{kz} erfc(a) - e^{-kz} erfc(b)); the Gaussian parts cancel
                grad[:, 2] += pref * ((c * k * (f1 - f2)) @ q)

    # k = 0 term
    phi += -2.0 * math.pi / A * ((z * erf(alpha * z) + np.exp(-(alpha * z) ** 2) / (alpha * math.sqrt(math.pi))) @ q)
    if forces:
        grad[:, 2] += -2.0 * math.pi / A * (erf(alpha * z) @ q)
    # self term
    phi += -2.0 * alpha / math.sqrt(math.pi) * q[t]
    return dict(phi=phi, grad=grad)


def energy(q, phi):
    """U = 1/2 sum_i q_i Phi_i (eq. Errortol_P's left-hand side, and the usual definition)."""
    return 0.5 * float(np.dot(q, phi))


def brute_force_damped(x, q, box, R):
    """sum_j sum'_n q_j exp(-|n o L|^2/R^2) / |r_ij + n o L| over the xy images n, for
    tiny inputs.  The Gaussian damping of the image lattice makes the
    truncation error a smooth function of 1/R (no lattice-point counting
    noise), so ``brute_force_extrapolated`` can extrapolate it to R -> infinity.
    An independent pin of Ewald2D: plain image sums of 1/r, nothing else."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    Lx, Ly, _ = (float(v) for v in box)
    N = x.shape[0]
    nxm, nym = int(8 * R / Lx) + 1, int(8 * R / Ly) + 1
    nx, ny = np.meshgrid(np.arange(-nxm, nxm + 1), np.arange(-nym, nym + 1), indexing="ij")
    sh = np.stack([nx.ravel() * Lx, ny.ravel() * Ly, np.zeros(nx.size)], axis=1)
    damp = np.exp(-np.sum(sh * sh, axis=1) / (R * R))
    phi = np.zeros(N)
    for i in range(N):
        for j in range(N):
            dd = x[i] - x[j] + sh
            r = np.sqrt(np.sum(dd * dd, axis=1))
            keep = r > 0  # drops only the self term i == j, n == 0
            phi[i] += q[j] * np.sum(damp[keep] / r[keep])
    return phi


def brute_force_extrapolated(x, q, box, R0=None, npts=9, ratio=2 ** (1 / 3), degree=6):
    """Extrapolate ``brute_force_damped`` to R -> infinity by a least-squares
    polynomial in 1/R over R = R0 ratio^k, k = 0..npts-1."""
    if R0 is None:
        R0 = 10.0 * max(box[0], box[1])
    Rs = R0 * ratio ** np.arange(npts)
    P = np.array([brute_force_damped(x, q, box, R) for R in Rs])
    V = np.vander(1.0 / Rs, degree + 1)
    coef = np.linalg.lstsq(V, P, rcond=None)[0]
    return coef[-1]
