"""The oracle's own parameter choice (Sec. 4.3), for runs that ask for a tolerance
instead of explicit parameters.

Test infrastructure only (see ``oracle/__init__``).  Simple rules written from the
paper's error estimates, one error budget eps = tol/20 per term:
* decomposition: the first Table 1 row with energy and force errors <= tol/2;
  r_c = 3 rho^{-1/3} (Sec. 4.3: r_c ~ rho^{-1/3}), at most min(Lx, Ly)/2;
  M so that the omitted wide Gaussians' z^2 term stays below 1e-2 eps.
* range split: eta = 1/2, m = max{l : s_l <= eta Lz} (Sec. 3.1).
* mid range: K_max from exp(-s_0^2 K^2/4) (Thm thm::trunFour with the Gaussian's
  transform exp(-s^2 k^2/4), Sec. 2.2), h = pi/K_max; the smallest odd P_w whose
  window error max(exp(-S), exp(-pi^2 mu (P_w-1)^2/(4 s_0^2 S))) (Thm thm::scal) is
  below eps for the best S; padding so that the widest mid-range Gaussian decays
  over the extension (Thm thm::pad).
* long range, direct form: P from Thm thm::Che (with the constants its proof drops),
  |k| <= 2 sqrt(log(1/eps))/s_{m+1} (Thm thm::Fcheb).
"""
import math

import numpy as np

from .sog import SOG, table_row_for_tol


def _smooth(n, even):
    while True:
        m = n
        for p in (2, 3, 5, 7):
            while m % p == 0:
                m //= p
        if m == 1 and (not even or n % 2 == 0):
            return n
        n += 1


def _window_error(Pw, h, s):
    """min over S of max(exp(-S), aliasing term), by a scan over S."""
    u = Pw - 1
    H = u * h / 2
    best = (1.0, None)
    for S in np.linspace(1.0, 60.0, 1200):
        mu = s * s - H * H / S
        if mu <= 0:
            continue
        e = max(math.exp(-S), math.exp(-math.pi ** 2 * mu * u * u / (4 * s * s * S)))
        if e < best[0]:
            best = (e, float(S))
    return best


def plan(box, N, tol, eta=0.5, rc=None):
    """Parameters (a dict for fast.solve) for N particles in box at relative tolerance tol;
    eta sets the range split, rc (default 3 rho^{-1/3}) the near-field cutoff."""
    Lx, Ly, Lz = (float(v) for v in box)
    eps = tol / 20.0
    b, r0, om = table_row_for_tol(tol)[:3]
    rho = N / (Lx * Ly * Lz)
    rc = min(3.0 * rho ** (-1.0 / 3.0) if rc is None else float(rc), 0.5 * min(Lx, Ly))
    sigma = rc / r0
    wl1 = math.sqrt(2 / math.pi) * math.log(b) / sigma
    rhs = 1e-2 * eps * Lx * Ly / (math.pi * N * Lz * Lz) * (1 - 1 / b) / wl1
    M = max(int(math.ceil(-math.log(rhs) / math.log(b))), table_row_for_tol(tol)[4])
    sog = SOG(b, r0, om, rc, M)
    m = sog.split_index(eta, Lz)
    mid = None
    if m >= 0:
        s0 = sog.s[0]
        # the window's aliasing exponent can not exceed the grid's own (pi s_0 / 2h)^2, so
        # resolve the narrowest Gaussian two e-folds beyond eps
        K = 2 * math.sqrt(math.log(1.0 / eps) + 2.0) / s0
        h = math.pi / K
        I = [_smooth(int(math.ceil(L / h)), True) for L in (Lx, Ly)]
        Iz = int(math.ceil(Lz / h))
        hmax = max(Lx / I[0], Ly / I[1], Lz / Iz)
        Pw, S = None, None
        for p in range(5, 33, 2):
            e, Sp = _window_error(p, hmax, s0)
            if e <= eps:
                Pw, S = p, Sp
                break
        if Pw is None:
            raise ValueError("no window meets the tolerance")
        I = [max(v, 2 * Pw) for v in I]
        hz = Lz / Iz
        delta = sog.s[m] * math.sqrt(math.log(1 / eps) / 2)
        Lzs = Lz + (Pw - 1) * hz + delta
        Izs = 2 * _smooth(int(math.ceil(Lzs / hz / 2)), False)
        Izs = max(Izs, Iz + Pw + 2 + (Iz + Pw) % 2)
        mid = dict(I=(I[0], I[1], Iz), Izs=Izs, Pw=(Pw, Pw, Pw), S=S)
    long = None
    if m < M:
        sl = sog.s[m + 1]
        e = sl / Lz
        P = 2
        while 4 * 1.0865 / (math.sqrt(math.factorial(P)) * (2 * math.sqrt(2) * e) ** P) > eps and P < 64:
            P += 1
        K = 2 * math.sqrt(math.log(1 / eps)) / sl
        nk = (int(K * Lx / (2 * math.pi)), int(K * Ly / (2 * math.pi)))
        long = dict(form="direct", P=P, nk=nk)
    return dict(sog=dict(b=b, r0=r0, omega=om, rc=rc, M=M), m=m, mid=mid, long=long)
