"""The plain fast spectral SOG method, FP64 NumPy, every step in the paper's order.

Test infrastructure only (see ``oracle/__init__``).

Parameters are explicit (a dict, see ``make_params``); nothing here picks a
grid or a degree.  Coordinates: the box is Omega = [-Lx/2,Lx/2] x [-Ly/2,Ly/2] x
[-Lz/2,Lz/2] (Sec. 2.1); inputs in [0,Lx) x [0,Ly) x [0,Lz] are wrapped in x,y and
shifted by -L/2.

Mid range (Alg. al::mid, eqs. gridding, widehat-tilde, Phiconv; constants
derived from eq. PhiNDF with the k_z integral discretised on the padded
period L_z*, Sec. 3.4):
  grid nodes X_a = -Lx/2 + a h_x (a < I_x), likewise y, and Z_c = -L_z*/2 + c h_z
  (c < I_z*), h_z = Lz/I_z, L_z* = I_z* h_z;
  Gaussian window W(x) = exp(-S (x/H)^2) 1_{|x|<=H}, H = (P_w-1) h/2, with
  transform What(k) = sqrt(pi/S) H exp(-k^2 H^2/(4S)) (eq. GS);
  Ghat_mid(k) = 4 pi tauhat_mid(k)/k^2 = pi^{3/2} sum_{l<=m} w_l s_l^3 exp(-s_l^2 k^2/4);
  1. S(g) = sum_j q_j W(g - r_j)  (x,y periodic)
  2. Shat = fftn(S)
  3. multiply by Ghat_mid(k) / What(k)^2   (k = 2 pi fftfreq)
  4. u = ifftn(.)
  5. Phi_mid_i = h_x h_y h_z sum_g W(r_i - g) u(g), grad with dW.
  Optionally the ES window (window_1d_es) with its transform by quadrature, or the
  Kaiser-Bessel window (window_1d_kb, closed-form transform), exact or replaced by its
  degree-nu Chebyshev interpolants per node (window_poly_1d, Remark rmk::PWindow).

Long range, direct form (App. B, Alg. al::long_nonfft), with Chebyshev
interpolation in the target z and anterpolation in the source z (the
"interpolation/anterpolation" of the abstract; App. A.2 for nodes and V^-1):
  Chebyshev nodes t_c = cos((c+1/2) pi/P), z_c = (Lz/2) t_c (eq. Chebyshevnode);
  Lagrange basis L_c(t) = (1/P)[1 + 2 sum_{n=1}^{P-1} T_n(t_c) T_n(t)], the
  closed form of V^-1 (eq. ChebyshevInt, no primed sum);
  kernel on the nodes, from eq. trun2:
    K(k;c,c') = pi sum_{l>m} w_l s_l^2 exp(-s_l^2 |k|^2/4) exp(-(z_c-z_c')^2/s_l^2)
  (for k = 0 the constant pi sum w_l s_l^2 is dropped: it multiplies
  sum_c' rho(0,c') = sum_j q_j = 0; expm1 keeps the rest accurate);
  1. rho(k,c') = sum_j q_j exp(-i k.r_j) L_c'(z_j)   (gridding + interpolation)
  2. v(k,c) = sum_c' K(k;c,c') rho(k,c')             (scaling)
  3. Phi_long_i = (1/A) Re sum_k exp(i k.r_i) sum_c L_c(z_i) v(k,c)   (gathering)
  with k over |n_x| <= nk_x, |n_y| <= nk_y.

Long range, FFT form (Alg. al::long): the same three steps with the x,y
Fourier sums replaced by a 2D Gaussian-window spread on an I^long grid, 2D
FFTs and a window gather, exactly as the mid range does in 3D:
  S2(g,c') = sum_j q_j W2(g - r_j) L_c'(z_j); u(.,c) = ifft2(sum_c' K/What2^2 fft2 S2(.,c'));
  Phi_long_i = h_x h_y sum_g W2(r_i - g) sum_c L_c(z_i) u(g,c).

Near field (eq. phiNDR): all pairs within r_c over xy images (no z images),
N(r) = 1/r - F(r) with the full sum of M+1 Gaussians.

Totals: Phi = Phi_N + Phi_mid + Phi_long - q_i sum_l w_l;  U = 1/2 sum q_i Phi_i;
F_i = -q_i grad Phi_i.
"""
import math
import time

import numpy as np
from scipy.spatial import cKDTree

from .sog import SOG


# ----------------------------------------------------------------------------- parameters

def make_params(b, r0, omega, rc, M, m, mid=None, long=None):
    """Explicit parameter set.

    mid: dict(I=(Ix,Iy,Iz), Izs=I_z*, Pw=(px,py,pz), S=shape) or None (m < 0); with
         window='es' and beta=beta the ES window replaces the Gaussian (S unused).
    long: dict(form='direct', P=P, nk=(nkx,nky)) or
          dict(form='fft', P=P, I=(Ix,Iy), Pw=(px,py), S=shape) or None (m == M); with
          Q=Q > 0 the FFT form takes the Taylor acceleration of App. C."""
    return dict(sog=dict(b=b, r0=r0, omega=omega, rc=rc, M=M), m=m, mid=mid, long=long)


def centered(x, box):
    """Wrap x,y into [0,L) and shift every coordinate by -L/2 (Sec. 2.1 box Omega)."""
    x = np.array(x, dtype=np.float64, copy=True)
    for d in (0, 1):
        x[:, d] = np.mod(x[:, d], box[d])
        x[:, d] = np.where(x[:, d] >= box[d], x[:, d] - box[d], x[:, d])
    return x - 0.5 * np.asarray(box, dtype=np.float64)


# ----------------------------------------------------------------------------- windows

def window_1d(xc, origin, h, n, Pw, S, periodic):
    """Gaussian-window weights of every particle on its Pw nearest grid points (eq. GS).

    Returns (idx (N,Pw) grid indices, W (N,Pw) weights, dW (N,Pw) d/dx_particle of W(x_p - x_g))."""
    H = 0.5 * (Pw - 1) * h
    a0 = np.round((xc - origin) / h).astype(np.int64)
    off = np.arange(Pw) - (Pw - 1) // 2
    idx = a0[:, None] + off[None, :]
    dx = xc[:, None] - (origin + idx * h)  # x_p - x_g
    W = np.where(np.abs(dx) <= H, np.exp(-S * (dx / H) ** 2), 0.0)
    dW = -2.0 * S * dx / (H * H) * W
    if periodic:
        idx = np.mod(idx, n)
    else:
        if np.any(idx < 0) or np.any(idx >= n):
            raise ValueError("window support leaves the padded z grid")
    return idx, W, dW


def window_hat(k, h, Pw, S):
    """Fourier transform of the (untruncated) Gaussian window, eq. GS."""
    H = 0.5 * (Pw - 1) * h
    return math.sqrt(math.pi / S) * H * np.exp(-(k * k) * H * H / (4.0 * S))


# The "exponential of semicircle" window, one of the compactly supported windows of the
# Kaiser-Bessel family that Sec. 5's experiments use in place of the Gaussian (the paper
# prints no formula for them; this is the reading of the library's window option):
#   W(x) = exp(beta (sqrt(1 - (x/a)^2) - 1)) for |x| < a,  0 otherwise,  a = P_w h / 2,
# so the P_w nodes nearest a particle are exactly the nodes inside the support.  Its
# transform has no closed form and is computed by quadrature.

def window_1d_es(xc, origin, h, n, Pw, beta, periodic):
    """ES-window weights of every particle on its Pw nearest grid points; same returns as
    window_1d (d/dx_particle of W(x_p - x_g) in dW)."""
    a = 0.5 * Pw * h
    a0 = np.round((xc - origin) / h).astype(np.int64)
    off = np.arange(Pw) - (Pw - 1) // 2
    idx = a0[:, None] + off[None, :]
    dx = xc[:, None] - (origin + idx * h)  # x_p - x_g
    t2 = (dx / a) ** 2
    inside = t2 < 1.0
    root = np.sqrt(np.where(inside, 1.0 - t2, 1.0))
    W = np.where(inside, np.exp(beta * (root - 1.0)), 0.0)
    dW = np.where(inside, -beta * dx / (a * a * root) * W, 0.0)
    if periodic:
        idx = np.mod(idx, n)
    else:
        if np.any(idx < 0) or np.any(idx >= n):
            raise ValueError("window support leaves the padded z grid")
    return idx, W, dW


def window_hat_es(k, h, Pw, beta):
    """Fourier transform of the ES window, What(k) = int W(x) exp(-i k x) dx.  With
    x = a sin(theta) the integrand exp(beta (cos theta - 1)) cos(k a sin theta) a cos theta
    is smooth on [0, pi/2]; Gauss-Legendre with enough nodes for the oscillation."""
    a = 0.5 * Pw * h
    k = np.asarray(k, dtype=np.float64)
    kmax = float(np.max(np.abs(k))) if k.size else 0.0
    nq = 64 + int(math.ceil(2.0 * kmax * a))
    t, w = np.polynomial.legendre.leggauss(nq)
    th = 0.25 * math.pi * (t + 1.0)
    wt = 0.25 * math.pi * w
    f = np.exp(beta * (np.cos(th) - 1.0)) * a * np.cos(th) * wt
    kf = k.reshape(-1)
    out = 2.0 * (np.cos(np.outer(kf * a, np.sin(th))) @ f)
    return out.reshape(k.shape)


# The Kaiser-Bessel window, the window of the paper's experiments (Sec. 5, Remark
# rmk::PWindow; the paper prints no formula):
#   W(x) = I_0(beta sqrt(1 - (x/a)^2)) / I_0(beta) for |x| <= a,  0 otherwise,  a = P_w h / 2,
# with the closed-form transform of the truncated window (the standard Kaiser-Bessel pair)
#   What(k) = (2 a / I_0(beta)) sinh(sqrt(beta^2 - (k a)^2)) / sqrt(beta^2 - (k a)^2),
# continued by sin(sqrt((k a)^2 - beta^2)) / sqrt((k a)^2 - beta^2) for |k a| > beta.

def window_1d_kb(xc, origin, h, n, Pw, beta, periodic, nu=None):
    """KB-window weights of every particle on its Pw nearest grid points; same returns as
    window_1d (d/dx_particle of W(x_p - x_g) in dW: W' = I_1(beta r) beta (-x/a^2)/r / I_0(beta),
    r = sqrt(1 - (x/a)^2)).  With nu, the weights are those of the window's polynomial
    approximation of degree nu (window_poly_1d)."""
    from scipy.special import i0, i1
    a = 0.5 * Pw * h
    a0 = np.round((xc - origin) / h).astype(np.int64)
    off = np.arange(Pw) - (Pw - 1) // 2
    idx = a0[:, None] + off[None, :]
    if nu is not None:
        W, dW = window_poly_1d(lambda d: kb_value_mp(d, a, beta), (xc - origin) / h - a0, h, Pw, nu)
        return _wrap_idx(idx, n, periodic), W, dW
    dx = xc[:, None] - (origin + idx * h)  # x_p - x_g
    t2 = (dx / a) ** 2
    inside = t2 <= 1.0
    r = np.sqrt(np.where(inside, 1.0 - t2, 1.0))
    norm = 1.0 / i0(beta)
    W = np.where(inside, i0(beta * r) * norm, 0.0)
    # I_1(beta r)/r -> beta/2 as r -> 0 (the support edge)
    ratio = np.where(r > 1e-8, i1(beta * r) / np.where(r > 1e-8, r, 1.0), 0.5 * beta)
    dW = np.where(inside, -beta * dx / (a * a) * ratio * norm, 0.0)
    if periodic:
        idx = np.mod(idx, n)
    else:
        if np.any(idx < 0) or np.any(idx >= n):
            raise ValueError("window support leaves the padded z grid")
    return idx, W, dW


def kb_value(x, a, beta):
    """The KB window at x (array), zero outside [-a, a]."""
    from scipy.special import i0
    t2 = (np.asarray(x, dtype=np.float64) / a) ** 2
    return np.where(t2 <= 1.0, i0(beta * np.sqrt(np.where(t2 <= 1.0, 1.0 - t2, 0.0))) / i0(beta), 0.0)


def kb_value_mp(x, a, beta):
    """The KB window at one distance x, in mpmath's working precision."""
    import mpmath as mp
    t = mp.mpf(x) / a
    if abs(t) > 1:
        return mp.mpf(0)
    return mp.besseli(0, beta * mp.sqrt(1 - t * t)) / mp.besseli(0, beta)


def window_poly_1d(wexact, u, h, Pw, nu):
    """Remark rmk::PWindow: a window replaced by polynomials of degree nu built by
    Chebyshev interpolation.  A particle at offset u in [-1/2, 1/2] (grid units) from its
    nearest node puts weight W(h (node - particle)) on node o = -(Pw-1)/2 .. (Pw-1)/2;
    for each o this weight is a smooth function of u on [-1/2, 1/2] (the window's support
    ends at u = +-1/2 for the outermost nodes), interpolated at the nu + 1 Chebyshev
    points of that interval.  wexact(x) evaluates the window at one distance x in mpmath
    precision: the interpolant's derivative magnifies errors of its samples up to 2 nu^2
    times at the interval's ends, so the samples and the Chebyshev coefficients are
    formed at 30 digits and only the coefficients are rounded to float64.  Returns
    (W, dW) of shape (N, Pw); dW = d W / d x_particle = -(1/h) d/d(node - particle)."""
    import mpmath as mp
    from numpy.polynomial import chebyshev as C
    off = np.arange(Pw) - (Pw - 1) // 2
    u = np.asarray(u, dtype=np.float64)
    W = np.empty((u.size, Pw))
    dW = np.empty((u.size, Pw))
    n1 = nu + 1
    with mp.workdps(30):
        th = [(j + mp.mpf(1) / 2) * mp.pi / n1 for j in range(n1)]
        for col, o in enumerate(off):
            # weight on node o as a function of t = 2u in [-1, 1], sampled at t_j = cos(th_j)
            f = [wexact(mp.mpf(h) * (o - mp.cos(t) / 2)) for t in th]
            c = [2 * mp.fsum(f[j] * mp.cos(k * th[j]) for j in range(n1)) / n1 for k in range(n1)]
            c[0] /= 2
            # derivative series: c'_{k-1} = c'_{k+1} + 2 k c_k (the usual recurrence)
            cd = [mp.mpf(0)] * (n1 + 1)
            for k in range(nu, 0, -1):
                cd[k - 1] = cd[k + 1] + 2 * k * c[k]
            cd[0] /= 2
            c64 = np.array([float(v) for v in c])
            cd64 = np.array([float(v) for v in cd[:nu]]) if nu > 0 else np.zeros(1)
            W[:, col] = C.chebval(2.0 * u, c64)
            # d/dx_p = (1/h) d/du = (2/h) d/dt
            dW[:, col] = (2.0 / h) * C.chebval(2.0 * u, cd64)
    return W, dW


def _wrap_idx(idx, n, periodic):
    if periodic:
        return np.mod(idx, n)
    if np.any(idx < 0) or np.any(idx >= n):
        raise ValueError("window support leaves the padded z grid")
    return idx


def window_hat_kb(k, h, Pw, beta):
    """Closed-form Fourier transform of the KB window (see above)."""
    from scipy.special import i0
    a = 0.5 * Pw * h
    k = np.asarray(k, dtype=np.float64)
    z2 = beta * beta - (k * a) ** 2
    out = np.empty_like(k)
    pos, neg = z2 > 1e-12, z2 < -1e-12
    zp = np.sqrt(z2[pos])
    out[pos] = np.sinh(zp) / zp
    zn = np.sqrt(-z2[neg])
    out[neg] = np.sin(zn) / zn
    out[~(pos | neg)] = 1.0
    return 2.0 * a * out / i0(beta)


# ----------------------------------------------------------------------------- mid range

def mid_range(xc, q, box, sog: SOG, m, mid):
    """Alg. al::mid; returns (phi (N,), grad (N,3))."""
    Lx, Ly, Lz = box
    Ix, Iy, Iz = mid["I"]
    Izs = mid["Izs"]
    px, py, pz = mid["Pw"]
    kind = mid.get("window", "gaussian")
    S = mid["beta"] if kind in ("es", "kb") else mid["S"]
    wfun, hfun = {"es": (window_1d_es, window_hat_es), "kb": (window_1d_kb, window_hat_kb)}.get(
        kind, (window_1d, window_hat))
    if kind == "kb" and mid.get("nu"):
        # the KB window by its degree-nu polynomials (Remark rmk::PWindow); the multiplier
        # keeps the exact window's transform
        nu = mid["nu"]
        wfun = lambda xc_, o_, h_, n_, p_, s_, per_: window_1d_kb(xc_, o_, h_, n_, p_, s_, per_, nu=nu)
    hx, hy, hz = Lx / Ix, Ly / Iy, Lz / Iz
    Lzs = Izs * hz
    ix, Wx, dWx = wfun(xc[:, 0], -Lx / 2, hx, Ix, px, S, True)
    iy, Wy, dWy = wfun(xc[:, 1], -Ly / 2, hy, Iy, py, S, True)
    iz, Wz, dWz = wfun(xc[:, 2], -Lzs / 2, hz, Izs, pz, S, False)
    N = xc.shape[0]
    # 1. gridding: S(g) = sum_j q_j W(g - r_j), added node by node (one scatter-add per
    #    (x, y) window node, over all particles and their P_w z nodes)
    grid = np.zeros(Ix * Iy * Izs)
    for a in range(px):
        for b in range(py):
            lin_xy = (ix[:, a] * Iy + iy[:, b]) * Izs
            wxy = q * Wx[:, a] * Wy[:, b]
            np.add.at(grid, (lin_xy[:, None] + iz).ravel(), (wxy[:, None] * Wz).ravel())
    grid = grid.reshape(Ix, Iy, Izs)
    # 2.-4. FFT, scaling, inverse FFT.  S is real and the multiplier is real and even in
    #    k, so the product's spectrum is Hermitian and the half spectrum (rfftn / irfftn)
    #    holds all of it: u = ifftn(G/What^2 fftn(S)), which is real.
    kx = 2 * np.pi * np.fft.fftfreq(Ix, d=hx)
    ky = 2 * np.pi * np.fft.fftfreq(Iy, d=hy)
    kz = 2 * np.pi * np.fft.rfftfreq(Izs, d=hz)
    G = np.zeros((Ix, Iy, kz.size))
    for ell in range(m + 1):
        # exp(-s^2 |k|^2 / 4) as the product of its three directional factors
        s2 = sog.s[ell] ** 2
        ex, ey, ez = (np.exp(-s2 * k * k / 4.0) for k in (kx, ky, kz))
        G += math.pi ** 1.5 * sog.w[ell] * sog.s[ell] ** 3 * (ex[:, None, None] * ey[None, :, None] * ez[None, None, :])
    What2 = (hfun(kx, hx, px, S)[:, None, None] ** 2 * hfun(ky, hy, py, S)[None, :, None] ** 2
             * hfun(kz, hz, pz, S)[None, None, :] ** 2)
    G /= What2
    del What2
    u = np.fft.irfftn(G * np.fft.rfftn(grid), s=(Ix, Iy, Izs), axes=(0, 1, 2)).ravel()
    del G, grid
    # 5. gathering
    phi = np.zeros(N)
    grad = np.zeros((N, 3))
    for a in range(px):
        for b in range(py):
            lin_xy = (ix[:, a] * Iy + iy[:, b]) * Izs
            uu = u[lin_xy[:, None] + iz]  # (N, P_w): u on the particle's z nodes
            acc0 = np.sum(Wz * uu, axis=1)
            acc1 = np.sum(dWz * uu, axis=1)
            phi += Wx[:, a] * Wy[:, b] * acc0
            grad[:, 0] += dWx[:, a] * Wy[:, b] * acc0
            grad[:, 1] += Wx[:, a] * dWy[:, b] * acc0
            grad[:, 2] += Wx[:, a] * Wy[:, b] * acc1
    V = hx * hy * hz
    return V * phi, V * grad


# ----------------------------------------------------------------------------- Chebyshev

def cheb_nodes(P):
    """First-kind Chebyshev nodes t_c = cos((c + 1/2) pi / P), c = 0..P-1 (eq. Chebyshevnode)."""
    return np.cos((np.arange(P) + 0.5) * np.pi / P)


def lagrange(t, P):
    """L_c(t) and dL_c/dt for the first-kind nodes, from
    L_c(t) = (1/P)[1 + 2 sum_{n=1}^{P-1} T_n(t_c) T_n(t)] (the closed form of V^-1,
    eq. ChebyshevInt).  T_n by the three-term recurrence of App. A.1 and
    T_n' = n U_{n-1}."""
    t = np.asarray(t, dtype=np.float64)
    tc = cheb_nodes(P)
    Tc = np.ones((P, P))  # Tc[n, c] = T_n(t_c)
    if P > 1:
        Tc[1] = tc
    for n in range(2, P):
        Tc[n] = 2 * tc * Tc[n - 1] - Tc[n - 2]
    T = np.ones((P, t.size))
    dT = np.zeros((P, t.size))
    U = np.ones((P, t.size))  # U_n
    if P > 1:
        T[1] = t
        U[1] = 2 * t
    for n in range(2, P):
        T[n] = 2 * t * T[n - 1] - T[n - 2]
        U[n] = 2 * t * U[n - 1] - U[n - 2]
    for n in range(1, P):
        dT[n] = n * U[n - 1]
    coef = np.ones(P)
    coef[1:] = 2.0
    L = (coef[:, None] * Tc).T @ T / P  # (P_c, N)
    dL = (coef[:, None] * Tc).T @ dT / P
    return L.T, dL.T  # (N, P)


def long_kernel(kvec2, sog: SOG, m, zc):
    """K(k;c,c') on the Chebyshev nodes for a list of |k|^2 values (from eq. trun2).
    Returns (nk, P, P)."""
    dz2 = (zc[:, None] - zc[None, :]) ** 2
    K = np.zeros((kvec2.size, zc.size, zc.size))
    for ell in range(m + 1, sog.M + 1):
        s2 = sog.s[ell] ** 2
        ek = np.exp(-s2 * kvec2 / 4.0)
        zero = kvec2 == 0.0
        ez = np.exp(-dz2 / s2)
        ezm1 = np.expm1(-dz2 / s2)
        coef = math.pi * sog.w[ell] * s2
        K += coef * np.where(zero[:, None, None], ezm1[None], ek[:, None, None] * ez[None])
    return K


def long_range_direct(xc, q, box, sog: SOG, m, lp):
    """Direct (non-FFT) Fourier-Chebyshev long range; returns (phi, grad)."""
    Lx, Ly, Lz = box
    A = Lx * Ly
    P = lp["P"]
    nkx, nky = lp["nk"]
    nx, ny = np.meshgrid(np.arange(-nkx, nkx + 1), np.arange(-nky, nky + 1), indexing="ij")
    kx = (2 * np.pi / Lx * nx).ravel()
    ky = (2 * np.pi / Ly * ny).ravel()
    zc = 0.5 * Lz * cheb_nodes(P)
    Kmat = long_kernel(kx * kx + ky * ky, sog, m, zc)  # (nk, P, P)
    L, dL = lagrange(2.0 * xc[:, 2] / Lz, P)  # (N, P)
    ph = np.exp(-1j * (np.outer(xc[:, 0], kx) + np.outer(xc[:, 1], ky)))  # (N, nk)
    rho = (ph * q[:, None]).T @ L  # (nk, P)
    v = np.einsum("kab,kb->ka", Kmat, rho)  # (nk, P)
    Uk = L @ v.T  # (N, nk): sum_c L_c(z_i) v(k,c)
    dUk = dL @ v.T
    e = np.conj(ph)  # exp(+i k.r_i)
    phi = np.real(np.sum(e * Uk, axis=1)) / A
    grad = np.zeros((xc.shape[0], 3))
    grad[:, 0] = np.real(np.sum(1j * kx[None, :] * e * Uk, axis=1)) / A
    grad[:, 1] = np.real(np.sum(1j * ky[None, :] * e * Uk, axis=1)) / A
    grad[:, 2] = np.real(np.sum(e * dUk, axis=1)) / A * (2.0 / Lz)
    return phi, grad


def long_range_fft(xc, q, box, sog: SOG, m, lp):
    """FFT form of the Fourier-Chebyshev long range (Alg. al::long); returns (phi, grad)."""
    Lx, Ly, Lz = box
    P = lp["P"]
    Ix, Iy = lp["I"]
    px, py = lp["Pw"]
    S = lp["S"]
    hx, hy = Lx / Ix, Ly / Iy
    N = xc.shape[0]
    ix, Wx, dWx = window_1d(xc[:, 0], -Lx / 2, hx, Ix, px, S, True)
    iy, Wy, dWy = window_1d(xc[:, 1], -Ly / 2, hy, Iy, py, S, True)
    L, dL = lagrange(2.0 * xc[:, 2] / Lz, P)
    # 1. gridding on proxy points R^2 x C
    grid = np.zeros((P, Ix * Iy))
    for a in range(px):
        for b in range(py):
            lin = ix[:, a] * Iy + iy[:, b]
            wxy = q * Wx[:, a] * Wy[:, b]
            for c in range(P):
                grid[c] += np.bincount(lin, weights=wxy * L[:, c], minlength=Ix * Iy)
    grid = grid.reshape(P, Ix, Iy)
    # 2.-4. 2D FFTs, scaling with the z kernel, inverse 2D FFTs
    kx = 2 * np.pi * np.fft.fftfreq(Ix, d=hx)
    ky = 2 * np.pi * np.fft.fftfreq(Iy, d=hy)
    k2 = (kx[:, None] ** 2 + ky[None, :] ** 2).ravel()
    zc = 0.5 * Lz * cheb_nodes(P)
    Kmat = long_kernel(k2, sog, m, zc)  # (Ix*Iy, P, P)
    What2 = (window_hat(kx, hx, px, S)[:, None] ** 2 * window_hat(ky, hy, py, S)[None, :] ** 2).ravel()
    Ghat = np.fft.fft2(grid, axes=(1, 2)).reshape(P, -1)  # (P, nk)
    uhat = np.einsum("kab,bk->ak", Kmat, Ghat) / What2[None, :]
    u = np.real(np.fft.ifft2(uhat.reshape(P, Ix, Iy), axes=(1, 2))).reshape(P, -1)
    # 5. gathering
    phi = np.zeros(N)
    grad = np.zeros((N, 3))
    for a in range(px):
        for b in range(py):
            lin = ix[:, a] * Iy + iy[:, b]
            uu = u[:, lin].T  # (N, P)
            acc0 = np.sum(L * uu, axis=1)
            acc1 = np.sum(dL * uu, axis=1)
            phi += Wx[:, a] * Wy[:, b] * acc0
            grad[:, 0] += dWx[:, a] * Wy[:, b] * acc0
            grad[:, 1] += Wx[:, a] * dWy[:, b] * acc0
            grad[:, 2] += Wx[:, a] * Wy[:, b] * acc1 * (2.0 / Lz)
    return hx * hy * phi, hx * hy * grad


# ----------------------------------------------------------------------------- App. C Taylor form

def taylor_gaussian(z, s, Q):
    """The Q-term Taylor polynomial of exp(-z^2/s^2) in -z^2/s^2 (Lemma lemma::Taylor):
    sum_{p<Q} (1/p!) (-z^2/s^2)^p."""
    x = -(np.asarray(z, dtype=np.float64) / s) ** 2
    out = np.zeros_like(x)
    term = np.ones_like(x)
    for p in range(Q):
        out += term
        term = term * x / (p + 1)
    return out


def taylor_coefficients(k2, sog: SOG, m, Lz, Q):
    """A_p(k) without the window factor: ((-1)^p/p!) sum_{l>m} w_l Lz^{2p} s_l^{2-2p}
    exp(-s_l^2 |k|^2/4), p < Q (App. C, with |k|^2 in the exponent).  Returns (nk, Q).
    At k = 0 the p = 0 term, the constant sum_l w_l s_l^2, is left out: it multiplies
    sum_j q_j = 0 (the same reading as the exact kernel's expm1)."""
    A = np.zeros((k2.size, Q))
    for ell in range(m + 1, sog.M + 1):
        s2 = sog.s[ell] ** 2
        ek = np.exp(-s2 * k2 / 4.0)
        for p in range(Q):
            A[:, p] += ((-1) ** p / math.factorial(p)) * sog.w[ell] * Lz ** (2 * p) * s2 ** (1 - p) * ek
    A[k2 == 0.0, 0] = 0.0
    return A


def long_range_fft_taylor(xc, q, box, sog: SOG, m, lp):
    """FFT form of the long range with the Taylor acceleration of App. C, in the paper's
    order (the steps replace steps 1-3 of Alg. al::long):
      1. S^p(g, c) = sum_j q_j W2(g - r_j) ((z_c - z_j)/Lz)^{2p}, p < Q, on the x,y grid
         times the Chebyshev nodes z_c;
      2. 2D FFT of every (p, c);
      3. Chebyshev interpolation in c: Stilde^p(k, n) = sum_c (2 - delta_n0)/P T_n(t_c) Shat^p(k, c);
      4. Shat_scal(k, n) = sum_p A_p(k) / What2(k)^2 Stilde^p(k, n);
      5. inverse 2D FFTs;
      6. Phi_long_i = pi h_x h_y sum_g W2(r_i - g) sum_n T_n(2 z_i/Lz) u(g, n)
         (pi: the prefactor of eq. trun2; the gradient in z from T_n').
    Returns (phi, grad)."""
    Lx, Ly, Lz = box
    P, Q = lp["P"], lp["Q"]
    Ix, Iy = lp["I"]
    px, py = lp["Pw"]
    S = lp["S"]
    hx, hy = Lx / Ix, Ly / Iy
    N = xc.shape[0]
    ix, Wx, dWx = window_1d(xc[:, 0], -Lx / 2, hx, Ix, px, S, True)
    iy, Wy, dWy = window_1d(xc[:, 1], -Ly / 2, hy, Iy, py, S, True)
    zc = 0.5 * Lz * cheb_nodes(P)
    # 1. gridding of the Taylor moments on R^2 x C
    mom = ((zc[None, :] - xc[:, 2][:, None]) / Lz) ** 2  # (N, P)
    grid = np.zeros((Q, P, Ix * Iy))
    for a in range(px):
        for b in range(py):
            lin = ix[:, a] * Iy + iy[:, b]
            wxy = q * Wx[:, a] * Wy[:, b]
            powp = np.ones_like(mom)
            for p in range(Q):
                for c in range(P):
                    grid[p, c] += np.bincount(lin, weights=wxy * powp[:, c], minlength=Ix * Iy)
                powp = powp * mom
    # 2. 2D FFTs
    Ghat = np.fft.fft2(grid.reshape(Q, P, Ix, Iy), axes=(2, 3)).reshape(Q, P, -1)
    # 3. Chebyshev interpolation: values at the nodes -> coefficients of T_n
    tc = cheb_nodes(P)
    Tc = np.ones((P, P))  # Tc[n, c] = T_n(t_c)
    if P > 1:
        Tc[1] = tc
    for n in range(2, P):
        Tc[n] = 2 * tc * Tc[n - 1] - Tc[n - 2]
    coef = np.full(P, 2.0 / P)
    coef[0] = 1.0 / P
    Stil = np.einsum("nc,pck->pnk", coef[:, None] * Tc, Ghat)  # (Q, P_n, nk)
    # 4. combination with A_p(k) / What2(k)^2
    kx = 2 * np.pi * np.fft.fftfreq(Ix, d=hx)
    ky = 2 * np.pi * np.fft.fftfreq(Iy, d=hy)
    k2 = (kx[:, None] ** 2 + ky[None, :] ** 2).ravel()
    A = taylor_coefficients(k2, sog, m, Lz, Q)  # (nk, Q)
    What2 = (window_hat(kx, hx, px, S)[:, None] ** 2 * window_hat(ky, hy, py, S)[None, :] ** 2).ravel()
    Sscal = np.einsum("kp,pnk->nk", A / What2[:, None], Stil)
    # 5. inverse 2D FFTs
    u = np.real(np.fft.ifft2(Sscal.reshape(P, Ix, Iy), axes=(1, 2))).reshape(P, -1)
    # 6. gathering with T_n(2 z_i / Lz)
    t = 2.0 * xc[:, 2] / Lz
    T = np.ones((N, P))
    dT = np.zeros((N, P))
    U = np.ones((N, P))  # U_n, for T_n' = n U_{n-1}
    if P > 1:
        T[:, 1] = t
        U[:, 1] = 2 * t
        dT[:, 1] = 1.0
    for n in range(2, P):
        T[:, n] = 2 * t * T[:, n - 1] - T[:, n - 2]
        U[:, n] = 2 * t * U[:, n - 1] - U[:, n - 2]
        dT[:, n] = n * U[:, n - 1]
    phi = np.zeros(N)
    grad = np.zeros((N, 3))
    for a in range(px):
        for b in range(py):
            lin = ix[:, a] * Iy + iy[:, b]
            uu = u[:, lin].T  # (N, P)
            acc0 = np.sum(T * uu, axis=1)
            acc1 = np.sum(dT * uu, axis=1)
            phi += Wx[:, a] * Wy[:, b] * acc0
            grad[:, 0] += dWx[:, a] * Wy[:, b] * acc0
            grad[:, 1] += Wx[:, a] * dWy[:, b] * acc0
            grad[:, 2] += Wx[:, a] * Wy[:, b] * acc1 * (2.0 / Lz)
    c = math.pi * hx * hy
    return c * phi, c * grad


# ----------------------------------------------------------------------------- near field

def near_field(xc, q, box, sog: SOG, chunk=1 << 18):
    """eq. phiNDR over all pairs within r_c (xy periodic, z free); returns (phi, grad)."""
    Lx, Ly, Lz = box
    rc = sog.rc
    pts = np.array(xc, copy=True)
    pts[:, 0] += Lx / 2
    pts[:, 1] += Ly / 2
    pts[:, 2] += Lz / 2 + rc
    for d, L in ((0, Lx), (1, Ly)):
        pts[:, d] = np.where(pts[:, d] >= L, pts[:, d] - L, pts[:, d])
        pts[:, d] = np.where(pts[:, d] < 0, pts[:, d] + L, pts[:, d])
    tree = cKDTree(pts, boxsize=(Lx, Ly, 2 * Lz + 4 * rc))
    pairs = tree.query_pairs(rc, output_type="ndarray")
    N = xc.shape[0]
    phi = np.zeros(N)
    grad = np.zeros((N, 3))
    w, s = sog.w, sog.s
    for st in range(0, pairs.shape[0], chunk):
        i, j = pairs[st:st + chunk, 0], pairs[st:st + chunk, 1]
        d = xc[i] - xc[j]
        d[:, 0] -= Lx * np.round(d[:, 0] / Lx)
        d[:, 1] -= Ly * np.round(d[:, 1] / Ly)
        r = np.sqrt(np.sum(d * d, axis=1))
        keep = r < rc
        i, j, d, r = i[keep], j[keep], d[keep], r[keep]
        e = np.exp(-(r[:, None] ** 2) / s ** 2)
        Nr = 1.0 / r - e @ w
        dN = -1.0 / r ** 2 - (e * (-2.0 * r[:, None] / s ** 2)) @ w
        phi += np.bincount(i, weights=q[j] * Nr, minlength=N) + np.bincount(j, weights=q[i] * Nr, minlength=N)
        g = (dN / r)[:, None] * d  # grad_i of N(|r_i - r_j|)
        for c in range(3):
            grad[:, c] += np.bincount(i, weights=q[j] * g[:, c], minlength=N) - np.bincount(j, weights=q[i] * g[:, c], minlength=N)
    return phi, grad


# ----------------------------------------------------------------------------- totals

def solve(x, q, box, params, parts=False, times=None):
    """Energy, potentials and forces by the fast SOG method with explicit parameters.

    Returns dict(U, phi (N,), force (N,3), grad (N,3)) plus the per-part arrays when parts=True.
    If times is a dict, the wall-clock seconds of the three parts are stored in it under
    "short", "mid" and "long" (the split of the paper's timing tables)."""
    box = tuple(float(v) for v in box)
    q = np.asarray(q, dtype=np.float64)
    xc = centered(x, box)
    sp = params["sog"]
    sog = SOG(sp["b"], sp["r0"], sp["omega"], sp["rc"], sp["M"])
    m = params["m"]
    N = q.size
    t = [time.perf_counter()]
    phi_n, g_n = near_field(xc, q, box, sog)
    t.append(time.perf_counter())
    if m >= 0:
        phi_m, g_m = mid_range(xc, q, box, sog, m, params["mid"])
    else:
        phi_m, g_m = np.zeros(N), np.zeros((N, 3))
    t.append(time.perf_counter())
    if m < sog.M:
        lp = params["long"]
        if lp["form"] == "direct":
            fn = long_range_direct
        elif lp.get("Q", 0) > 0:
            fn = long_range_fft_taylor
        else:
            fn = long_range_fft
        phi_l, g_l = fn(xc, q, box, sog, m, lp)
    else:
        phi_l, g_l = np.zeros(N), np.zeros((N, 3))
    t.append(time.perf_counter())
    if times is not None:
        times.update(short=t[1] - t[0], mid=t[2] - t[1], long=t[3] - t[2])
    phi_self = q * sog.self_coeff()
    phi = phi_n + phi_m + phi_l - phi_self
    grad = g_n + g_m + g_l
    out = dict(U=0.5 * float(q @ phi), phi=phi, grad=grad, force=-q[:, None] * grad)
    if parts:
        out.update(phi_near=phi_n, grad_near=g_n, phi_mid=phi_m, grad_mid=g_m,
                   phi_long=phi_l, grad_long=g_l, phi_self=phi_self)
    return out
