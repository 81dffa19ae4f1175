"""Pins of the CPU oracle against the paper and against mathematics that does not
come from the oracle itself (printed tables, closed forms, brute force,
invariants).  CPU only."""
import math
import os

import numpy as np
import pytest

from oracle import ewald2d as ew
from oracle import fast
from oracle.direct import gaussian_lattice_sum, sog_direct
from oracle.sog import SOG, TABLE1, continuity_residuals, far, solve_r0_omega, weights
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1_fixture():
    rows = []
    with open(os.path.join(GOLDEN, "table1.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = line.split()
                rows.append((float(v[0]), float(v[1]), float(v[2]), float(v[3]), int(v[4]), float(v[5]), int(v[6])))
    return rows


# ---------------------------------------------------------------- SOG decomposition (Sec. 2.2, Table 1)

def test_table1_matches_paper_fixture():
    fx = _table1_fixture()
    assert len(fx) == len(TABLE1) == 6
    for a, b in zip(fx, TABLE1):
        assert a == pytest.approx(b, rel=1e-15)


@pytest.mark.parametrize("row", range(6))
def test_table1_rows_satisfy_c1_continuity(row):
    b, r0, om = _table1_fixture()[row][:3]
    g0, g1 = continuity_residuals(b, r0, om)
    assert abs(g0) < 1e-13 and abs(g1) < 1e-13


def test_newton_recovers_table_row():
    b, r0, om = _table1_fixture()[3][:3]
    r, o = solve_r0_omega(b, r0 * 0.99, 1.0)
    g = continuity_residuals(b, r, o)
    assert max(abs(g[0]), abs(g[1])) < 1e-13
    # the C^1 system is very flat in r0 (the u-series error oscillation is ~1e-8), so r0 is
    # fixed only to ~1e-5 relative while omega is fixed to ~1e-11
    assert abs(o - om) < 1e-9 and abs(r - r0) < 1e-4 * r0


@pytest.mark.parametrize("row", [2, 3, 4])
def test_far_part_reproduces_one_over_r(row):
    """BSA (eq. BSA / pointwiseerror): beyond r_c the far part alone is 1/r up to the
    aliasing error 2 sqrt(2) exp(-pi^2/(2 log b)) and the omitted l<0 terms."""
    b, r0, om = _table1_fixture()[row][:3]
    sigma = 0.7
    rc = r0 * sigma
    w, s = weights(b, sigma, om, 400)
    r = np.linspace(rc, 50 * rc, 200)
    relerr = np.abs(r * far(r, w, s) - 1.0)
    bound = 2 * math.sqrt(2) * math.exp(-math.pi ** 2 / (2 * math.log(b))) + b * math.exp(-(rc / (s[0] / b)) ** 2) * 10
    assert relerr.max() < bound


def test_near_kernel_is_c1_at_cutoff():
    """r_c is a root of 1/r - F and of its derivative (eqs. 2.20, 2.22)."""
    b, r0, om = _table1_fixture()[3][:3]
    sog = SOG(b, r0, om, 3.0, 300)
    rc = sog.rc
    f = 1 / rc - far(rc, sog.w, sog.s)
    h = 1e-5
    fp = ((1 / (rc + h) - far(rc + h, sog.w, sog.s)) - (1 / (rc - h) - far(rc - h, sog.w, sog.s))) / (2 * h)
    assert abs(f) < 1e-12 and abs(fp) < 1e-8


# ---------------------------------------------------------------- Ewald2D

def _small_system(seed=3, N=6, box=(1.0, 1.3, 2.0)):
    rng = np.random.default_rng(seed)
    x = rng.random((N, 3)) * box
    q = np.array([1, -1, 1, -1, 2, -2.0])[:N]
    return x, q, box


def test_ewald2d_alpha_independent():
    x, q, box = _small_system()
    a = ew.ewald2d(x, q, box, alpha=2.0)
    for alpha in (1.0, 4.5):
        b = ew.ewald2d(x, q, box, alpha=alpha)
        assert np.max(np.abs(a["phi"] - b["phi"])) < 1e-12 * np.max(np.abs(a["phi"]))
        assert np.max(np.abs(a["grad"] - b["grad"])) < 1e-12 * np.max(np.abs(a["grad"]))


def test_ewald2d_matches_brute_force_image_sum():
    """Plain image sums of 1/r (Gaussian-damped lattice, extrapolated to no damping)."""
    x, q, box = _small_system()
    e = ew.ewald2d(x, q, box)["phi"]
    bf = ew.brute_force_extrapolated(x, q, box)
    assert np.max(np.abs(bf - e)) < 1e-9 * np.max(np.abs(e))


def test_ewald2d_forces_are_minus_energy_gradient():
    x, q, box = _small_system(seed=5)
    g = ew.ewald2d(x, q, box)["grad"]
    h = 1e-5
    for i in range(3):
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, d] += h
            xm[i, d] -= h
            dU = (ew.energy(q, ew.ewald2d(xp, q, box, forces=False)["phi"])
                  - ew.energy(q, ew.ewald2d(xm, q, box, forces=False)["phi"])) / (2 * h)
            assert dU == pytest.approx(q[i] * g[i, d], abs=1e-8)


def test_ewald2d_translation_invariance():
    x, q, box = _small_system(seed=7)
    a = ew.ewald2d(x, q, box)["phi"]
    y = x + np.array([0.37, -0.21, 0.15])
    b = ew.ewald2d(y, q, box)["phi"]
    assert np.max(np.abs(a - b)) < 1e-12


# ---------------------------------------------------------------- SOG-direct

def test_gaussian_lattice_sum_poisson_identity():
    """Real-space image sum == Poisson-summed Fourier form (App. A.5), both ways."""
    rng = np.random.default_rng(0)
    box = (3.0, 2.5, 4.0)
    d = (rng.random((40, 3)) - 0.5) * box
    q = rng.choice([-1.0, 1.0], 40)
    q[-1] = -q[:-1].sum()  # neutral, as the expm1 form of k = 0 requires
    # width where both forms are affordable: force each form by the box scale trick
    s = 1.6
    v_auto, g_auto = gaussian_lattice_sum(d, q, s, box)
    # explicit real-space sum
    val, g = 0.0, np.zeros(3)
    for nx in range(-20, 21):
        for ny in range(-20, 21):
            dd = d + np.array([nx * box[0], ny * box[1], 0])
            e = q * np.exp(-np.sum(dd * dd, 1) / s ** 2)
            val += e.sum()
            g += -2 / s ** 2 * (e @ dd)
    assert v_auto == pytest.approx(val, abs=1e-12)
    assert np.allclose(g_auto, g, atol=1e-12)
    # explicit Fourier sum
    A = box[0] * box[1]
    vf = 0.0
    for nx in range(-30, 31):
        for ny in range(-30, 31):
            kx, ky = 2 * math.pi * nx / box[0], 2 * math.pi * ny / box[1]
            vf += np.sum(q * math.pi * s * s / A * np.exp(-d[:, 2] ** 2 / s ** 2) * math.exp(-s * s * (kx * kx + ky * ky) / 4)
                         * np.cos(kx * d[:, 0] + ky * d[:, 1]))
    assert vf == pytest.approx(val, abs=1e-12)


def _fig1_system():
    """Sec. 2.3: 100 random monovalent particles in a unit cube, r_c = 0.3 (Fig. 1 setup)."""
    x, q = workloads.uniform(100, (1.0, 1.0, 1.0), seed=11)
    return x, q, (1.0, 1.0, 1.0)


@pytest.fixture(scope="module")
def fig1_reference():
    x, q, box = _fig1_system()
    return x, q, box, ew.ewald2d(x, q, box)


@pytest.mark.parametrize("row", [2, 3, 4, 5])
def test_sog_direct_within_table1_error(fig1_reference, row):
    """SOG decomposition error vs Ewald2D is within Table 1's printed energy and force errors."""
    x, q, box, ref = fig1_reference
    b, r0, om, eE, ME, eF, MF = _table1_fixture()[row]
    sog = SOG(b, r0, om, 0.3, ME)
    o = sog_direct(x, q, box, sog, m=sog.split_index(0.5, 1.0), targets=np.arange(q.size))
    Uref = ew.energy(q, ref["phi"])
    eU = abs(ew.energy(q, o["phi"]) - Uref) / abs(Uref)
    Fref = -q[:, None] * ref["grad"]
    F = -q[:, None] * o["grad"]
    eFm = np.max(np.abs(F - Fref)) / np.max(np.abs(Fref))
    assert eU <= max(eE, 1e-14)
    assert eFm <= max(eF, 1e-13)


def test_sog_direct_split_and_cutoff_invariance(fig1_reference):
    """m only moves Gaussians between two sums; r_c changes the decomposition but not the
    answer (both tested against Ewald2D at b = 1.1488, error ~1e-15)."""
    x, q, box, ref = fig1_reference
    b, r0, om = _table1_fixture()[5][:3]
    T = np.arange(0, 100, 7)
    outs = []
    for rc, eta in ((0.3, 0.2), (0.3, 0.8), (0.45, 0.5)):
        sog = SOG(b, r0, om, rc, 320)
        outs.append(sog_direct(x, q, box, sog, m=sog.split_index(eta, 1.0), targets=T))
    for o in outs:
        assert np.max(np.abs(o["phi"] - ref["phi"][T])) < 1e-12 * np.max(np.abs(ref["phi"]))
    assert np.max(np.abs(outs[0]["phi_mid"] - outs[1]["phi_mid"])) > 1e-3  # the split really moved


# ---------------------------------------------------------------- Chebyshev (App. A.2, Thm thm::Che)

def test_lagrange_basis_interpolates_polynomials_exactly():
    P = 9
    t = np.linspace(-1, 1, 57)
    L, dL = fast.lagrange(t, P)
    tc = fast.cheb_nodes(P)
    for deg in range(P):
        c = np.random.default_rng(deg).normal(size=deg + 1)
        f = np.polynomial.polynomial.polyval(tc, c)
        assert np.allclose(L @ f, np.polynomial.polynomial.polyval(t, c), atol=1e-12)
        dc = np.polynomial.polynomial.polyder(c)
        assert np.allclose(dL @ f, np.polynomial.polynomial.polyval(t, dc) if deg else 0 * t, atol=1e-10)
    assert np.allclose(L.sum(axis=1), 1.0, atol=1e-14)
    # cardinal property at the nodes
    Ln, _ = fast.lagrange(tc, P)
    assert np.allclose(Ln, np.eye(P), atol=1e-13)


def test_chebyshev_digits_of_theorem_che():
    rows = []
    with open(os.path.join(GOLDEN, "chebyshev_digits.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                eta, P, dig = line.split()
                rows.append((float(eta), int(P), int(dig)))
    Lz = 1.0
    z = np.linspace(-Lz / 2, Lz / 2, 2001)
    for eta, P, dig in rows:
        s = eta * Lz
        f = lambda zz: np.exp(-zz ** 2 / s ** 2)
        L, _ = fast.lagrange(2 * z / Lz, P)
        err = np.max(np.abs(L @ f(0.5 * Lz * fast.cheb_nodes(P)) - f(z)))
        # Thm thm::Che's bound with the two constants its proof drops: the monic Chebyshev
        # node polynomial has max 2^(1-P) (not 2^-P) and Cramer's Hermite-function
        # inequality behind eq. 2.38 carries a factor 1.0865
        bound = 2 * 1.0865 / (math.sqrt(math.factorial(P)) * (2 * math.sqrt(2) * eta) ** P)
        assert err <= bound + 1e-14  # 1e-14: the FP64 round-off floor of the evaluation
        assert err <= max(5 * 10.0 ** (-dig), 1e-14)  # "about dig digits"


# ---------------------------------------------------------------- fast method vs SOG-direct

@pytest.fixture(scope="module")
def cube_case():
    """N=1000 in a 20^3 box (Sec. 5.1's accuracy-test box), b = 1.3207, r_c = 4, eta = 0.4."""
    x, q = workloads.uniform(1000, (20.0, 20.0, 20.0), seed=1)
    box = (20.0, 20.0, 20.0)
    b, r0, om = _table1_fixture()[3][:3]
    sog = SOG(b, r0, om, 4.0, 100)
    m = sog.split_index(0.4, 20.0)
    T = np.arange(0, 1000, 25)
    ref = sog_direct(x, q, box, sog, m, T)
    return x, q, box, sog, m, T, ref


def test_fast_near_is_exact(cube_case):
    x, q, box, sog, m, T, ref = cube_case
    p, g = fast.near_field(fast.centered(x, box), q, box, sog)
    assert np.max(np.abs(p[T] - ref["phi_near"])) < 1e-12
    assert np.max(np.abs(g[T] - ref["grad_near"])) < 1e-11


def test_fast_mid_converges_gaussian_rate_in_grid(cube_case):
    """Fig. 2(b) / Thm thm::trunFour: error falls like exp(-C I^2) with the grid size I."""
    x, q, box, sog, m, T, ref = cube_case
    xc = fast.centered(x, box)
    scale = np.max(np.abs(ref["phi"]))
    errs = []
    for I in (24, 28, 32):
        mid = dict(I=(I, I, I), Izs=2 * I + 40, Pw=(19, 19, 19), S=0.455 * math.pi * 19)
        p, _ = fast.mid_range(xc, q, box, sog, m, mid)
        errs.append(np.max(np.abs(p[T] - ref["phi_mid"])) / scale)
    # exp(-(pi s0 / 2h)^2) times a constant: successive ratios must match the Gaussian rate
    s0 = sog.s[0]
    for (I1, e1), (I2, e2) in zip(((24, errs[0]), (28, errs[1])), ((28, errs[1]), (32, errs[2]))):
        pred = math.exp(-(math.pi * s0 / 2) ** 2 * ((I2 / 20.0) ** 2 - (I1 / 20.0) ** 2))
        assert 0.2 * pred < e2 / e1 < 5 * pred
    assert errs[-1] < 1e-5


def test_fast_mid_converges_in_window_support(cube_case):
    """Fig. 2(a) / Thm thm::scal: error falls with the window support P_w."""
    x, q, box, sog, m, T, ref = cube_case
    xc = fast.centered(x, box)
    scale = np.max(np.abs(ref["phi"]))
    prev = 1.0
    for Pw in (5, 9, 13):
        mid = dict(I=(48, 48, 48), Izs=140, Pw=(Pw, Pw, Pw), S=0.455 * math.pi * Pw)
        p, g = fast.mid_range(xc, q, box, sog, m, mid)
        e = np.max(np.abs(p[T] - ref["phi_mid"])) / scale
        assert e < 0.1 * prev
        prev = e
    assert prev < 2e-7
    assert np.max(np.abs(g[T] - ref["grad_mid"])) < 1e-6 * np.max(np.abs(ref["grad"]))


def test_fast_long_direct_converges_spectrally(cube_case):
    x, q, box, sog, m, T, ref = cube_case
    xc = fast.centered(x, box)
    scale = np.max(np.abs(ref["phi"]))
    errs = []
    for P, nk in ((8, 3), (12, 4), (20, 6)):
        p, g = fast.long_range_direct(xc, q, box, sog, m, dict(form="direct", P=P, nk=(nk, nk)))
        errs.append(np.max(np.abs(p[T] - ref["phi_long"])) / scale)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-11
    assert np.max(np.abs(g[T] - ref["grad_long"])) < 1e-10 * np.max(np.abs(ref["grad"]))


def test_fast_long_fft_form_converges(cube_case):
    x, q, box, sog, m, T, ref = cube_case
    xc = fast.centered(x, box)
    scale = np.max(np.abs(ref["phi"]))
    errs = []
    for I2, Pw2 in ((16, 7), (24, 11), (32, 15)):
        lp = dict(form="fft", P=16, I=(I2, I2), Pw=(Pw2, Pw2), S=0.455 * math.pi * Pw2)
        p, g = fast.long_range_fft(xc, q, box, sog, m, lp)
        errs.append(np.max(np.abs(p[T] - ref["phi_long"])) / scale)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-8


# ---------------------------------------------------------------- invariants of the fast discrete operator

@pytest.fixture(scope="module")
def small_fast():
    x, q = workloads.uniform(200, (8.0, 9.0, 7.0), seed=21)
    box = (8.0, 9.0, 7.0)
    b, r0, om = _table1_fixture()[3][:3]
    rc = 2.5
    sog = SOG(b, r0, om, rc, 120)
    m = sog.split_index(0.35, box[2])
    params = fast.make_params(b, r0, om, rc, 120, m,
                              mid=dict(I=(20, 24, 18), Izs=44, Pw=(9, 9, 9), S=0.455 * math.pi * 9),
                              long=dict(form="direct", P=14, nk=(5, 5)))
    return x, q, box, params


def test_fast_forces_are_minus_gradient_of_discrete_energy(small_fast):
    x, q, box, params = small_fast
    o = fast.solve(x, q, box, params)
    h = 1e-6
    for i in (0, 57, 133):
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, d] += h
            xm[i, d] -= h
            dU = (fast.solve(xp, q, box, params)["U"] - fast.solve(xm, q, box, params)["U"]) / (2 * h)
            assert -dU == pytest.approx(o["force"][i, d], abs=2e-6 * max(1.0, abs(o["force"][i, d])))


def test_fast_charge_flip_and_net_force(small_fast):
    x, q, box, params = small_fast
    a = fast.solve(x, q, box, params)
    b = fast.solve(x, -q, box, params)
    assert a["U"] == pytest.approx(b["U"], rel=1e-12)
    assert np.allclose(a["phi"], -b["phi"], atol=1e-11)
    assert np.allclose(a["force"], b["force"], atol=1e-10)
    # Newton's third law holds for the exact operator; the grid breaks translation
    # invariance, so the discrete one keeps it only to its discretisation error (~2e-4
    # per particle at these coarse parameters)
    assert np.max(np.abs(a["force"].sum(axis=0))) < 1e-2 * np.max(np.abs(a["force"]))


def test_fast_total_matches_ewald2d():
    """End to end: the fast method at tight parameters reproduces Ewald2D (Sec. 5.1 box)."""
    x, q = workloads.uniform(1000, (20.0, 20.0, 20.0), seed=1)
    box = (20.0, 20.0, 20.0)
    b, r0, om = _table1_fixture()[4][:3]
    rc = 4.0
    sog = SOG(b, r0, om, rc, 200)
    m = sog.split_index(0.4, 20.0)
    params = fast.make_params(b, r0, om, rc, 200, m,
                              mid=dict(I=(64, 64, 64), Izs=200, Pw=(17, 17, 17), S=0.455 * math.pi * 17),
                              long=dict(form="direct", P=20, nk=(6, 6)))
    o = fast.solve(x, q, box, params)
    T = np.arange(0, 1000, 9)
    ref = ew.ewald2d(x, q, box, targets=T)
    assert np.max(np.abs(o["phi"][T] - ref["phi"])) < 1e-8 * np.max(np.abs(ref["phi"]))
    Fref = -q[T, None] * ref["grad"]
    assert np.max(np.abs(o["force"][T] - Fref)) < 1e-7 * np.max(np.abs(Fref))


def test_all_long_regime_matches_mid_plus_long():
    """Remark after the range-splitting definition: with every Gaussian long-range the
    mid-range solver is skipped and the answer is unchanged."""
    x, q = workloads.uniform(300, (12.0, 12.0, 1.5), seed=9)
    box = (12.0, 12.0, 1.5)
    b, r0, om = _table1_fixture()[4][:3]
    rc = 2.0
    sog = SOG(b, r0, om, rc, 200)
    ref = sog_direct(x, q, box, sog, m=-1, targets=np.arange(0, 300, 11))
    # s_0 = 0.5 is narrow, so the direct form needs |k| up to ~21 (nk = 40) here
    params = fast.make_params(b, r0, om, rc, 200, -1, long=dict(form="direct", P=20, nk=(40, 40)))
    o = fast.solve(x, q, box, params)
    T = np.arange(0, 300, 11)
    assert np.max(np.abs(o["phi"][T] - ref["phi"])) < 1e-8 * np.max(np.abs(ref["phi"]))


# ---------------------------------------------------------------- ES window (oracle option)

def test_es_window_transform_pins():
    """The quadrature transform of the ES window: beta = 0 is the box window, whose
    transform is 2 sin(k a)/k; for beta = 2.3 P_w it agrees with a fine midpoint sum of
    the definition (an independent rule)."""
    h, Pw = 0.4, 7
    a = 0.5 * Pw * h
    k = np.array([0.1, 1.0, 3.0, 7.7, 15.0])
    assert np.max(np.abs(fast.window_hat_es(k, h, Pw, 0.0) - 2 * np.sin(k * a) / k)) < 1e-12
    beta = 2.3 * Pw
    M = 400_000
    xm = (np.arange(M) + 0.5) / M * 2 * a - a
    W = np.exp(beta * (np.sqrt(1 - (xm / a) ** 2) - 1))
    for kk in (0.0, 2.0, 7.8):
        bf = np.sum(W * np.cos(kk * xm)) * (2 * a / M)
        assert abs(fast.window_hat_es(np.array([kk]), h, Pw, beta)[0] - bf) < 1e-9 * abs(bf) + 1e-13


def test_es_window_weights_and_derivative():
    """Weights: the P_w nodes nearest x are exactly the nodes inside the support, W is 1 at
    the centre and exp(-beta) at the edge; dW agrees with central differences of W."""
    h, Pw, beta = 0.5, 7, 16.0
    xs = np.array([0.013, 1.2345, -0.74, 3.0 - 1e-3])
    idx, W, dW = fast.window_1d_es(xs, 0.0, h, 100, Pw, beta, True)
    dx = xs[:, None] - idx * h
    dx = dx - 100 * h * np.round(dx / (100 * h))
    assert np.all(np.abs(dx) < 0.5 * Pw * h)
    i0, W0, _ = fast.window_1d_es(np.array([0.0]), 0.0, h, 100, Pw, beta, True)
    assert abs(W0[0, (Pw - 1) // 2] - 1.0) < 1e-15
    e = 1e-6
    _, Wp, _ = fast.window_1d_es(xs + e, 0.0, h, 100, Pw, beta, True)
    _, Wm, _ = fast.window_1d_es(xs - e, 0.0, h, 100, Pw, beta, True)
    assert np.max(np.abs((Wp - Wm) / (2 * e) - dW)) < 1e-6 * np.max(np.abs(dW))


def test_fast_mid_es_window_converges(cube_case):
    """With the ES window the mid range converges to SOG-direct as the support grows,
    faster than the Gaussian window (at I = 48: P_w = 9 beats the Gaussian's P_w = 13)."""
    x, q, box, sog, m, T, ref = cube_case
    xc = fast.centered(x, box)
    scale = np.max(np.abs(ref["phi"]))
    gscale = np.max(np.abs(ref["grad"]))
    prev = 1.0
    for Pw in (5, 7, 9):
        mid = dict(I=(48, 48, 48), Izs=144, Pw=(Pw, Pw, Pw), window="es", beta=2.3 * Pw)
        p, g = fast.mid_range(xc, q, box, sog, m, mid)
        e = np.max(np.abs(p[T] - ref["phi_mid"])) / scale
        assert e < 0.05 * prev
        prev = e
    assert prev < 2e-8
    assert np.max(np.abs(g[T] - ref["grad_mid"])) < 2e-7 * gscale


# ---------------------------------------------------------------- KB window, polynomial windows

def test_kb_window_transform_pins():
    """The closed-form KB transform: beta = 0 is the box window (2 sin(k a)/k); for
    beta = 2.3 P_w it agrees with a fine midpoint sum of the definition, on both sides of
    k a = beta (the sinh and sin branches) and at the branch point itself."""
    from scipy.special import i0
    h, Pw = 0.4, 7
    a = 0.5 * Pw * h
    k = np.array([0.1, 1.0, 3.0, 7.7, 15.0])
    assert np.max(np.abs(fast.window_hat_kb(k, h, Pw, 0.0) - 2 * np.sin(k * a) / k)) < 1e-12
    beta = 2.3 * Pw
    M = 400_000
    xm = (np.arange(M) + 0.5) / M * 2 * a - a
    W = i0(beta * np.sqrt(1 - (xm / a) ** 2)) / i0(beta)
    for kk in (0.0, 2.0, beta / a, 15.0, 25.0):
        bf = np.sum(W * np.cos(kk * xm)) * (2 * a / M)
        assert abs(fast.window_hat_kb(np.array([kk]), h, Pw, beta)[0] - bf) < 1e-8 * abs(fast.window_hat_kb(np.array([0.0]), h, Pw, beta)[0])


def test_kb_window_weights_and_derivative():
    """Weights: the P_w nodes nearest x are inside the support, W is 1 at the centre and
    1/I_0(beta) at the support's edge; dW agrees with central differences of W."""
    from scipy.special import i0
    h, Pw, beta = 0.5, 7, 16.0
    xs = np.array([0.013, 1.2345, -0.74, 3.0 - 1e-3])
    idx, W, dW = fast.window_1d_kb(xs, 0.0, h, 100, Pw, beta, True)
    dx = xs[:, None] - idx * h
    dx = dx - 100 * h * np.round(dx / (100 * h))
    assert np.all(np.abs(dx) <= 0.5 * Pw * h)
    _, W0, _ = fast.window_1d_kb(np.array([0.0]), 0.0, h, 100, Pw, beta, True)
    assert abs(W0[0, (Pw - 1) // 2] - 1.0) < 1e-15
    assert abs(fast.kb_value(np.array([0.5 * Pw * h]), 0.5 * Pw * h, beta)[0] - 1 / i0(beta)) < 1e-15
    e = 1e-6
    _, Wp, _ = fast.window_1d_kb(xs + e, 0.0, h, 100, Pw, beta, True)
    _, Wm, _ = fast.window_1d_kb(xs - e, 0.0, h, 100, Pw, beta, True)
    assert np.max(np.abs((Wp - Wm) / (2 * e) - dW)) < 1e-6 * np.max(np.abs(dW))


def test_polynomial_window_exact_on_polynomials_and_converges():
    """Remark rmk::PWindow's polynomial windows: a window that is itself a polynomial of
    degree <= nu in the offset is reproduced to rounding (with its derivative), and the KB
    window's approximation error falls geometrically with nu (below 1e-11 at nu = 10 and
    P_w = 9, the Sec. 5.1 setting)."""
    h, Pw = 0.5, 5
    u = np.linspace(-0.5, 0.5, 41)
    poly = lambda x: 1.0 + 0.3 * x - 0.7 * x ** 3 + 0.05 * x ** 4  # degree 4 in x = h (o - u)
    dpoly = lambda x: 0.3 - 2.1 * x ** 2 + 0.2 * x ** 3
    W, dW = fast.window_poly_1d(poly, u, h, Pw, 4)
    off = np.arange(Pw) - (Pw - 1) // 2
    X = h * (off[None, :] - u[:, None])
    assert np.max(np.abs(W - poly(X))) < 1e-13
    assert np.max(np.abs(dW + dpoly(X))) < 1e-12  # d/dx_particle = -d/dX
    Pw, beta = 9, 2.3 * 9
    xs = np.random.default_rng(0).uniform(-10, 10, 500)
    _, W1, d1 = fast.window_1d_kb(xs, 0.0, h, 100, Pw, beta, True)
    errs = []
    for nu in (4, 6, 8, 10):
        _, W2, d2 = fast.window_1d_kb(xs, 0.0, h, 100, Pw, beta, True, nu=nu)
        errs.append(np.max(np.abs(W2 - W1)))
    assert all(errs[i + 1] < 0.02 * errs[i] for i in range(3))
    assert errs[-1] < 1e-11


def test_fast_mid_kb_window_converges(cube_case):
    """With the KB window the mid range converges to SOG-direct as the support grows (as
    fast as ES: P_w = 9 at I = 48 within 1e-8), and the degree-10 polynomial form gives the
    same potentials as the exact window to 1e-10."""
    x, q, box, sog, m, T, ref = cube_case
    xc = fast.centered(x, box)
    scale = np.max(np.abs(ref["phi"]))
    gscale = np.max(np.abs(ref["grad"]))
    prev = 1.0
    for Pw in (5, 7, 9):
        mid = dict(I=(48, 48, 48), Izs=144, Pw=(Pw, Pw, Pw), window="kb", beta=2.3 * Pw)
        p, g = fast.mid_range(xc, q, box, sog, m, mid)
        e = np.max(np.abs(p[T] - ref["phi_mid"])) / scale
        assert e < 0.05 * prev
        prev = e
    assert prev < 1e-8
    assert np.max(np.abs(g[T] - ref["grad_mid"])) < 5e-7 * gscale
    mid["nu"] = 10
    p2, g2 = fast.mid_range(xc, q, box, sog, m, mid)
    assert np.max(np.abs(p2 - p)) < 1e-10 * scale
    assert np.max(np.abs(g2 - g)) < 1e-9 * gscale


@pytest.mark.parametrize("system", [86, 32])
def test_batch_golden_values_match_ewald2d(system):
    """The stored sampled targets of the batch (oracle SOG-direct per system) agree with the
    independent Ewald2D sum on a tall thin system (Lz/Lx = 8, Lx = 4) and a flat one
    (Lz/Lx = 1/8) to the Table 1 row's decomposition error."""
    d = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_256_targets.txt"),
                   comments="#")
    rows = d[d[:, 0] == system]
    N, box, seed = workloads.batch_specs()[system]
    x, q = workloads.uniform(N, box, seed)
    o = ew.ewald2d(x, q, box, targets=rows[:, 1].astype(np.int64))
    assert np.max(np.abs(o["phi"] - rows[:, 2])) <= 1e-8 * np.max(np.abs(rows[:, 2]))
    assert np.max(np.abs(o["grad"] - rows[:, 3:6])) <= 1e-8 * np.max(np.abs(rows[:, 3:6]))


# ---------------------------------------------------------------- App. C Taylor form (strongly confined boxes)

def test_taylor_series_matches_lemma_digits():
    """Lemma lemma::Taylor: the Q-term series of exp(-z^2/s^2) with s = eta Lz errs by at
    most 1/(Q! (2 eta)^{2Q}) on [-Lz/2, Lz/2], which is the printed number of digits for
    eta = 1 (tests/golden/taylor_digits.txt).  On [-Lz, Lz] (the range of z - z_j, the
    reading the algorithm needs) the bound is 1/(Q! eta^{2Q})."""
    rows = np.loadtxt(os.path.join(GOLDEN, "taylor_digits.txt"), comments="#")
    Lz = 1.0
    for eta, Q, dig in rows:
        Q = int(Q)
        s = eta * Lz
        z = np.linspace(-Lz / 2, Lz / 2, 2001)
        err = np.max(np.abs(np.exp(-(z / s) ** 2) - fast.taylor_gaussian(z, s, Q)))
        # 4e-16: the float64 rounding of exp and of the series near 1
        assert err <= 1.0 / (math.factorial(Q) * (2 * eta) ** (2 * Q)) + 4e-16
        assert 10.0 ** (-dig - 1) < err + 1e-16 <= 10.0 ** (-dig + 0.5)
        z2 = np.linspace(-Lz, Lz, 4001)
        err2 = np.max(np.abs(np.exp(-(z2 / s) ** 2) - fast.taylor_gaussian(z2, s, Q)))
        assert err2 <= 1.0 / (math.factorial(Q) * eta ** (2 * Q)) + 4e-16


def test_taylor_coefficients_rebuild_the_exact_kernel():
    """sum_p A_p(k) (dz/Lz)^{2p} is the z kernel pi^{-1} K(k; dz) of eq. trun2 (oracle
    long_kernel, which sums the Gaussians themselves) once Q is large; at k = 0 both leave
    out the constant that multiplies the total charge."""
    b, r0, om = _table1_fixture()[3][:3]
    sog = SOG(b, r0, om, 3.0, 120)
    Lz = 0.3
    k2 = np.array([0.0, 0.04, 0.9, 7.5])
    zc = np.array([-0.15, 0.0, 0.11])
    K = fast.long_kernel(k2, sog, -1, zc)  # (nk, 3, 3), pi included
    A = fast.taylor_coefficients(k2, sog, -1, Lz, 9)
    dz = (zc[:, None] - zc[None, :]) / Lz
    KT = np.einsum("kp,pab->kab", A, np.stack([dz ** (2 * p) for p in range(9)]))
    assert np.max(np.abs(math.pi * KT - K)) < 1e-12 * np.max(np.abs(K))
    assert np.all(A[0, 0] == 0.0)


@pytest.fixture(scope="module")
def thin_case():
    """The paper's strongly confined setting at N ~ 1000: surface density 1.1, Lz = 0.3
    (Sec. 5.3 and App. E), every Gaussian long range (s_0 > eta Lz)."""
    box = (30.0, 30.0, 0.3)
    x, q = workloads.uniform(990, box, 41)
    b, r0, om = _table1_fixture()[3][:3]
    sog = SOG(b, r0, om, 3.0, 120)
    T = np.arange(0, 990, 45)
    ref = sog_direct(x, q, box, sog, -1, T)
    return x, q, box, sog, T, ref


def test_fast_long_taylor_converges_at_lemma_rate(thin_case):
    """Fig. 5(c): the Taylor form's error falls with Q within the bound of Lemma
    lemma::Taylor (read on [-Lz, Lz]: 1/(Q! eta^{2Q}), eta = s_0/Lz), down to the floor
    the 2D grid and P set, where it agrees with the exact-kernel FFT form."""
    x, q, box, sog, T, ref = thin_case
    xc = fast.centered(x, box)
    scale = np.max(np.abs(ref["phi"]))
    lp = dict(form="fft", P=8, I=(96, 96), Pw=(15, 15), S=0.455 * math.pi * 15)
    pe, ge = fast.long_range_fft(xc, q, box, sog, -1, lp)
    floor = np.max(np.abs(pe[T] - ref["phi_long"])) / scale
    assert floor < 5e-8
    eta = sog.s[0] / box[2]
    errs = []
    for Q in (1, 2, 3, 4):
        p, g = fast.long_range_fft_taylor(xc, q, box, sog, -1, dict(lp, Q=Q))
        e = np.max(np.abs(p[T] - ref["phi_long"])) / scale
        errs.append(e)
        assert e <= 1.0 / (math.factorial(Q) * eta ** (2 * Q)) + 2 * floor
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    p, g = fast.long_range_fft_taylor(xc, q, box, sog, -1, dict(lp, Q=6))
    assert np.max(np.abs(p - pe)) < 2e-8 * scale
    assert np.max(np.abs(g[T] - ref["grad_long"])) < 1e-7 * np.max(np.abs(ref["grad"]))
