"""Host-side checks of the C ABI (no GPU needed, no compute calls).

* the library loads and exports every function include/sog.h declares;
* status strings, option defaults;
* the planner (sog_plan_resolve runs on a machine without a GPU): argument checks, and
  the structural properties every plan must have for the workloads of the benchmark.
"""
import math
import os
import re

import pytest

import paper_2412_04595_amd as sog
from paper_2412_04595_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sog.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(sog_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("sog_plan", "sog_energy_potential_force", "sog_destroy", "sog_plan_resolve"):
        assert must in names


def test_library_exports_every_declared_function():
    L = _lib.lib()
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding covers exactly what the header declares
    assert sorted(_lib.EXPORTS) == _declared_functions()


def test_status_strings():
    for code, name in _lib.STATUS.items():
        assert sog.sog_status_string(code) == name
    assert "unknown" in sog.sog_status_string(99).lower()


def test_option_defaults():
    o = sog.sog_options_default()
    assert o.precision == sog.SOG_PREC_FP64 and o.device == 0 and not o.stream
    assert o.pointers_on_device == 0 and o.check_inputs == 1 and o.timing == 0
    assert o.params.mid_I[0] == 0 and o.params.long_P == 0


def _resolve_status(box, n, tol, precision="fp64", params=None):
    try:
        sog.plan_parameters(box, n, tol, precision, params)
        return _lib.SOG_OK
    except sog.SogError as e:
        assert sog.sog_last_error()  # every failure leaves a message
        return e.status


@pytest.mark.parametrize("box,n,tol,prec,status", [
    ((0, 10, 10), 100, 1e-4, "fp64", 1),
    ((10, -1, 10), 100, 1e-4, "fp64", 1),
    ((10, 10, float("inf")), 100, 1e-4, "fp64", 1),
    ((10, 10, 10), 1, 1e-4, "fp64", 1),
    ((10, 10, 10), (1 << 26) + 1, 1e-4, "fp64", 1),
    ((10, 10, 10), 100, 1e-13, "fp64", 4),
    ((10, 10, 10), 100, 1e-6, "fp32", 4),
    ((10, 10, 10), 100, 0.5, "fp64", 4),
    ((10, 10, 10), 100, float("nan"), "fp64", 4),
])
def test_resolve_rejects_bad_arguments(box, n, tol, prec, status):
    assert _resolve_status(box, n, tol, prec) == status


@pytest.mark.parametrize("params", [
    dict(mid_Pw=[8, 8, 8]),        # even window
    dict(mid_Pw=[9, 9, 7]),        # not equal in x, y, z
    dict(long_P=65),
    dict(mid_Izs=81),              # odd padded z grid
    dict(mid_Pw=[17, 17, 17]),     # wider than the kernels are built for
    dict(mid_window=4),            # no such window
    dict(mid_window=2, mid_S=12.0),  # the Gaussian's shape given for the ES window
    dict(mid_window=3, mid_S=12.0),  # ... or for the KB window
    dict(mid_beta=-1.0),
    dict(mid_nu=8),                # a polynomial degree for a window that takes none
    dict(mid_window=3, mid_nu=1),  # degree out of [2, 16]
    dict(mid_window=3, mid_nu=17),
])
def test_resolve_rejects_bad_overrides(params):
    assert _resolve_status((20, 20, 20), 1000, 1e-4, "fp64", params) == _lib.SOG_ERR_INVALID_ARG


def _smooth(n):
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


WORKLOADS = {
    "cube_small": ((20.0, 20.0, 20.0), 1000),
    "cube_1e6": ((100.0, 100.0, 100.0), 1000000),
    "slab_1e6": ((400.0, 400.0, 25.0), 1000000),
    "tall_1e6": ((50.0, 50.0, 800.0), 1000000),
    "layered_2e5": ((150.0, 150.0, 60.0), 200000),
}


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("fp64", 1e-4), ("fp64", 1e-6)])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_plan_structure(name, prec, tol):
    box, n = WORKLOADS[name]
    p = sog.plan_parameters(box, n, tol, prec)
    Lx, Ly, Lz = box
    # the cut-off fits the periodic cell (minimum image in x, y)
    assert 0 < p["rc"] <= 0.5 * min(Lx, Ly) + 1e-12
    # Table-1 rows: b in (1, 2]; the decomposition has M >= m
    assert 1.0 < p["b"] <= 2.0 and p["M"] >= p["m"] >= -1
    sigma = p["rc"] / p["r0"]
    s = [math.sqrt(2.0) * sigma * p["b"] ** l for l in range(p["M"] + 1)]  # s_l = sqrt(2) b^l sigma
    if p["m"] >= 0:
        I, Izs, Pw = p["mid_I"], p["mid_Izs"], p["mid_Pw"][0]
        # mid range: the split m = max{l : s_l <= eta Lz} with the planner's eta <= 2;
        # grids even, FFT-smooth, window odd
        assert s[p["m"]] <= 2.0 * Lz * (1 + 1e-12)
        assert I[0] % 2 == 0 and I[1] % 2 == 0 and Izs % 2 == 0
        assert _smooth(I[0]) and _smooth(I[1]) and _smooth(Izs // 2)
        assert Pw % 2 == 1 and 3 <= Pw <= 15  # the widest window the kernels are built for
        # the padded z grid holds the box, the window support and some padding
        hz = Lz / I[2]
        assert Izs * hz >= Lz + (Pw - 1) * hz
        # the grid resolves the narrowest mid-range Gaussian: exp(-(s0 pi / (2 h))^2) < tol
        h = max(Lx / I[0], Ly / I[1], hz)
        assert math.exp(-(s[0] * math.pi / (2 * h)) ** 2) < tol
    if p["m"] < p["M"]:
        assert 1 <= p["long_P"] <= 64
        assert p["long_form"] in (_lib.SOG_LONG_DIRECT, _lib.SOG_LONG_FFT)
        if p["long_form"] == _lib.SOG_LONG_DIRECT:
            assert p["long_nk"][0] >= 0 and p["long_nk"][1] >= 0
        else:
            assert _smooth(p["long_I"][0]) and _smooth(p["long_I"][1]) and p["long_Pw"][0] % 2 == 1


def test_resolve_is_deterministic_and_respects_overrides():
    a = sog.plan_parameters((20, 20, 20), 1000, 1e-6, "fp64")
    b = sog.plan_parameters((20, 20, 20), 1000, 1e-6, "fp64")
    assert a == b
    c = sog.plan_parameters((20, 20, 20), 1000, 1e-6, "fp64",
                            dict(mid_I=[32, 32, 32], mid_Izs=80, mid_Pw=[9, 9, 9]))
    assert c["mid_I"] == [32, 32, 32] and c["mid_Izs"] == 80 and c["mid_Pw"] == [9, 9, 9]


def test_eta_sets_the_range_split():
    """eta (the range-splitting definition, Sec. 3.1): m is the last Gaussian with
    s_l <= eta L_z, so a larger eta moves Gaussians into the mid range; the resolved eta
    is the given one, or s_m / L_z of the split the cost model chose; set_m wins over eta."""
    import numpy as np
    from oracle.sog import SOG
    box, n, tol = (50.0, 50.0, 200.0), 100000, 1e-4
    auto = sog.plan_parameters(box, n, tol, "fp32")
    s = SOG(auto["b"], auto["r0"], auto["omega"], auto["rc"], auto["M"]).s
    assert auto["m"] >= 0 and abs(auto["eta"] - s[auto["m"]] / box[2]) < 1e-12
    for eta in (0.1, 0.3, 1.0):
        p = sog.plan_parameters(box, n, tol, "fp32", dict(eta=eta))
        s = SOG(p["b"], p["r0"], p["omega"], p["rc"], p["M"]).s
        want = int(np.max(np.nonzero(s[: p["M"] + 1] <= eta * box[2])[0], initial=-1))
        assert p["m"] == want and p["eta"] == eta
    lo = sog.plan_parameters(box, n, tol, "fp32", dict(eta=0.1))
    hi = sog.plan_parameters(box, n, tol, "fp32", dict(eta=1.0))
    # a wider long range needs fewer Chebyshev terms in z (Thm thm::Che)
    assert lo["m"] < hi["m"] and lo["long_P"] > hi["long_P"]
    forced = sog.plan_parameters(box, n, tol, "fp32", dict(eta=1.0, set_m=1, m=lo["m"]))
    assert forced["m"] == lo["m"]
    assert _resolve_status(box, n, tol, "fp32", dict(eta=-1.0)) == _lib.SOG_ERR_INVALID_ARG


def test_deterministic_plans():
    """The deterministic option keeps every parameter of the plan (only the gridding tiles
    may shrink, which the parameters do not show) and is refused for values other than 0
    and 1."""
    for box, n, tol, prec in [((100, 100, 100), 1000000, 1e-4, "fp32"), ((20, 20, 20), 1000, 1e-8, "fp64"),
                              ((953.5, 953.5, 0.3), 1000000, 1e-4, "fp32")]:
        a = sog.plan_parameters(box, n, tol, prec)
        b = sog.plan_parameters(box, n, tol, prec, deterministic=True)
        assert a == b
    o = sog.make_options("fp64")
    o.deterministic = 2
    with pytest.raises(sog.SogError):
        _lib.sog_plan_resolve((20, 20, 20), 1000, 1e-6, o)


def test_tighter_tolerance_refines():
    lo = sog.plan_parameters((100, 100, 100), 1000000, 1e-4, "fp64")
    hi = sog.plan_parameters((100, 100, 100), 1000000, 1e-8, "fp64")
    assert hi["b"] <= lo["b"]
    assert hi["mid_Pw"][0] >= lo["mid_Pw"][0]


@pytest.mark.parametrize("tol", [1e-6, 1e-8, 1e-10, 1e-12])
def test_tight_tolerance_small_box_plans(tol):
    # every window the planner picks fits the kernels (P_w <= 15); the lane-node table of
    # the gridding kernel holds 4 passes of 64 nodes
    p = sog.plan_parameters((24.0, 24.0, 12.0), 400, tol, "fp64")
    if p["m"] >= 0:
        assert p["mid_Pw"][0] <= 15
    if p["m"] < p["M"] and p["long_form"] == _lib.SOG_LONG_FFT:
        assert p["long_Pw"][0] <= 15


def test_window_choice():
    """AUTO takes a compact window where it is cheaper (the 10^6 cube: KB, which wins the
    tie with ES), the Gaussian when its shape is given; each explicit choice is honoured and
    reported with its shape."""
    box, n = (100.0, 100.0, 100.0), 1000000
    auto = sog.plan_parameters(box, n, 1e-4, "fp32")
    assert auto["mid_window"] == _lib.SOG_WINDOW_KB and auto["mid_beta"] > 0 and auto["mid_S"] == 0
    g = sog.plan_parameters(box, n, 1e-4, "fp32", dict(mid_window=_lib.SOG_WINDOW_GAUSSIAN))
    assert g["mid_window"] == _lib.SOG_WINDOW_GAUSSIAN and g["mid_S"] > 0 and g["mid_beta"] == 0
    assert auto["mid_Pw"][0] < g["mid_Pw"][0]  # the compact window needs fewer points
    gs = sog.plan_parameters(box, n, 1e-4, "fp32", dict(mid_S=12.0))
    assert gs["mid_window"] == _lib.SOG_WINDOW_GAUSSIAN and gs["mid_S"] == 12.0
    es = sog.plan_parameters((20, 20, 20), 1000, 1e-6, "fp64",
                             dict(mid_window=_lib.SOG_WINDOW_ES, mid_Pw=[9, 9, 9], mid_beta=19.0))
    assert es["mid_window"] == _lib.SOG_WINDOW_ES and es["mid_Pw"] == [9, 9, 9] and es["mid_beta"] == 19.0
    # a forced window keeps its shape even where the planner would not pick it (a coarse
    # grid on which its deconvolution grows at the band edge)
    t = sog.plan_parameters((10, 10, 60), 1200, 1e-6, "fp64",
                            dict(mid_window=_lib.SOG_WINDOW_ES, mid_I=[20, 20, 120], mid_Izs=252, mid_Pw=[9, 9, 9],
                                 mid_beta=19.8))
    assert t["mid_beta"] == 19.8
    t = sog.plan_parameters((10, 10, 60), 1200, 1e-6, "fp64",
                            dict(mid_window=_lib.SOG_WINDOW_ES, mid_I=[20, 20, 120], mid_Izs=252, mid_Pw=[9, 9, 9]))
    assert t["mid_beta"] > 0


def test_kb_window_plans():
    """The KB window: the same support as ES on the 10^6 cube (their aliasing is alike),
    the polynomial degree chosen from the tolerance (higher for a tighter one) or taken as
    given; AUTO takes KB on the tie."""
    box, n = (100.0, 100.0, 100.0), 1000000
    es = sog.plan_parameters(box, n, 1e-4, "fp32", dict(mid_window=_lib.SOG_WINDOW_ES))
    kb = sog.plan_parameters(box, n, 1e-4, "fp32", dict(mid_window=_lib.SOG_WINDOW_KB))
    assert kb["mid_window"] == _lib.SOG_WINDOW_KB and kb["mid_beta"] > 0 and kb["mid_S"] == 0
    assert abs(kb["mid_Pw"][0] - es["mid_Pw"][0]) <= 2 and 4 <= kb["mid_nu"] <= 16
    assert es["mid_window"] == _lib.SOG_WINDOW_ES and es["mid_nu"] == 0
    assert sog.plan_parameters(box, n, 1e-4, "fp32") == kb
    tight = sog.plan_parameters((20, 20, 20), 1000, 1e-10, "fp64", dict(mid_window=_lib.SOG_WINDOW_KB))
    assert tight["mid_window"] == _lib.SOG_WINDOW_KB and tight["mid_nu"] > kb["mid_nu"]
    given = sog.plan_parameters((20, 20, 20), 1000, 1e-6, "fp64",
                                dict(mid_window=_lib.SOG_WINDOW_KB, mid_Pw=[9, 9, 9], mid_beta=20.0, mid_nu=10))
    assert (given["mid_Pw"], given["mid_beta"], given["mid_nu"]) == ([9, 9, 9], 20.0, 10)


@pytest.mark.parametrize("case, status", [
    ("no_systems", _lib.SOG_ERR_INVALID_ARG),
    ("one_particle", _lib.SOG_ERR_INVALID_ARG),
    ("timing", _lib.SOG_ERR_INVALID_ARG),
    ("bad_tol", _lib.SOG_ERR_TOL_UNREACHABLE),
    ("bad_box", _lib.SOG_ERR_INVALID_ARG),
])
def test_batch_plan_rejects_bad_arguments(case, status):
    """sog_batch_plan checks its arguments and resolves every system before it touches a
    device, so each rejection is reached on a machine without a GPU; the message names the
    failing system."""
    boxes = [(10.0, 10.0, 10.0), (8.0, 8.0, 64.0), (20.0, 20.0, 2.5)]
    ns = [1000, 4000, 1000]
    tol = 1e-4
    opt = sog.make_options("fp32")
    if case == "no_systems":
        boxes, ns = [], []
    elif case == "one_particle":
        ns[1] = 1
    elif case == "timing":
        opt.timing = 1
    elif case == "bad_tol":
        tol = 1e-9  # below the float32 range
    elif case == "bad_box":
        boxes[2] = (20.0, -1.0, 2.5)
    with pytest.raises(sog.SogError) as ei:
        sog.sog_batch_plan(boxes, ns, tol, opt)
    assert ei.value.status == status
    if case in ("one_particle", "bad_box"):
        assert "system 1" in str(ei.value) or "system 2" in str(ei.value)


def test_batch_workload_plans():
    """Every system of the 256-system batch (N log-uniform in [500, 20000], Lz/Lx in
    {1/8, 1, 8}, density 1) has a float32 plan at tol 1e-4 with the structure every plan
    needs, and the batch totals about 1.3 million particles."""
    import workloads
    specs = workloads.batch_specs()
    assert len(specs) == 256
    total = 0
    for N, box, _seed in specs:
        assert 500 <= N <= 20000 and N % 2 == 0
        p = sog.plan_parameters(box, N, 1e-4, "fp32")
        assert p["rc"] <= min(box[0], box[1]) / 2 + 1e-12
        assert p["m"] <= p["M"]
        if p["m"] >= 0:
            # periodic x, y and the padded z extent each hold at least two windows
            sizes = (p["mid_I"][0], p["mid_I"][1], p["mid_Izs"])
            assert all(I >= 2 * pw for I, pw in zip(sizes, p["mid_Pw"]))
        total += N
    assert 1.0e6 < total < 2.0e6
    assert {round(b[2] / b[0], 3) for _n, b, _s in specs} == {0.125, 1.0, 8.0}


@pytest.mark.parametrize("name, prec, cap", [("cube_8e6", "fp32", 4608), ("cube_1e6", "fp64", 2304),
                                             ("cube_1e6", "fp32", 4608)])
def test_planner_keeps_fft_batches_wide(name, prec, cap):
    """The planner charges x/y line lengths that leave the FFT line kernels fewer than 8
    lines per batch (short row segments): on the cubes it picks grids whose x and y lines
    allow at least 8 (I <= cap / 8; the kernels batch n W <= cap elements)."""
    import workloads
    N, box = workloads.NAMED[name]
    p = sog.plan_parameters(box, N, 1e-4, prec)
    assert max(p["mid_I"][0], p["mid_I"][1]) * 8 <= cap


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("box", [(953.5, 953.5, 0.3), (400.0, 400.0, 2.0), (300.0, 300.0, 1.0)])
def test_strongly_confined_boxes_plan_all_long_fft(box, prec):
    """Strongly confined boxes (Table 4's 953.5 x 953.5 x 0.3 at surface density 1.1, and
    Lx/Lz = 200, 300) need the long range's FFT form (the direct form would need millions of
    modes); in Table 4's box every Gaussian is long range (s_0 > 2 L_z, the Remark after the
    range-splitting definition).  The plan's grid holds whole windows and has far more tiles
    than compute units."""
    p = sog.plan_parameters(box, 10**6, 1e-4, prec)
    assert p["long_form"] == _lib.SOG_LONG_FFT
    if box[2] < 0.5:
        assert p["m"] == -1  # s_0 > 2 L_z: nothing is left for the mid range
    I = p["long_I"]
    assert min(I) >= 2 * p["long_Pw"][0] and I[1] % 2 == 0
    assert (I[0] // 16) * (I[1] // 16) >= 1024
    assert p["long_Q"] == -1 or p["long_Q"] > 0


def test_unreachable_plans_name_the_limit():
    """A box the kernels cannot discretise at the tolerance returns SOG_ERR_TOL_UNREACHABLE
    with the binding limit in the message (not SOG_ERR_INVALID_ARG)."""
    with pytest.raises(sog.SogError) as ei:
        sog.plan_parameters((953.5, 953.5, 0.3), 10**6, 1e-4, "fp32", params=dict(long_form="direct"))
    assert ei.value.status == _lib.SOG_ERR_TOL_UNREACHABLE and "65536" in str(ei.value)
    with pytest.raises(sog.SogError) as ei:
        sog.plan_parameters((953.5, 953.5, 0.3), 10**6, 1e-4, "fp32", params=dict(long_form="fft", long_Pw=[3, 3],
                                                                                    long_I=[5000, 5000]))
    assert ei.value.status in (_lib.SOG_ERR_TOL_UNREACHABLE, _lib.SOG_ERR_INVALID_ARG)


def test_direct_form_limited_by_the_moments_lds():
    """The direct long range's moments kernel holds a batch of at least 16 particles' plane
    waves (2 n_kx + 1 + n_ky + 1 rows) in LDS: 129 + 65 rows fit in float32, not in float64,
    where a forced direct form is refused naming the limit and the automatic choice is the
    FFT form."""
    from tests._cases import gpu_params
    params = gpu_params(dict(row=3, rc=2.5, M=120, m=-1, mid=None, long=dict(form="direct", P=4, nk=(64, 64))))
    box = (40.0, 40.0, 4.0)
    p = sog.plan_parameters(box, 600, 1e-4, "fp32", params=params)
    assert p["long_form"] == 1 and list(p["long_nk"]) == [64, 64]
    with pytest.raises(sog.SogError) as ei:
        sog.plan_parameters(box, 600, 1e-6, "fp64", params=params)
    assert ei.value.status == _lib.SOG_ERR_TOL_UNREACHABLE and "LDS" in str(ei.value)
    auto = {k: v for k, v in params.items() if not k.startswith("long_")}
    assert sog.plan_parameters(box, 600, 1e-6, "fp64", params=auto)["long_form"] == 2
    # 121 + 41 rows still fit in float64, unpadded
    p = sog.plan_parameters((24.0, 20.0, 4.0), 400, 1e-6, "fp64", params=dict(params, long_nk=[60, 40]))
    assert p["long_form"] == 1 and list(p["long_nk"]) == [60, 40]


def test_taylor_form_is_planned_on_request():
    """long_Q > 0 asks for App. C's Taylor form of the z kernel (2Q - 1 source planes, at most
    2Q - 1 target terms); long_Q = -1 for the exact kernel; both plan on the Table 4 box."""
    box = (953.5, 953.5, 0.3)
    t = sog.plan_parameters(box, 10**6, 1e-4, "fp32", params=dict(long_form="fft", long_Q=4))
    e = sog.plan_parameters(box, 10**6, 1e-4, "fp32", params=dict(long_form="fft", long_Q=-1))
    assert t["long_Q"] == 4 and t["long_P"] <= 7
    assert e["long_Q"] == -1
    with pytest.raises(sog.SogError) as ei:
        sog.plan_parameters(box, 10**6, 1e-4, "fp32", params=dict(long_Q=17))
    assert ei.value.status == _lib.SOG_ERR_INVALID_ARG
