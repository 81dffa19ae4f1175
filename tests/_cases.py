"""Explicit parameter sets shared by the GPU parity tests: the same dict configures the
HIP plan (sog_params overrides) and the oracle (oracle.fast.make_params).  Nothing here
is computed by the HIP library."""
import math

TABLE1_ROWS = {
    3: (1.32070036405934420, 4.3914554711638349, 1.0018891411481198),
    4: (1.21812525709410644, 5.6355288151271085, 1.0009014615603334),
}

# name: N, box, seed, decomposition row, r_c, M, m, mid (I, I_z*, P_w), long
CASES = {
    # the Sec. 5.1 box; several 16^3 tiles, mid + direct long range
    "cube_small": dict(N=1000, box=(20.0, 20.0, 20.0), seed=1, row=3, rc=4.0, M=100, m=6,
                       mid=dict(I=(32, 32, 32), Izs=80, Pw=9), long=dict(form="direct", P=12, nk=(4, 4))),
    # non-cubic box, grid sizes that are not multiples of the tile (ragged tiles), P_w = 7
    "ragged": dict(N=2000, box=(13.0, 17.0, 9.0), seed=7, row=3, rc=3.0, M=120, m=5,
                   mid=dict(I=(30, 40, 24), Izs=64, Pw=7), long=dict(form="direct", P=10, nk=(3, 4))),
    # direct long range over 4901 half-plane modes: the moments kernel's float64 LDS rows
    # unpadded (padded ones would not fit)
    "wide_direct": dict(N=400, box=(24.0, 20.0, 4.0), seed=17, row=3, rc=2.5, M=120, m=-1,
                        mid=None, long=dict(form="direct", P=4, nk=(60, 40))),
    # direct long range with more Chebyshev terms than the register evaluation takes (40 in
    # float32, 16 in float64), the coefficient table too large to stage in LDS (841 modes x
    # 44) and small enough (8 modes x 44)
    "deep_direct": dict(N=400, box=(24.0, 20.0, 6.0), seed=18, row=3, rc=2.5, M=120, m=-1,
                        mid=None, long=dict(form="direct", P=44, nk=(20, 20))),
    "deep_narrow": dict(N=400, box=(24.0, 20.0, 6.0), seed=19, row=3, rc=2.5, M=120, m=-1,
                        mid=None, long=dict(form="direct", P=44, nk=(2, 1))),
    # flat slab, every Gaussian long range (Remark after the range-splitting definition),
    # Fourier-Chebyshev solver with 2D FFTs
    "slab_all_long_fft": dict(N=1500, box=(24.0, 20.0, 4.0), seed=8, row=3, rc=2.5, M=120, m=-1,
                              mid=None, long=dict(form="fft", P=24, I=(72, 60), Pw=9)),
    # mid range plus the FFT form of the long range
    "slab_mid_fft": dict(N=2400, box=(30.0, 30.0, 6.0), seed=12, row=3, rc=3.0, M=120, m=3,
                         mid=dict(I=(50, 50, 10), Izs=40, Pw=9), long=dict(form="fft", P=14, I=(40, 40), Pw=9)),
    # strongly confined (Table 4's surface density 1.1 and L_z = 0.3, Lx/Lz = 133): every
    # Gaussian long range, FFT form with the exact z kernel, and with App. C's Taylor form
    # (Q = 4: 7 source planes, 5 target terms; Q = 6: two 8-plane passes of the gridding);
    # grids that are not multiples of the 16-node tile, window 15 (half-width 7)
    "confined_exact": dict(N=1760, box=(40.0, 40.0, 0.3), seed=41, row=3, rc=3.0, M=90, m=-1,
                           mid=None, long=dict(form="fft", P=6, Q=-1, I=(90, 84), Pw=11)),
    "confined_taylor": dict(N=1760, box=(40.0, 40.0, 0.3), seed=41, row=3, rc=3.0, M=90, m=-1,
                            mid=None, long=dict(form="fft", P=5, Q=4, I=(90, 84), Pw=11)),
    "confined_taylor6": dict(N=1500, box=(36.0, 30.0, 0.6), seed=42, row=4, rc=3.0, M=180, m=-1,
                             mid=None, long=dict(form="fft", P=9, Q=6, I=(70, 60), Pw=15)),
    # a long grid of 2 x 2 tiles (every tile's windows reach all tiles), Taylor form
    "confined_small": dict(N=600, box=(18.0, 15.0, 0.5), seed=43, row=3, rc=3.0, M=90, m=-1,
                           mid=None, long=dict(form="fft", P=6, Q=5, I=(24, 20), Pw=9)),
    # tall cell: long z lines in the FFT, many Chebyshev terms
    "tall": dict(N=1200, box=(10.0, 10.0, 60.0), seed=13, row=3, rc=3.0, M=140, m=8,
                 mid=dict(I=(20, 20, 120), Izs=252, Pw=9), long=dict(form="direct", P=20, nk=(1, 1))),
    # clustered input in a tall box (workloads.clustered): cells holding hundreds of
    # particles next to long runs of nearly empty cells, several z frames of the near
    # field's coordinates
    "clustered": dict(N=3000, box=(12.0, 12.0, 48.0), seed=15, row=3, rc=3.0, M=140, m=8, gen="clustered",
                      mid=dict(I=(24, 24, 96), Izs=200, Pw=9), long=dict(form="direct", P=20, nk=(1, 1))),
    # one cell of 1149 particles (a cluster centred inside a cell): too many to sort by z,
    # so the near field's range bisection is switched off for the call
    "dense_cluster": dict(N=3000, box=(10.5, 10.5, 45.0), seed=16, row=3, rc=3.0, M=140, m=8, gen="clustered",
                          gen_args=dict(frac=0.4, sd=0.7),
                          mid=dict(I=(24, 24, 90), Izs=200, Pw=9), long=dict(form="direct", P=20, nk=(1, 1))),
    # the ES window (sog_window ES, oracle window="es"): the cube with P_w = 7 and a tall
    # box (z frames, long z lines) with P_w = 9
    "cube_es": dict(N=1000, box=(20.0, 20.0, 20.0), seed=1, row=3, rc=4.0, M=100, m=6,
                    mid=dict(I=(32, 32, 32), Izs=80, Pw=7, window="es", beta=16.1),
                    long=dict(form="direct", P=12, nk=(4, 4))),
    "tall_es": dict(N=1200, box=(10.0, 10.0, 60.0), seed=13, row=3, rc=3.0, M=140, m=8,
                    mid=dict(I=(20, 20, 120), Izs=252, Pw=9, window="es", beta=19.8),
                    long=dict(form="direct", P=20, nk=(1, 1))),
    # the KB window by its polynomials (sog_window KB, oracle window="kb" with nu): the
    # cube with P_w = 7 and the Sec. 5.1 degree nu = 10, the tall box with P_w = 9 and
    # nu = 8, and the widest window with nu = 12
    "cube_kb": dict(N=1000, box=(20.0, 20.0, 20.0), seed=1, row=3, rc=4.0, M=100, m=6,
                    mid=dict(I=(32, 32, 32), Izs=80, Pw=7, window="kb", beta=16.1, nu=10),
                    long=dict(form="direct", P=12, nk=(4, 4))),
    "tall_kb": dict(N=1200, box=(10.0, 10.0, 60.0), seed=13, row=3, rc=3.0, M=140, m=8,
                    mid=dict(I=(20, 20, 120), Izs=252, Pw=9, window="kb", beta=20.7, nu=8),
                    long=dict(form="direct", P=20, nk=(1, 1))),
    "pw15_kb": dict(N=1200, box=(18.0, 22.0, 14.0), seed=35, row=4, rc=5.0, M=170, m=8,
                    mid=dict(I=(40, 48, 30), Izs=96, Pw=15, window="kb", beta=34.5, nu=12),
                    long=dict(form="direct", P=16, nk=(2, 3))),
    # window 13 and odd-radix FFT lengths (3, 5, 7)
    "radix_mix": dict(N=900, box=(21.0, 15.0, 10.0), seed=14, row=4, rc=3.5, M=200, m=5,
                      mid=dict(I=(42, 30, 20), Izs=70, Pw=13), long=dict(form="direct", P=14, nk=(3, 2))),
    # every other window width the gridding and gathering kernels are built for: 3, 5, 11
    # and 15 points, Gaussian and ES (11 with ES is the planner's choice for the Sec. 5.1
    # box at tol 1e-6)
    "pw3": dict(N=800, box=(16.0, 16.0, 12.0), seed=31, row=3, rc=3.5, M=100, m=5,
                mid=dict(I=(40, 40, 30), Izs=80, Pw=3), long=dict(form="direct", P=12, nk=(3, 3))),
    "pw5_es": dict(N=800, box=(16.0, 16.0, 12.0), seed=32, row=3, rc=3.5, M=100, m=5,
                   mid=dict(I=(40, 40, 30), Izs=80, Pw=5, window="es", beta=11.5),
                   long=dict(form="direct", P=12, nk=(3, 3))),
    "pw11": dict(N=1000, box=(20.0, 20.0, 20.0), seed=1, row=4, rc=6.0, M=166, m=8,
                 mid=dict(I=(36, 36, 36), Izs=108, Pw=11), long=dict(form="direct", P=16, nk=(2, 2))),
    "pw11_es": dict(N=1000, box=(20.0, 20.0, 20.0), seed=1, row=4, rc=6.0, M=166, m=8,
                    mid=dict(I=(36, 36, 36), Izs=108, Pw=11, window="es", beta=22.0),
                    long=dict(form="direct", P=16, nk=(2, 2))),
    "pw15": dict(N=1200, box=(18.0, 22.0, 14.0), seed=33, row=4, rc=5.0, M=170, m=8,
                 mid=dict(I=(40, 48, 30), Izs=96, Pw=15), long=dict(form="direct", P=16, nk=(2, 3))),
    "pw15_es": dict(N=1200, box=(18.0, 22.0, 14.0), seed=34, row=4, rc=5.0, M=170, m=8,
                    mid=dict(I=(40, 48, 30), Izs=96, Pw=15, window="es", beta=33.0),
                    long=dict(form="direct", P=16, nk=(2, 3))),
}


def _window_S(Pw):
    # the shape used with a P_w-point Gaussian window in the paper's experiments (Sec. 5.1)
    return 0.455 * math.pi * Pw


def gpu_params(c):
    b, r0, om = TABLE1_ROWS[c["row"]]
    p = dict(b=b, r0=r0, omega=om, rc=c["rc"], M=c["M"], m=c["m"], set_m=1)
    if c["mid"]:
        p.update(mid_I=list(c["mid"]["I"]), mid_Izs=c["mid"]["Izs"], mid_Pw=[c["mid"]["Pw"]] * 3)
        if c["mid"].get("window") == "es":
            p.update(mid_window=2, mid_beta=c["mid"]["beta"])
        elif c["mid"].get("window") == "kb":
            p.update(mid_window=3, mid_beta=c["mid"]["beta"], mid_nu=c["mid"]["nu"])
        else:
            p.update(mid_window=1, mid_S=_window_S(c["mid"]["Pw"]))
    lp = c["long"]
    if lp:
        p.update(long_form=lp["form"], long_P=lp["P"])
        if lp["form"] == "direct":
            p.update(long_nk=list(lp["nk"]))
        else:
            p.update(long_I=list(lp["I"]), long_Pw=[lp["Pw"]] * 2, long_S=_window_S(lp["Pw"]),
                     long_Q=lp.get("Q", -1))
    return p


def oracle_params(c):
    from oracle import fast
    b, r0, om = TABLE1_ROWS[c["row"]]
    mid = None
    if c["mid"]:
        Pw = c["mid"]["Pw"]
        mid = dict(I=tuple(c["mid"]["I"]), Izs=c["mid"]["Izs"], Pw=(Pw, Pw, Pw), S=_window_S(Pw))
        if c["mid"].get("window") == "es":
            mid.update(window="es", beta=c["mid"]["beta"])
        elif c["mid"].get("window") == "kb":
            mid.update(window="kb", beta=c["mid"]["beta"], nu=c["mid"]["nu"])
    lp = dict(c["long"]) if c["long"] else None
    if lp and lp["form"] == "fft":
        lp = dict(form="fft", P=lp["P"], I=tuple(lp["I"]), Pw=(lp["Pw"], lp["Pw"]), S=_window_S(lp["Pw"]),
                  Q=max(0, lp.get("Q", 0)))
    return fast.make_params(b, r0, om, c["rc"], c["M"], c["m"], mid=mid, long=lp)


def oracle_params_from_info(info):
    """The oracle's parameter dict for a plan the library resolved (sog_params as a dict):
    the same decomposition, split, grids, windows and long-range form."""
    from oracle import fast
    mid = None
    if info["m"] >= 0:
        Pw = info["mid_Pw"][0]
        mid = dict(I=tuple(info["mid_I"]), Izs=info["mid_Izs"], Pw=(Pw, Pw, Pw), S=info["mid_S"])
        if info["mid_window"] == 2:
            mid.update(window="es", beta=info["mid_beta"])
        elif info["mid_window"] == 3:
            mid.update(window="kb", beta=info["mid_beta"], nu=info["mid_nu"])
    lp = None
    if info["m"] < info["M"]:
        if info["long_form"] == 1:
            lp = dict(form="direct", P=info["long_P"], nk=tuple(info["long_nk"]))
        else:
            lp = dict(form="fft", P=info["long_P"], I=tuple(info["long_I"]), Pw=tuple(info["long_Pw"]),
                      S=info["long_S"], Q=max(0, info["long_Q"]))
    return fast.make_params(info["b"], info["r0"], info["omega"], info["rc"], info["M"], info["m"], mid=mid, long=lp)
