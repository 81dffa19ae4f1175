"""Write the sampled-target reference values for the full-size workloads.

Calls only oracle/ (SOG-direct: the exact value of the SOG decomposition, pinned
against Ewald2D in tests/test_oracle_pins.py) and the seeded generators in
workloads/.  Decomposition: Table 1 row b = 1.2181 (printed errors 7e-10 / 5e-10),
r_c = 3 rho^{-1/3}, M from the omitted-tail bound; the values are therefore the
potentials and gradients of the quasi-2D Coulomb sum itself to ~1e-9 relative.

Usage: python tests/golden/make_golden.py [name ...]   (default: every workload)
Output: tests/golden/<name>_targets.txt.  Also, by name: cube_small_ewald2d (Ewald2D on
every particle of the 1000-particle cube) and <workload>_energy (the workload's energy from
the plain fast method at two tolerances, tests/golden/<workload>_energy.txt).
"""
import math
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.direct import sog_direct  # noqa: E402
from oracle.sog import SOG, TABLE1  # noqa: E402
import workloads  # noqa: E402

NTARGETS = 24
# the benchmark's workload gets about a hundred targets
NTARGETS_BY_NAME = {"cube_1e6": 100}
ROW = 4  # b = 1.21812525709410644


def decomposition(N, box):
    Lx, Ly, Lz = box
    b, r0, om = TABLE1[ROW][:3]
    rho = N / (Lx * Ly * Lz)
    rc = min(3.0 * rho ** (-1 / 3), 0.5 * min(Lx, Ly))
    sigma = rc / r0
    # omitted wide Gaussians leave (pi/A) sum_{l>M} w_l sum_j q_j z_ij^2; keep below 1e-13
    wl1 = math.sqrt(2 / math.pi) * math.log(b) / sigma
    rhs = 1e-13 * Lx * Ly / (math.pi * N * Lz * Lz) * (1 - 1 / b) / wl1
    M = int(math.ceil(-math.log(rhs) / math.log(b)))
    return b, r0, om, rc, M


_CTX = {}


def _init(name):
    x, q, box = workloads.named(name)
    b, r0, om, rc, M = decomposition(len(q), box)
    _CTX.update(x=x, q=q, box=box, sog=SOG(b, r0, om, rc, M))


def _one(i):
    c = _CTX
    o = sog_direct(c["x"], c["q"], c["box"], c["sog"], m=c["sog"].M, targets=np.array([i]))
    return i, float(o["phi"][0]), o["grad"][0].tolist()


def make(name, procs=8):
    x, q, box = workloads.named(name)
    N = len(q)
    rng = np.random.default_rng(12345)
    # fewer targets for the 8-million cube: each costs about four minutes of one core
    targets = np.sort(rng.choice(N, 8 if N > 4_000_000 else NTARGETS_BY_NAME.get(name, NTARGETS), replace=False))
    b, r0, om, rc, M = decomposition(N, box)
    t0 = time.time()
    with Pool(procs, initializer=_init, initargs=(name,)) as pool:
        rows = pool.map(_one, targets.tolist())
    path = os.path.join(HERE, f"{name}_targets.txt")
    with open(path, "w") as f:
        f.write(f"# Reference potentials and gradients of sampled particles of workload {name}\n")
        f.write(f"# (N={N}, box={box}, seed={workloads.NAMED_SEED[name]}), written by tests/golden/make_golden.py\n")
        f.write("# with oracle.direct.sog_direct: exact SOG decomposition, Table 1 row\n")
        f.write(f"# b={b!r} r0={r0!r} omega={om!r}, r_c={rc!r}, M={M}.\n")
        f.write("# columns: index phi dphi/dx dphi/dy dphi/dz\n")
        for i, phi, g in rows:
            f.write(f"{i} {phi:.17g} {g[0]:.17g} {g[1]:.17g} {g[2]:.17g}\n")
    print(f"{name}: {len(rows)} targets in {time.time() - t0:.0f} s -> {path}", flush=True)


BATCH_TARGETS = 4


def _init_batch(s):
    N, box, seed = workloads.batch_specs()[s]
    x, q = workloads.uniform(N, box, seed)
    b, r0, om, rc, M = decomposition(N, box)
    _CTX.update(x=x, q=q, box=box, sog=SOG(b, r0, om, rc, M))


def _batch_rows(s):
    N, box, seed = workloads.batch_specs()[s]
    _init_batch(s)
    rng = np.random.default_rng(1000 + s)
    targets = np.sort(rng.choice(N, BATCH_TARGETS, replace=False))
    b, r0, om, rc, M = decomposition(N, box)
    return [(s, *_one(int(i))) for i in targets], (b, r0, om, rc, M)


def make_batch(procs=8):
    """Sampled targets of the systems workloads.BATCH_CHECKED of the 256-system batch,
    each system with its own Table 1 decomposition (row 4, r_c from its density)."""
    t0 = time.time()
    with Pool(procs) as pool:
        res = pool.map(_batch_rows, list(workloads.BATCH_CHECKED))
    path = os.path.join(HERE, "batch_256_targets.txt")
    with open(path, "w") as f:
        f.write("# Reference potentials and gradients of sampled particles of systems of the 256-system batch\n")
        f.write("# (workloads.batch_specs(): N log-uniform in [500, 20000], Lz/Lx in {1/8, 1, 8}, density 1,\n")
        f.write("# uniform positions, +/-1 charges), written by tests/golden/make_golden.py with\n")
        f.write("# oracle.direct.sog_direct: exact SOG decomposition per system, Table 1 row 4\n")
        f.write(f"# (b={TABLE1[ROW][0]!r}), r_c = min(3 rho^(-1/3), min(Lx, Ly)/2), M from the omitted-tail bound.\n")
        f.write("# columns: system index-in-system phi dphi/dx dphi/dy dphi/dz\n")
        for rows, _dec in res:
            for s, i, phi, g in rows:
                f.write(f"{s} {i} {phi:.17g} {g[0]:.17g} {g[1]:.17g} {g[2]:.17g}\n")
    print(f"batch_256: {sum(len(r) for r, _ in res)} targets in {time.time() - t0:.0f} s -> {path}", flush=True)


def make_cube_small_ewald2d():
    """Ewald2D (oracle.ewald2d, alpha-independent, pinned against brute-force image sums)
    on every particle of the 1000-particle cube of Sec. 5.1 (20^3, seed 1): the energy
    and each particle's potential and gradient."""
    from oracle import ewald2d as ew
    x, q, box = workloads.named("cube_small")
    t0 = time.time()
    o = ew.ewald2d(x, q, box)
    U = ew.energy(q, o["phi"])
    path = os.path.join(HERE, "cube_small_ewald2d.txt")
    with open(path, "w") as f:
        f.write("# Ewald2D potentials and gradients of every particle of workload cube_small\n")
        f.write(f"# (N={len(q)}, box={box}, seed={workloads.NAMED_SEED['cube_small']}), written by\n")
        f.write("# tests/golden/make_golden.py cube_small_ewald2d with oracle.ewald2d.ewald2d (default alpha).\n")
        f.write(f"# U {U:.17g}\n")
        f.write("# columns: index phi dphi/dx dphi/dy dphi/dz\n")
        for i in range(len(q)):
            g = o["grad"][i]
            f.write(f"{i} {o['phi'][i]:.17g} {g[0]:.17g} {g[1]:.17g} {g[2]:.17g}\n")
    print(f"cube_small_ewald2d: U={U!r} in {time.time() - t0:.0f} s -> {path}", flush=True)


# The energy reference of a full-size workload: the plain fast method of oracle.fast at two
# tolerances, with the oracle's own parameter choice.  The energy's relative error is the
# potentials' error amplified by the cancellation in U = 1/2 sum q_i phi_i (|U| is ~40x
# below sum |q_i phi_i| for uniform +/-1 charges), so the two runs must agree to 1e-7; the
# tighter run is kept as the reference.
ENERGY_TOLS = (1e-8, 1e-10)
ENERGY_AGREE = 1e-7


def make_energy(name):
    from oracle import fast, planner
    x, q, box = workloads.named(name)
    N = len(q)
    res = []
    for tol in ENERGY_TOLS:
        p = planner.plan(box, N, tol)
        tm = {}
        t0 = time.time()
        o = fast.solve(x, q, box, p, times=tm)
        res.append((tol, o["U"], time.time() - t0, tm, p))
        print(f"{name}: tol {tol:g} U={o['U']!r} in {time.time() - t0:.0f} s {tm}", flush=True)
        del o
    (t1, U1, s1, _, p1), (t2, U2, s2, _, p2) = res
    agree = abs(U1 - U2) / abs(U2)
    if agree > ENERGY_AGREE:
        raise SystemExit(f"{name}: the two oracle runs disagree by {agree:.2e} > {ENERGY_AGREE:g}; nothing written")
    path = os.path.join(HERE, f"{name}_energy.txt")
    with open(path, "w") as f:
        f.write(f"# Reference energy of workload {name} (N={N}, box={box}, seed={workloads.NAMED_SEED[name]}),\n")
        f.write(f"# written by tests/golden/make_golden.py {name}_energy: oracle.fast.solve with\n")
        f.write("# oracle.planner.plan parameters at two tolerances; the tighter run is the reference.\n")
        for tol, U, sec, tm, p in res:
            f.write(f"# tol {tol:g}: U={U!r}, {sec:.0f} s (near {tm['short']:.0f}, mid {tm['mid']:.0f}, "
                    f"long {tm['long']:.0f}); b={p['sog']['b']!r} r_c={p['sog']['rc']!r} M={p['sog']['M']} "
                    f"m={p['m']} mid={p['mid']} long={p['long']}\n")
        f.write(f"# relative difference of the two energies: {agree:.3e}\n")
        f.write(f"U {U2:.17g}\n")
        f.write(f"U_loose {U1:.17g}\n")
    print(f"{name}_energy: U={U2!r} (agreement {agree:.2e}) -> {path}", flush=True)


def load_energy(name):
    """The reference energy from tests/golden/<name>_energy.txt, or None."""
    path = os.path.join(HERE, f"{name}_energy.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split()
        if f and f[0] == "U":
            return float(f[1])
    return None


def load(name):
    """(indices, phi, grad) from tests/golden/<name>_targets.txt"""
    d = np.loadtxt(os.path.join(HERE, f"{name}_targets.txt"), comments="#")
    return d[:, 0].astype(np.int64), d[:, 1], d[:, 2:5]


if __name__ == "__main__":
    names = sys.argv[1:] or ["cube_1e6", "slab_1e6", "tall_1e6", "layered_2e5", "batch_256"]
    for n in names:
        if n == "batch_256":
            make_batch()
        elif n == "cube_small_ewald2d":
            make_cube_small_ewald2d()
        elif n.endswith("_energy"):
            make_energy(n[: -len("_energy")])
        else:
            make(n)
