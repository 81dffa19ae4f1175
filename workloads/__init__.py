"""Seeded synthetic particle sets for the SOG solver's tests and benchmark.

This module holds no arithmetic of the method: it only draws positions and
charges.  Both the HIP path's tests/benchmark and the CPU oracle's tests take
their inputs from here, so that the two sides see identical inputs.

Conventions: positions in [0,Lx) x [0,Ly) x [0,Lz] (x,y periodic, z free),
float64 arrays of shape (N,3); charges float64 (N,), +/-1 with exactly half of
each sign (charge neutral, as the problem statement requires).

Workloads (the paper's experiments use uniform random monovalent particles,
Sec. 5; the layered set stands in for an electrolyte between two interfaces; the
confined set has the size and shape of the strongly confined runs of Sec. 5.2, Table 4):

* ``uniform(N, box, seed)``
* ``layered(N, box, seed, ...)``: x,y uniform; half of the particles have z drawn
  from N(z1, sd^2), half from N(z2, sd^2), each redrawn until it lies in [0,Lz];
  the lower layer holds a fraction ``enrich`` of positive charges, the upper
  layer the complement, so the cell is neutral with a large z dipole.
* ``batch_specs(n_systems, seed, ...)``: N_s log-uniform in [Nmin, Nmax] (even),
  aspect Lz/Lx from {1/8, 1, 8}, density 1.
* ``clustered(N, box, seed, ...)``: a fraction ``frac`` of the particles in a Gaussian
  cluster (standard deviation ``sd`` in each direction, z redrawn into [0, L_z], x and y
  wrapped) about the box centre; of the rest, a fraction ``top`` uniform in the upper
  half of the box and the others uniform in the lower half.  Dense cells next to long
  runs of nearly empty ones, for the near field's work division.
"""
import numpy as np

NAMED = {
    # name: (N, box) -- the configurations the solver is measured and checked on
    "cube_small": (1000, (20.0, 20.0, 20.0)),
    "cube_1e6": (1_000_000, (100.0, 100.0, 100.0)),
    "slab_1e6": (1_000_000, (400.0, 400.0, 25.0)),
    "tall_1e6": (1_000_000, (50.0, 50.0, 800.0)),
    "layered_2e5": (200_000, (150.0, 150.0, 60.0)),
    "cube_8e6": (8_000_000, (200.0, 200.0, 200.0)),
    # strongly confined: Table 4's box, surface density N/(Lx Ly) = 1.1 at L_z = 0.3
    "confined_1e6": (1_000_000, (953.5, 953.5, 0.3)),
}
NAMED_SEED = {"cube_small": 1, "cube_1e6": 2, "slab_1e6": 3, "tall_1e6": 4, "layered_2e5": 6, "cube_8e6": 7,
              "confined_1e6": 8}


def _charges(rng, N):
    if N % 2:
        raise ValueError("N must be even for an exactly neutral +/-1 system")
    q = np.ones(N)
    q[N // 2:] = -1.0
    rng.shuffle(q)
    return q


def uniform(N, box, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((N, 3)) * np.asarray(box, dtype=np.float64)
    return x, _charges(rng, N)


def layered(N, box, seed, z1=5.0, z2=55.0, sd=3.0, enrich=0.6):
    if N % 4:
        raise ValueError("N must be a multiple of 4")
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz = box
    x = np.empty((N, 3))
    x[:, 0] = rng.random(N) * Lx
    x[:, 1] = rng.random(N) * Ly
    half = N // 2

    def draw(center, n):
        z = np.empty(n)
        todo = np.arange(n)
        while todo.size:
            z[todo] = rng.normal(center, sd, todo.size)
            todo = todo[(z[todo] < 0.0) | (z[todo] > Lz)]
        return z

    x[:half, 2] = draw(z1, half)
    x[half:, 2] = draw(z2, N - half)
    n_pos_low = int(round(enrich * half))
    q = np.empty(N)
    ql = -np.ones(half)
    ql[:n_pos_low] = 1.0
    rng.shuffle(ql)
    qu = np.ones(N - half)
    qu[:n_pos_low] = -1.0
    rng.shuffle(qu)
    q[:half], q[half:] = ql, qu
    return x, q


def clustered(N, box, seed, frac=0.4, sd=0.7, top=0.05):
    rng = np.random.default_rng(seed)
    Lx, Ly, Lz = box
    nc = int(round(frac * N))
    nt = int(round(top * (N - nc)))
    nb = N - nc - nt
    x = np.empty((N, 3))
    c = rng.normal(0.0, sd, (nc, 3)) + 0.5 * np.asarray(box, dtype=np.float64)
    bad = (c[:, 2] < 0.0) | (c[:, 2] > Lz)
    while bad.any():
        c[bad, 2] = rng.normal(0.5 * Lz, sd, int(bad.sum()))
        bad = (c[:, 2] < 0.0) | (c[:, 2] > Lz)
    c[:, 0] %= Lx
    c[:, 1] %= Ly
    x[:nc] = c
    x[nc:, 0] = rng.random(N - nc) * Lx
    x[nc:, 1] = rng.random(N - nc) * Ly
    x[nc:nc + nb, 2] = rng.random(nb) * (0.5 * Lz)
    x[nc + nb:, 2] = 0.5 * Lz + rng.random(nt) * (0.5 * Lz)
    return x, _charges(rng, N)


def named(name):
    N, box = NAMED[name]
    seed = NAMED_SEED[name]
    if name.startswith("layered"):
        return (*layered(N, box, seed), box)
    return (*uniform(N, box, seed), box)


def batch_specs(n_systems=256, seed=5, Nmin=500, Nmax=20000, density=1.0):
    """List of (N_s, box, seed_s) for the batched workload."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_systems):
        N = int(np.exp(rng.uniform(np.log(Nmin), np.log(Nmax))))
        N -= N % 2
        a = float(rng.choice([1.0 / 8.0, 1.0, 8.0]))
        Lx = (N / density / a) ** (1.0 / 3.0)
        out.append((N, (Lx, Lx, a * Lx), seed + s))
    return out


def batch(specs=None):
    """(x, q, boxes, ns) of a batch: each system uniform in its own box with its own seed,
    the systems' particles stored one after another."""
    specs = batch_specs() if specs is None else specs
    xs, qs = [], []
    for N, box, seed in specs:
        x, q = uniform(N, box, seed)
        xs.append(x)
        qs.append(q)
    return np.concatenate(xs), np.concatenate(qs), [b for _n, b, _s in specs], [n for n, _b, _s in specs]


# systems of the 256-system batch with stored reference values: the three smallest and the
# three largest, and two of each height ratio (1/8, 1, 8) of middle size
BATCH_CHECKED = (6, 32, 82, 86, 93, 136, 138, 144, 150, 195, 197, 230)
