#!/usr/bin/env python
"""Benchmark of the MI355X SOG solver: particles/s for one energy + potential + force
evaluation at 1e-4 relative tolerance, N = 10^6 (uniform, 100^3 box), FP32-bulk form
and plain FP64 form, inputs resident in HBM.

Prints ONE JSON line.  Timed region: K calls of sog_energy_potential_force with device
pointers, bracketed by torch.cuda.synchronize().  Per-kernel device times come from the
library's HIP events, recorded on the plan's stream (torch's current stream) during
the same timed calls; the roofline entry uses them for the dominant kernel.

Only this benchmark's cpu_baseline leg runs the CPU oracle (on a bounded sample).
"""
import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: HBM3E 8 TB/s; FP32 vector 157.3 TFLOP/s; FP64 vector 78.6 TFLOP/s.
# The kernels are built without packed-FP32 instructions, so the FP32 rate they can reach
# is one FMA per lane per clock, 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz =
# 78.6 TFLOP/s; that figure is reported beside the published one (frac_nonpacked).
PEAK = {"hbm_GBs": 8000.0, "fp32_alu_TFs": 157.3, "fp32_nonpacked_TFs": 78.6, "fp64_alu_TFs": 78.6}
# algorithmic work per unit of the method: ~30 flops per ordered near-field pair within r_c
# (distance, the kernel N(r) and N'(r)/r, accumulation of the potential and gradient)
NEAR_FLOPS_PER_PAIR = 30
METRIC = "particles/s energy+forces at 1e-4 rel err, N=1e6; FP32-bulk vs FP64 plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_models(info, sizes, N, box, rs):
    """Algorithmic work of one launch of the main kernels (flops, HBM bytes); rs is the
    working precision's bytes per real: per ordered near-field pair, per particle and window
    point, and per grid point of each FFT pass, times the units one launch processes."""
    Pw = info["mid_Pw"][0]
    # the z planes the gridding, the z transforms and the gathering touch
    Nb = info["mid_I"][0] * info["mid_I"][1] * (sizes["mid_zband"][1] - sizes["mid_zband"][0])
    rc = info["rc"]
    deg = sizes["near_degree"]
    rho = N / (box[0] * box[1] * box[2])
    pairs = N * (4.0 * math.pi / 3.0) * rc ** 3 * rho   # ordered pairs within r_c (uniform density)
    m = {}
    # near: per ordered pair within r_c; bytes: the packed particle in, 4 results out
    m["near"] = dict(flops=pairs * NEAR_FLOPS_PER_PAIR, bytes=N * (4 * rs + 4 + 4 * rs), bound="alu")
    # spread: one FMA per window node; particle records in, grid read and written once
    m["mid_spread"] = dict(flops=N * 2 * Pw ** 3, bytes=N * (16 + 4 * rs) + 2 * Nb * rs, bound="alu")
    # gather: two FMAs per window node (value and z derivative) plus the y and x sums
    m["mid_gather"] = dict(flops=N * (4 * Pw ** 3 + 6 * Pw ** 2 + 8 * Pw), bytes=N * (16 + 4 * rs + 4 * rs) + Nb * rs,
                           bound="alu")
    Kz = info["mid_Izs"] // 2 + 1
    cg = info["mid_I"][0] * info["mid_I"][1] * Kz * 2 * rs
    m["fft_z_fwd"] = dict(flops=None, bytes=Nb * rs + cg, bound="hbm")
    m["fft_z_inv"] = dict(flops=None, bytes=Nb * rs + cg, bound="hbm")
    m["fft_y_fwd"] = dict(flops=None, bytes=2 * cg, bound="hbm")
    m["fft_y_inv"] = dict(flops=None, bytes=2 * cg, bound="hbm")
    m["fft_x_scale"] = dict(flops=None, bytes=2 * cg, bound="hbm")
    return m


def roofline_of(mdl, t_s, fp64=False):
    if mdl["bound"] == "hbm":
        ach = mdl["bytes"] / t_s / 1e9
        return dict(bound="hbm", achieved=ach, peak=PEAK["hbm_GBs"], unit="GB/s", frac=ach / PEAK["hbm_GBs"])
    pk = PEAK["fp64_alu_TFs"] if fp64 else PEAK["fp32_alu_TFs"]
    ach = mdl["flops"] / t_s / 1e12
    out = dict(bound="alu", achieved=ach, peak=pk, unit="TFLOP/s", frac=ach / pk)
    if not fp64:
        out["frac_nonpacked"] = ach / PEAK["fp32_nonpacked_TFs"]
    return out


def spread_gather_hbm(info, sizes, N, per_launch, rs):
    """The gridding + gathering pair against the HBM roof, with the algorithmic bytes of
    the method: particle records in and out (16 B in, 16 B out in float32; 32 + 32 in
    float64) plus one write and one read of every mid-range grid point.  Also given for
    the z band of planes that windows can reach (the only planes the kernels touch)."""
    if "mid_spread" not in per_launch or "mid_gather" not in per_launch:
        return None
    Ng = info["mid_I"][0] * info["mid_I"][1] * info["mid_Izs"]
    t = (per_launch["mid_spread"] + per_launch["mid_gather"]) * 1e-3
    Nb = info["mid_I"][0] * info["mid_I"][1] * (sizes["mid_zband"][1] - sizes["mid_zband"][0])
    b_full = N * 8 * rs + 2 * Ng * rs
    b_band = N * 8 * rs + 2 * Nb * rs
    ach = b_full / t / 1e9
    return dict(bound="hbm", achieved=ach, peak=PEAK["hbm_GBs"], unit="GB/s", frac=ach / PEAK["hbm_GBs"],
                algorithmic_bytes=b_full, ms=t * 1e3, per_particle_bytes=b_full / N,
                band=dict(achieved=b_band / t / 1e9, frac=b_band / t / 1e9 / PEAK["hbm_GBs"],
                          algorithmic_bytes=b_band))


def source_digest():
    """Digest of the library's sources with comments and white space taken out, so that
    the committed profiles stay tied to the kernels' code and not to their comments."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2412_04595_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(f.encode())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch (fetched + written) from the committed rocprofv3 counter
    summary, if it was taken on the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    digest = source_digest()
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if len(f) >= 4 and f[0] == kernel and f[3] == digest:
            return float(f[1]) + float(f[2])
    return None


def counters_from_profiles(kernel, workload):
    """The committed rocprofv3 counter summary's line for the kernel (VALU issue, MFMA busy,
    LDS activity and bank conflicts, resident waves per CU), if taken on the current sources."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.txt")
    if not os.path.exists(path):
        return None
    digest = None
    for line in open(path):
        if line.startswith("# sources digest"):
            digest = line.split()[-1]
    if digest != source_digest():
        return None
    for line in open(path):
        f = line.split()
        if f and not line.startswith("#") and f[0] == kernel and len(f) >= 9:
            return {"valu_issue": float(f[3]), "mfma_busy": float(f[4]), "lds_active": float(f[5]),
                    "lds_bank_conflict": float(f[6]), "waves_per_cu": float(f[7]),
                    "source": f"profiles/counters_{workload}.txt"}
    return None


def reference_energy(workload):
    """The oracle's energy of the workload (plain fast method at two tolerances that
    agree), from tests/golden/<workload>_energy.txt, or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_energy.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split()
        if f and f[0] == "U":
            return float(f[1])
    return None


def accuracy(workload, U, phi, F, q):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_targets.txt")
    if not os.path.exists(path):
        return None
    d = np.loadtxt(path, comments="#")
    idx = d[:, 0].astype(np.int64)
    rphi, rgrad = d[:, 1], d[:, 2:5]
    rF = -q[idx, None] * rgrad
    Uref = reference_energy(workload)
    return dict(
        n_targets=int(idx.size),
        energy_rel=None if Uref is None else abs(U - Uref) / abs(Uref),
        phi_rel_linf=float(np.max(np.abs(phi[idx] - rphi)) / np.max(np.abs(rphi))),
        phi_rel_rms=float(np.sqrt(np.mean((phi[idx] - rphi) ** 2) / np.mean(rphi ** 2))),
        force_rel_linf=float(np.max(np.abs(F[idx] - rF)) / np.max(np.abs(rF))),
        force_rel_rms=float(np.sqrt(np.mean(np.sum((F[idx] - rF) ** 2, 1)) / np.mean(np.sum(rF ** 2, 1)))),
        reference="potentials and forces: oracle SOG-direct on sampled particles (exact decomposition, "
                  "b=1.2181), tests/golden/<workload>_targets.txt; energy: oracle fast method at tol 1e-10, "
                  "tests/golden/<workload>_energy.txt",
    )


def cpu_baseline(tol):
    """The oracle (plain NumPy fast SOG method) on a bounded sample of the workload:
    uniform particles at the same density (1 per unit volume) in a smaller cube, same
    tolerance, parameters from oracle.planner, single-threaded BLAS/FFT.  A first
    sample of 27000 particles (30^3) sets the pace; if it ran under 10 s, a second cube
    sized for about 15 s of oracle work (at most the full workload) is timed and
    reported."""
    from threadpoolctl import threadpool_limits
    from oracle import fast, planner
    import workloads

    def timed(L):
        Ns = int(L) ** 3
        box = (float(L),) * 3
        x, q = workloads.uniform(Ns, box, 2)
        p = planner.plan(box, Ns, tol)
        tm = {}
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            fast.solve(x, q, box, p, times=tm)
            return Ns, time.perf_counter() - t0, tm

    L = 30
    Ns, t, tm = timed(L)
    note = ""
    if t < 10.0:
        first = f"; a first sample of {Ns} took {t:.1f} s"
        # oracle time grows about as N^1.3 here; even side: even N
        L = min(100, max(L + 2, 2 * int(round(L * (15.0 / t) ** (1.0 / 3.9) / 2))))
        Ns, t, tm = timed(L)
        note = first
    return dict(value=Ns / t, unit="particles/s", cores=1, kind="oracle",
                host_cpu_count=os.cpu_count(),
                threads_used="1 (NumPy, SciPy FFT and BLAS limited to one thread)",
                stages_s={"t_short": tm["short"], "t_mid": tm["mid"], "t_long": tm["long"]},
                sample=f"oracle.fast.solve, N={Ns} uniform in {L}^3 (density 1 as the workload), tol {tol:g}, "
                       f"oracle.planner parameters, 1 thread of {os.cpu_count()} host cores: {t:.1f} s "
                       f"(near {tm['short']:.1f}, mid {tm['mid']:.1f}, long {tm['long']:.1f}){note}")


def run_form(sog, torch, xt, qt, box, N, tol, precision, steps, warmup, params=None, deterministic=False,
             autotune=False):
    """Times `steps` calls of a plan as the library runs them by default (the call's
    kernels replayed as one HIP graph): that is the step time.  A second plan with the same
    parameters and kernel timing on (HIP events around every kernel, launched one by one)
    then runs as many calls for the per-kernel durations of the roofline."""
    s = sog.Solver(box, N, tol, precision=precision, on_device=True, check_inputs=False, params=params,
                   deterministic=deterministic, autotune=autotune)
    tuning = s.tuning()
    info, sizes = s.info(), s.sizes()
    # one checked call first: inputs valid, neutral, z in range
    chk = sog.Solver(box, N, tol, precision=precision, on_device=True, check_inputs=True, params=params)
    chk(xt, qt)
    chk.close()
    for _ in range(warmup):
        s(xt, qt)
    torch.cuda.synchronize()
    # the step: energy, potentials and forces of every call left in device memory (the
    # next call is queued while one runs)
    t0 = time.perf_counter()
    for _ in range(steps):
        U, phi, F = s(xt, qt, energy_on_device=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    U = float(U[0])
    # the same with the energy read back to the host after every call (each call then
    # waits for the one before it to finish)
    t0 = time.perf_counter()
    for _ in range(steps):
        s(xt, qt)
    torch.cuda.synchronize()
    dt_host_energy = (time.perf_counter() - t0) / steps
    s.close()
    # the same parameters, kernel by kernel with events
    keep = ("b", "r0", "omega", "rc", "M", "m", "set_m", "mid_I", "mid_Izs", "mid_Pw", "mid_S", "mid_window",
            "mid_beta", "mid_nu", "long_form", "long_P", "long_nk", "long_I", "long_Pw", "long_S", "long_Q")
    st = sog.Solver(box, N, tol, precision=precision, on_device=True, check_inputs=False, timing=True,
                    params={k: info[k] for k in keep}, deterministic=deterministic)
    for _ in range(warmup):
        st(xt, qt)
    torch.cuda.synchronize()
    st.reset_kernel_times()
    t0 = time.perf_counter()
    for _ in range(steps):
        st(xt, qt)
    torch.cuda.synchronize()
    dt_eager = (time.perf_counter() - t0) / steps
    kt = st.kernel_times()
    st.close()
    return dict(dt=dt, dt_eager=dt_eager, dt_host_energy=dt_host_energy, U=U, phi=phi, F=F, kt=kt, info=info,
                sizes=sizes, tuning=tuning)


def secondary(sog, torch, name, tol, steps):
    """Both forms on a second workload (device-resident inputs, the same timing as the
    headline), with the sampled-target accuracy and the long range's kernel split."""
    import workloads
    x, q, box = workloads.named(name)
    N = len(q)
    xt = torch.from_numpy(x).cuda()
    qt = torch.from_numpy(q).cuda()
    out = {}
    for prec in ("fp32", "fp64"):
        r = run_form(sog, torch, xt, qt, box, N, tol, prec, steps, 2)
        acc = accuracy(name, r["U"], r["phi"].cpu().numpy(), r["F"].cpu().numpy(), q)
        info = r["info"]
        out[prec] = {"value": N / r["dt"], "unit": "particles/s", "ms_per_step": r["dt"] * 1e3, "accuracy": acc,
                     "kernels_ms_per_step": {k: round(v[0] / steps, 4) for k, v in
                                             sorted(r["kt"].items(), key=lambda kv: -kv[1][0])},
                     "plan": {k: info[k] for k in ("rc", "M", "m", "long_form", "long_P", "long_Q", "long_I",
                                                   "long_Pw")}}
        log(f"[bench] {name} {prec} {r['dt'] * 1e3:.3f} ms/step")
    return out


def batch_run(steps, warmup, tol):
    """The 256-system batch (N log-uniform in [500, 20000], Lz/Lx in {1/8, 1, 8}, density 1)
    in float32 through one batch plan: each timed step is one sog_batch_energy_potential_force
    call (input copy into the batch's buffers, one graph launch, output copy)."""
    import numpy as np
    import torch
    import paper_2412_04595_amd as sog
    import workloads

    x, q, boxes, ns = workloads.batch()
    N = len(q)
    xt = torch.from_numpy(x).cuda()
    qt = torch.from_numpy(q).cuda()
    log(f"[bench] batch_256: {len(ns)} systems, {N} particles, tol {tol}")
    chk = sog.BatchSolver(boxes, ns, tol, precision="fp32", on_device=True, check_inputs=True)
    chk(xt, qt)
    chk.close()
    t0 = time.perf_counter()
    b = sog.BatchSolver(boxes, ns, tol, precision="fp32", on_device=True, check_inputs=False)
    t_plan = time.perf_counter() - t0
    groups, launches = b.graph_info()
    for _ in range(warmup):
        b(xt, qt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        U, phi, F = b(xt, qt)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    phi, F = phi.cpu().numpy(), F.cpu().numpy()
    d = np.loadtxt(os.path.join(ROOT, "tests", "golden", "batch_256_targets.txt"), comments="#")
    sysi, idx = d[:, 0].astype(np.int64), d[:, 1].astype(np.int64)
    ephi = eF = 0.0
    for s in sorted(set(sysi.tolist())):
        m = sysi == s
        g = b.offsets[s] + idx[m]
        rF = -q[g, None] * d[m, 3:6]
        ephi = max(ephi, float(np.max(np.abs(phi[g] - d[m, 2])) / np.max(np.abs(d[m, 2]))))
        eF = max(eF, float(np.max(np.abs(F[g] - rF)) / np.max(np.abs(rF))))
    b.close()
    log(f"[bench] batch_256 {dt * 1e3:.3f} ms/step ({groups} groups, {launches} launches)")
    return dict(N=N, systems=len(ns), dt=dt, plan_seconds=t_plan, groups=groups, launches=launches,
                accuracy={"phi_rel_linf": ephi, "force_rel_linf": eF,
                          "reference": "tests/golden/batch_256_targets.txt (12 systems x 4 sampled targets)"})


def bench_batch(args):
    r = batch_run(args.steps, args.warmup, args.tol)
    out = {
        "metric": METRIC,
        "value": r["N"] / r["dt"],
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["dt"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch_256: {r['systems']} independent systems, N log-uniform in [500, 20000] "
                               f"(total {r['N']}), Lz/Lx in {{1/8, 1, 8}}, density 1, uniform +/-1 neutral, "
                               f"tol {args.tol:g}, FP32-bulk form, one graph launch per step",
                   "systems": r["systems"], "N": r["N"], "tol": args.tol},
        "plan_seconds": r["plan_seconds"],
        "graph": {"groups": r["groups"], "kernel_launches": r["launches"]},
        "accuracy": r["accuracy"],
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube_1e6")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-confined", action="store_true", help="skip the strongly confined box")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-system batch")
    ap.add_argument("--no-kb", action="store_true", help="skip the KB-window run of the headline workload")
    ap.add_argument("--no-deterministic", action="store_true",
                    help="skip the deterministic-mode run of the headline workload")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuned runs of the headline workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run three 256 MiB device-to-device copies (the known-size copy that scales the "
                         "HBM counters of a profiling run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the solver has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch_256":
        bench_batch(args)
        return
    import numpy as np
    import torch
    import paper_2412_04595_amd as sog
    import workloads

    x, q, box = workloads.named(args.workload)
    N = len(q)
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(x).to(dev)
    qt = torch.from_numpy(q).to(dev)
    torch.cuda.synchronize()
    log(f"[bench] {args.workload} N={N} box={box} tol={args.tol}")
    r32 = run_form(sog, torch, xt, qt, box, N, args.tol, "fp32", args.steps, args.warmup)
    log(f"[bench] fp32-bulk {r32['dt'] * 1e3:.3f} ms/step")
    r64 = None
    if not args.no_fp64:
        r64 = run_form(sog, torch, xt, qt, box, N, args.tol, "fp64", max(3, args.steps // 2), 1)
        log(f"[bench] fp64 {r64['dt'] * 1e3:.3f} ms/step")
    if args.copy_calibration:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    phi32 = r32["phi"].cpu().numpy()
    F32 = r32["F"].cpu().numpy()
    acc32 = accuracy(args.workload, r32["U"], phi32, F32, q)
    acc64 = accuracy(args.workload, r64["U"], r64["phi"].cpu().numpy(), r64["F"].cpu().numpy(), q) if r64 else None

    # roofline of the dominant kernel (FP32-bulk run), from the library's HIP events on
    # the plan's stream during the timed calls
    kt = r32["kt"]
    per_launch = {k: v[0] / max(v[1], 1) for k, v in kt.items()}
    per_step = {k: v[0] / args.steps for k, v in kt.items()}
    dom = max(per_step, key=per_step.get)
    models = kernel_models(r32["info"], r32["sizes"], N, box, 4)
    roof = None
    if dom in models:
        mdl = models[dom]
        roof = roofline_of(mdl, per_launch[dom] * 1e-3)
        roof["traffic"] = traffic_from_profiles(dom, args.workload)
        roof["counters"] = counters_from_profiles(dom, args.workload)
        roof["kernel"] = dom
        roof["kernel_ms"] = per_launch[dom]
        roof["algorithmic_bytes"] = mdl["bytes"]
        if mdl["flops"] is not None:
            roof["algorithmic_flops"] = mdl["flops"]
    others = {}
    for k, mdl in models.items():
        if k in per_launch:
            rf = roofline_of(mdl, per_launch[k] * 1e-3)
            others[k] = {"bound": rf["bound"], "frac": round(rf["frac"], 4), "achieved": round(rf["achieved"], 3),
                         "unit": rf["unit"], "ms": round(per_launch[k], 4)}
    # the same workload with the KB window by its polynomials (Remark rmk::PWindow) in place
    # of the planner's window
    kb = None
    if not args.no_kb:
        rk = run_form(sog, torch, xt, qt, box, N, args.tol, "fp32", max(5, args.steps // 2), 2,
                      params=dict(mid_window=sog._lib.SOG_WINDOW_KB))
        info = rk["info"]
        kb = {"value": N / rk["dt"], "unit": "particles/s", "ms_per_step": rk["dt"] * 1e3,
              "accuracy": accuracy(args.workload, rk["U"], rk["phi"].cpu().numpy(), rk["F"].cpu().numpy(), q),
              "plan": {k: info[k] for k in ("rc", "m", "mid_I", "mid_Izs", "mid_Pw", "mid_beta", "mid_nu")},
              "kernels_ms_per_step": {k: round(v[0] / max(5, args.steps // 2), 4) for k, v in
                                      sorted(rk["kt"].items(), key=lambda kv: -kv[1][0]) if k in ("mid_spread", "mid_gather")}}
        log(f"[bench] {args.workload} fp32 KB window {rk['dt'] * 1e3:.3f} ms/step")
    # the same workload with an autotuned plan (the planner's three cheapest r_c timed on a
    # uniform sample, the fastest kept)
    tuned = None
    if not args.no_autotune:
        for prec in ("fp32", "fp64"):
            if prec == "fp64" and args.no_fp64:
                continue
            rt = run_form(sog, torch, xt, qt, box, N, args.tol, prec, max(5, args.steps // 2), 2, autotune=True)
            tuned = tuned or {}
            tuned[prec] = {"value": N / rt["dt"], "unit": "particles/s", "ms_per_step": rt["dt"] * 1e3,
                           "plan": {k: rt["info"][k] for k in ("rc", "m", "mid_I", "mid_Pw", "long_P")},
                           "tuning_ms": [[round(rc, 4), m, round(ms, 4)] for rc, m, ms in rt["tuning"]]}
            log(f"[bench] {args.workload} {prec} autotuned {rt['dt'] * 1e3:.3f} ms/step (r_c {rt['info']['rc']:.3f})")
    # the same workload in the deterministic mode (canonical bin orders, coloured gridding)
    det = None
    if not args.no_deterministic:
        steps_d = max(5, args.steps // 2)
        rd = run_form(sog, torch, xt, qt, box, N, args.tol, "fp32", steps_d, 2, deterministic=True)
        det = {"value": N / rd["dt"], "unit": "particles/s", "ms_per_step": rd["dt"] * 1e3,
               "kernels_ms_per_step": {k: round(v[0] / steps_d, 4) for k, v in
                                       sorted(rd["kt"].items(), key=lambda kv: -kv[1][0]) if k.endswith("sort")
                                       or k in ("mid_spread", "near", "long2_spread")}}
        log(f"[bench] {args.workload} fp32 deterministic {rd['dt'] * 1e3:.3f} ms/step")
    confined = None
    if not args.no_confined:
        confined = secondary(sog, torch, "confined_1e6", args.tol, max(5, args.steps // 2))
        confined["workload"] = ("confined_1e6: N=1000000 uniform +/-1 neutral in 953.5x953.5x0.3 (surface density 1.1, "
                                "the strongly confined box of the paper's Table 4), tol %g" % args.tol)
        confined["paper_context"] = ("Table 4, same N and box: 11.5 s at eps_r 1e-3, 55.0 s at 1e-6, potentials only, one "
                                     "core of a Threadripper PRO 3995WX (Julia)")
    batched = None
    if not args.no_batch:
        r = batch_run(max(5, args.steps // 2), 2, args.tol)
        batched = {"value": r["N"] / r["dt"], "unit": "particles/s", "ms_per_step": r["dt"] * 1e3,
                   "workload": f"batch_256: {r['systems']} independent systems (total {r['N']} particles), N "
                               f"log-uniform in [500, 20000], Lz/Lx in {{1/8, 1, 8}}, density 1, FP32-bulk, tol "
                               f"{args.tol:g}, one graph launch per step",
                   "plan_seconds": r["plan_seconds"], "graph": {"groups": r["groups"], "kernel_launches": r["launches"]},
                   "accuracy": r["accuracy"]}
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on a bounded sample)")
        cpu = cpu_baseline(args.tol)
    value = N / r32["dt"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["dt"] * 1e3,
        "ms_per_step_eager_timed": r32["dt_eager"] * 1e3,
        "ms_per_step_host_energy": r32["dt_host_energy"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: N={N} uniform +/-1 neutral in {box[0]:g}x{box[1]:g}x{box[2]:g}, "
                               f"seed {workloads.NAMED_SEED[args.workload]}, tol {args.tol:g}, FP32-bulk form",
                   "N": N, "box": list(box), "tol": args.tol},
        "fp64": None if r64 is None else {"value": N / r64["dt"], "ms_per_step": r64["dt"] * 1e3,
                                         "accuracy": acc64},
        "speedup_fp32_vs_fp64": None if r64 is None else r64["dt"] / r32["dt"],
        "accuracy": acc32,
        "roofline": roof,
        "spread_gather_hbm": spread_gather_hbm(r32["info"], r32["sizes"], N, per_launch, 4),
        "roofline_kernels": others,
        "kb_window": kb,
        "deterministic": det,
        "autotuned": tuned,
        "strongly_confined": confined,
        "batched": batched,
        "cpu_baseline": cpu,
        "kernels_ms_per_step": {k: round(v, 4) for k, v in sorted(per_step.items(), key=lambda kv: -kv[1])},
        "plan": {k: r32["info"][k] for k in ("rc", "M", "m", "mid_I", "mid_Izs", "mid_Pw", "long_form", "long_P",
                                              "long_nk", "long_I", "long_Pw")},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
