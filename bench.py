"""Throughput benchmark of the fused ISLBM time step on one MI355X.

Workload (the metric's headline configuration): 2-D side-heated cavity,
Ra = 1e8, Pr = 0.71, 1024 x 1024 cosine-stretched mesh (x_j = (1 - cos(pi
j/(N+1)))/2 on both axes), D2Q9 flow + D2Q5 temperature populations, FP32
storage in population rows, start at rest, walls +-0.5.  One "step" is one
fused launch over the whole mesh.  Printed next to it: the same size on a
uniform mesh (plain-shift kernel), the roofline of the dominant kernel (its
working set fits the last-level cache, and says so), a 1 GiB device-copy
ceiling, the FP64 instantiation on the headline mesh, the workloads beyond the
cache (2-D 4096^2, 3-D 256^3 and 384^3 in FP32, 3-D 384^3 in FP16 and BF16,
each beside its uniform mesh), a small learned-warm-start study (steps to a
steady Nusselt number, warm against cold) and the FP64 CPU oracle timed on
the host cores over a bounded sample (all cores and one thread).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--headline-only] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E peak
N_CFG = 1024
RA, PR = 1e8, 0.71
BYTES_PER_LU = {2: {"fp32": 112, "fp64": 224, "fp16": 56, "bf16": 56, "fp32sr": 112},
                3: {"fp32": 208, "fp64": 416, "fp16": 104, "bf16": 104, "fp32sr": 208}}
KERNEL_SOURCES = ("paper_2509_01099_amd/csrc/islbm_kernels.hip",
                  "paper_2509_01099_amd/csrc/islbm_lattice.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step2d_fp32_cosine1024_traffic.json")
# workloads of --profile: (mesh kind, shape)
PROFILE_MESHES = {"2d": ("cosine", (N_CFG, N_CFG)), "2d-4096": ("cosine", (4096, 4096)),
                  "3d": ("tanh", (256, 256, 256)), "3d-384": ("tanh", (384, 384, 384)),
                  "3d-uniform": ("uniform", (256, 256, 256))}


def kernel_digest() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stable_uf(H_lu: float, dim: int = 2) -> float:
    """Largest u_f with a_T <= 1 (non-negative thermal rest weight): the
    throughput does not depend on u_f, the stability of the run does."""
    alpha_max = 5.0 / (20.0 * 3 ** 0.5) if dim == 2 else 7.0 / (42.0 * 3 ** 0.5)
    return min(0.1 / 3 ** 0.5, alpha_max * (RA * PR) ** 0.5 / H_lu)


def make_cavity(kind: str, n, storage="fp32", Ra=RA, **opts):
    import paper_2509_01099_amd as pkg

    sp = [pkg.islbm_mesh_spacing(kind, k, 1.5) for k in n]
    sp = [s / s[0] for s in sp]
    H = float(sum(sp[1]) - 0.5 * sp[1][0] - 0.5 * sp[1][-1])
    uf = opts.pop("u_f", None)
    if uf is None:
        uf = stable_uf(H, len(n)) if Ra == RA else 0.0
    return pkg.Cavity(sp, Ra, PR, storage=storage, u_f=uf, **opts), H, uf


def time_run(cav, steps: int, warmup: int):
    """Warm-up, then exactly `steps` fused launches bracketed by device
    synchronisation; returns (wall seconds, device-event seconds)."""
    import torch

    if warmup > 0:                      # through the timed entry point, as in time_run_split
        cav.time_steps(warmup)
    cav.plan(steps)                     # captures the launch graphs; runs no step
    cav.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = cav.time_steps(steps)          # HIP events on the launch stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ms / 1e3


def time_run_split(cav, steps: int, warmup: int):
    """As time_run, with the device time split at the final (reducing)
    launch: returns (wall s, all launches s, plain launches s, reducing s)."""
    import torch

    # the untimed warm-up steps go through the same timed entry point, so that
    # the runtime's one-time event set-up is not charged to the timed call
    if warmup > 0:
        cav.time_steps_split(warmup)
    cav.plan(steps)                     # captures the launch graphs; runs no step
    cav.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot, plain, red = cav.time_steps_split(steps)   # HIP events on the launch stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, tot / 1e3, plain / 1e3, red / 1e3


# Workloads beyond the 256 MB last-level cache (plus the uniform mesh of each
# size): (label, mesh kind, shape, storage, timed launches)
HBM_ROWS = (("2-D 4096^2 cosine, Ra 1e8", "cosine", (4096, 4096), "fp32", 300),
            ("2-D 4096^2 uniform, Ra 1e8", "uniform", (4096, 4096), "fp32", 300),
            ("3-D 256^3 tanh, Ra 1e7", "tanh", (256, 256, 256), "fp32", 200),
            ("3-D 256^3 uniform, Ra 1e7", "uniform", (256, 256, 256), "fp32", 200),
            ("3-D 384^3 tanh, Ra 1e7", "tanh", (384, 384, 384), "fp32", 100),
            ("3-D 384^3 uniform, Ra 1e7", "uniform", (384, 384, 384), "fp32", 100),
            ("3-D 384^3 tanh, Ra 1e7", "tanh", (384, 384, 384), "fp16", 100),
            ("3-D 384^3 tanh, Ra 1e7", "tanh", (384, 384, 384), "bf16", 100),
            ("3-D 384^3 uniform, Ra 1e7", "uniform", (384, 384, 384), "fp16", 100))


def step_row(label, kind, shape, storage, steps, warmup=10, copy_GBs=None, Ra=None):
    """MLUPS and algorithmic bandwidth of one workload from the device time of
    its plain launches (the final, reducing launch timed apart)."""
    three = len(shape) == 3
    Ra = Ra if Ra is not None else (1e7 if three else RA)
    cav, _, _ = make_cavity(kind, shape, storage=storage, Ra=Ra,
                            **({"u_f": 0.0} if three else {}))
    _, _, plain, red = time_run_split(cav, steps, warmup)
    bad = cav.stats(allow_nonfinite=True)["nonfinite"]
    cav.close()
    nodes = math.prod(shape)
    per = plain / (steps - 1)
    mlups = nodes / per / 1e6
    gbs = BYTES_PER_LU[len(shape)][storage] * nodes / per / 1e9
    row = {"workload": label, "storage": storage, "mlups": round(mlups, 1),
           "bytes_per_update": BYTES_PER_LU[len(shape)][storage],
           "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
           "avg_launch_us": round(per * 1e6, 2), "reducing_launch_us": round(red * 1e6, 2),
           "nonfinite_nodes": bad}
    if copy_GBs:
        row["frac_of_copy"] = round(gbs / copy_GBs, 4)
    return row


def copy_ceiling(nbytes: int = 1 << 30, reps: int = 20) -> dict:
    """Read + write bandwidth of 1 GiB device copies (the library's 16-byte
    vector copy and torch's copy_), HIP events on the current stream."""
    import torch

    import paper_2509_01099_amd as pkg

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    stream = torch.cuda.current_stream()
    out = {}
    for name, fn in (("vector16", lambda: pkg.islbm_copy_bytes(dst.data_ptr(), src.data_ptr(), nbytes,
                                                              stream.cuda_stream)),
                     ("torch_copy", lambda: dst.copy_(src))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        out[name] = round(2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9, 1)
    ok = bool(torch.equal(dst, src))
    del src, dst
    torch.cuda.empty_cache()
    return {"copy_ceiling_GBs": max(out.values()), "copies_GBs": out, "bytes": nbytes,
            "copy_verified": ok}


def warmstart_block() -> dict:
    """Learned warm start on a small 2-D cavity (129^2 erf mesh, FP64 storage):
    16 training and 4 held-out Rayleigh numbers in [1e6, 1e7]; steps to a
    steady Nusselt number from the network's prediction against the cold
    start from rest (the metric's second half)."""
    from paper_2509_01099_amd import warmstart as W

    return W.quick_study(n=129, n_train=16, n_held=4, steps=600_000, train_steps=8000, log=_log)


def traffic_entry(dig: str):
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_digest") != dig:
        return None
    return rec.get("bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            return next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        return "host CPU"


def _oracle_mlups(threads: int, seconds: float):
    """MLUPS of the unmodified FP64 oracle on the 1024^2 cosine workload
    (Ra 1e8, from rest) with `threads` OpenMP threads, over about `seconds`."""
    import oracle

    oracle.set_threads(threads)
    x = oracle.mesh("cosine", N_CFG)
    x = x / (x[1] - x[0])
    H = 0.5 * (x[-1] + x[-2]) - 0.5 * (x[0] + x[1])
    orc = oracle.Oracle([x, x], RA, PR, uf=stable_uf(H))
    orc.run(1)
    steps, el = 0, 0.0
    t0 = time.perf_counter()
    while el < seconds:
        orc.run(1)
        steps += 1
        el = time.perf_counter() - t0
    used = oracle.get_threads()
    del orc
    return N_CFG * N_CFG * steps / el / 1e6, steps, el, used


def cpu_baseline(seconds_all: float = 10.0, seconds_one: float = 8.0):
    """The FP64 oracle, unmodified, on the host cores: a bounded sample of
    the same workload (1024^2 cosine mesh, Ra 1e8, from rest), once on all
    the cores this process may use (capped by OMP_NUM_THREADS when set) and
    once on a single thread."""
    nproc = os.cpu_count() or 1
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = nproc
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(allowed, int(omp)) if omp.isdigit() and int(omp) > 0 else allowed
    cpu = _cpu_model()
    m_all, s_all, e_all, used = _oracle_mlups(threads, seconds_all)
    m_one, s_one, e_one, _ = _oracle_mlups(1, seconds_one)
    return {"value": round(m_all, 3), "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"{s_all} steps of the 1024^2 cosine 2-D cavity (Ra 1e8, FP64) in "
                      f"{e_all:.1f} s on {used} threads of {cpu}",
            "single_thread": {"value": round(m_one, 3), "unit": "MLUPS", "cores": 1,
                              "sample": f"{s_one} steps in {e_one:.1f} s on 1 thread"},
            "host": {"cpu_model": cpu, "nproc": nproc, "affinity_cpus": allowed,
                     "OMP_NUM_THREADS": omp or None}}


def precision_study(steps: int, n: int = 384, steady_steps: int = 1_600_000) -> dict:
    """Storage-precision study (growth row: FP16/BF16 deviation storage), the
    FP64 instantiation on the same GPU being the reference.
      throughput: MLUPS of each storage type on the 2-D benchmark workload
        (1024^2 cosine, Ra 1e8) and the 3-D workload (n^3 tanh, Ra 1e7);
      transient: the 3-D workload from rest for `steps` steps;
      steady: 2-D 257^2 erf cavity at Ra 1e7 run to steady state
        (`steady_steps`, the four storage types concurrently), with the steps
        until Nu_hot stays within 1e-3 of the FP64 steady value."""
    import paper_2509_01099_amd as pkg
    from paper_2509_01099_amd import warmstart as W

    kinds = ("fp64", "fp32", "fp16", "bf16", "fp32sr")
    keys = ("nu_vol", "nu_hot", "nu_cold", "re_vol", "re_rms", "umax", "vmax", "wmax")
    out = {"throughput": {}, "transient": {}, "steady": {}}
    for st in kinds:
        for label, kind, shape, ra, k in (("2d_cosine_1024", "cosine", (N_CFG, N_CFG), RA, 20000),
                                          (f"3d_tanh_{n}", "tanh", (n, n, n), 1e7, 400)):
            cav, H, uf = make_cavity(kind, shape, storage=st, Ra=ra)
            wall, dev = time_run(cav, k, 20)
            cav.close()
            nodes = math.prod(shape)
            bpl = BYTES_PER_LU[len(shape)][st]
            out["throughput"].setdefault(label, {})[st] = {
                "mlups": round(nodes * k / dev / 1e6, 1), "bytes_per_update": bpl,
                "achieved_GBs": round(bpl * nodes / (dev / k) / 1e9, 1)}
            _log(f"throughput {label} {st}: {out['throughput'][label][st]}")

    shape = (n, n, n)
    tr = {"workload": f"3-D side-heated cavity, Ra=1e7, Pr=0.71, {n}^3 tanh mesh (a=1.5), "
                      "D3Q19+D3Q7, Ma=0.1, from rest", "steps": steps, "runs": {}}
    ref = None
    for st in kinds:
        cav, H, uf = make_cavity("tanh", shape, storage=st, Ra=1e7, u_f=0.0)
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(2000, steps - done)
            cav.step(k)
            cav.sync()
            done += k
            _log(f"transient {st}: {done}/{steps} steps, {time.perf_counter() - t0:.0f}s")
        stats = cav.stats(allow_nonfinite=True)
        cav.close()
        rec = {"stats": {k: stats[k] for k in keys + ("mass",)}}
        if st == "fp64":
            ref = rec["stats"]
        else:
            rec["rel_err_vs_fp64"] = {k: abs(rec["stats"][k] - ref[k]) / abs(ref[k]) for k in keys}
        tr["runs"][st] = rec
    out["transient"] = tr

    sp = W.mesh_spacing("erf", 257, 1.5)
    cavs = [pkg.Cavity([sp, sp], 1e7, PR, storage=st, use_torch_buffers=False, own_stream=True)
            for st in kinds]
    t0 = time.perf_counter()

    def log(done, h):
        if done % 200000 == 0:
            _log(f"steady step {done} t={time.perf_counter() - t0:.0f}s "
                 f"nu_hot={[round(x[-1][1], 5) for x in h]}")

    hs = W.run_concurrent(cavs, steady_steps, 20000, log=log)
    finals = [c.stats(allow_nonfinite=True) for c in cavs]
    for c in cavs:
        c.close()
    nu_ref = finals[0]["nu_hot"]
    sd = {"workload": "2-D side-heated cavity, Ra=1e7, Pr=0.71, 257^2 erf mesh (a=1.5), Ma=0.1, "
                      "from rest", "steps": steady_steps, "runs": {}}
    for st, h, fin in zip(kinds, hs, finals):
        rec = {"stats": {k: fin[k] for k in keys if k != "wmax"},
               "steps_within_1e-3_of_fp64": W.steps_within([(r[0], r[1]) for r in h], nu_ref)}
        if st != "fp64":
            rec["rel_err_vs_fp64"] = {k: abs(fin[k] - finals[0][k]) / abs(finals[0][k])
                                      for k in keys if k != "wmax"}
        sd["runs"][st] = rec
    out["steady"] = sd
    return out


def _wall_coords(sp):
    """Fluid-node coordinates measured from the first wall, in units of the
    wall-to-wall extent (meshes of different N then share one frame)."""
    import numpy as np

    X = np.concatenate([[0.0], np.cumsum(sp)])
    w0 = 0.5 * (X[0] + X[1])
    return (X[1:-1] - w0) / (0.5 * (X[-1] + X[-2]) - w0)


def richardson(fc: float, fm: float, ff: float, r: float):
    """Observed order p, extrapolated value and fine-mesh GCI in percent
    (safety factor 1.25) from a coarse, medium and fine mesh refined by the
    constant ratio r (Sec. 3; r = 2 for the 2-D table, r = 1.41 for the 3-D
    table of Sec. 4)."""
    p = math.log(abs((fc - fm) / (fm - ff))) / math.log(r)
    rp = r ** p
    return p, (rp * ff - fm) / (rp - 1), 1.25 * abs((ff - fm) / ff) / (rp - 1) * 100


def converge(cav, max_steps: int, tol: float = 1e-9, interval: int = 2000,
             check: int = 50000, tag: str = ""):
    """Runs until the Sec. 3 steady-state measure over `interval` steps is
    below `tol` for both u and T (checked every `check` steps)."""
    done, t0 = 0, time.perf_counter()
    du = dT = float("inf")
    while done < max_steps:
        cav.step(check - interval)
        cav.steady_change()
        cav.step(interval)
        du, dT, _ = cav.steady_change()
        done += check
        if done % (10 * check) == 0:
            _log(f"{tag} step {done} du {du:.2e} dT {dT:.2e} t={time.perf_counter() - t0:.0f}s")
        if du < tol and dT < tol:
            break
    return done, du, dT, time.perf_counter() - t0


def convergence_study(Ra: float = 1e6, sizes=(257, 513, 1025), max_steps: int = 4_000_000,
                      storage: str = "fp64") -> dict:
    """Grid convergence of the steady 2-D cavity on erf meshes (a = 1.5)
    refined by 2: each mesh starts from the previous mesh's steady fields
    (interpolated) and runs to the Sec. 3 steady criterion; the observed
    order p and the extrapolated value follow the Richardson formulas of
    Sec. 3, and GCI_fine uses a safety factor of 1.25."""
    import numpy as np
    from scipy.interpolate import RegularGridInterpolator

    import paper_2509_01099_amd as pkg
    from paper_2509_01099_amd import warmstart as W

    keys = ("nu_vol", "nu_hot", "nu_mid", "re_rms")
    uf = 0.1 / 3 ** 0.5
    vals, runs, prev = {}, [], None
    for n in sizes:
        sp = W.mesh_spacing("erf", n, 1.5)
        cav = pkg.Cavity([sp, sp], Ra, PR, storage=storage, use_torch_buffers=False)
        c = _wall_coords(sp)
        if prev is not None:
            pc, pf = prev
            yy, xx = np.meshgrid(c, c, indexing="ij")
            pts = np.column_stack([yy.ravel(), xx.ravel()])
            init = {}
            for k in ("ux", "uy", "T"):
                ip = RegularGridInterpolator((pc, pc), pf[k], method="linear", bounds_error=False,
                                             fill_value=None)
                init[k] = ip(pts).reshape(n, n)
            # velocities scale with u_f in every mesh's own lattice units
            cav.init_fields(init["ux"], init["uy"], None, init["T"])
        steps, du, dT, secs = converge(cav, max_steps, tag=f"{n}^2")
        st = cav.stats()
        f = cav.fields()
        prev = (c, {k: f[k] for k in ("ux", "uy", "T")})
        vals[n] = {k: st[k] for k in keys}
        runs.append({"n": n, "steps": steps, "du": du, "dT": dT, "seconds": round(secs, 1),
                     "mlups": round(n * n * steps / secs / 1e6, 1), **vals[n]})
        _log(f"{n}^2: {runs[-1]}")
        cav.close()
    out = {"workload": f"2-D cavity Ra={Ra:g} Pr=0.71, erf meshes a=1.5, {storage}, "
                       "each refined mesh initialised from the previous steady fields",
           "runs": runs}
    if len(sizes) == 3:
        a, b, c3 = sizes
        rich = {}
        for k in keys:
            p, finf, gci = richardson(vals[a][k], vals[b][k], vals[c3][k], 2.0)
            rich[k] = {"p": p, "extrapolated": finf, "gci_fine_pct": gci}
        out["richardson"] = rich
    return out


# Sec. 4 table (3-D cavity, erf meshes a = 1.5): <Nu>, Nu_hot, Nu_cold, <Re>
# of the present ISLBM per (Ra, N).
TABLE_3D = {(1e5, 129): (4.3406, 4.3624, 4.3624, 39.4521),
            (1e5, 181): (4.3363, 4.3520, 4.3520, 39.3768),
            (1e5, 257): (4.3346, 4.3457, 4.3457, 39.3500),
            (1e6, 181): (8.6601, 8.6931, 8.6931, 97.4828),
            (1e6, 257): (8.6441, 8.6669, 8.6668, 97.0075),
            (1e6, 361): (8.6379, 8.6540, 8.6540, 96.8464),
            (1e7, 181): (16.5341, 16.6161, 16.6158, 237.3925),
            (1e7, 257): (16.4179, 16.4681, 16.4680, 230.7625),
            (1e7, 361): (16.3670, 16.4001, 16.4001, 228.4148)}


def converge_stats(cav, max_steps: int, tol: float = 1e-8, check: int = 20000, lag: int = 2,
                   tag: str = ""):
    """Steady criterion for storage with stochastic rounding: runs until
    <Nu>, Nu_hot and Re (rms) change by less than `tol` (relative) over the
    last `lag` checks of `check` steps.  The rounding noise is independent
    from node to node and step to step, so it averages out of the domain
    integrals but not out of the node-wise Sec. 3 measure, which is logged
    alongside."""
    keys = ("nu_vol", "nu_hot", "re_rms")
    done, t0, hist = 0, time.perf_counter(), []
    du = dT = float("inf")
    while done < max_steps:
        cav.step(check - 2000)
        cav.steady_change()
        cav.step(2000)
        du, dT, _ = cav.steady_change()
        done += check
        st = cav.stats()
        hist.append([st[k] for k in keys])
        rel = (max(abs(a / b - 1) for a, b in zip(hist[-1], hist[-1 - lag]))
               if len(hist) > lag else float("inf"))
        _log(f"{tag} step {done} nu_vol {st['nu_vol']:.8f} change {rel:.1e} du {du:.1e} "
             f"dT {dT:.1e} t={time.perf_counter() - t0:.0f}s")
        if rel < tol:
            break
    return done, rel, du, dT, time.perf_counter() - t0


def convergence_3d(Ra: float = 1e5, sizes=(129, 181, 257), storage: str = "fp32sr",
                   max_steps=(600_000, 600_000, 600_000), init_file: str = "",
                   save_file: str = "", prior: dict = None) -> dict:
    """Grid convergence of the steady 3-D cavity on the erf meshes of the
    Sec. 4 table (a = 1.5): the coarsest mesh starts at rest, each finer mesh
    from the previous mesh's steady fields (trilinear interpolation), each is
    run until its integrals are steady; Richardson extrapolation and GCI with
    the table's refinement ratio r = 1.41 over the last three meshes.
    A study can be split over several processes: `save_file` keeps the last
    mesh's steady fields (FP16, an initial guess only), `init_file` starts the
    first mesh from them, and `prior` (an earlier output) supplies the runs of
    the coarser meshes."""
    import numpy as np
    from scipy.interpolate import RegularGridInterpolator

    import paper_2509_01099_amd as pkg
    from paper_2509_01099_amd import warmstart as W

    keys = ("nu_vol", "nu_hot", "nu_cold", "re_rms")
    vals, runs, prev = {}, [], None
    for r in (prior or {}).get("runs", []):
        runs.append(r)
        vals[r["n"]] = {k: r[k] for k in keys}
    if init_file:
        with np.load(init_file, allow_pickle=False) as z:
            prev = (z["c"], {k: z[k].astype(np.float64) for k in ("ux", "uy", "uz", "T")})
    for n, cap in zip(sizes, max_steps):
        sp = W.mesh_spacing("erf", n, 1.5)
        cav = pkg.Cavity([sp, sp, sp], Ra, PR, storage=storage)
        c = _wall_coords(sp)
        if prev is not None:
            pc, pf = prev
            zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
            pts = np.column_stack([zz.ravel(), yy.ravel(), xx.ravel()])
            del zz, yy, xx
            init = {}
            for k in ("ux", "uy", "uz", "T"):
                init[k] = RegularGridInterpolator((pc, pc, pc), pf[k], bounds_error=False,
                                                  fill_value=None)(pts).reshape(n, n, n)
                _log(f"{n}^3: interpolated {k}")
            del pts
            cav.init_fields(init["ux"], init["uy"], init["uz"], init["T"])
            del init
        steps, rel, du, dT, secs = converge_stats(cav, cap, tag=f"{n}^3")
        st = cav.stats()
        f = cav.fields()
        prev = (c, {k: f[k] for k in ("ux", "uy", "uz", "T")})
        del f
        vals[n] = {k: st[k] for k in keys}
        row = {"n": n, "steps": steps, "integral_change": rel, "du": du, "dT": dT,
               "seconds": round(secs, 1), "mlups": round(n ** 3 * steps / secs / 1e6, 1),
               **vals[n]}
        ref = TABLE_3D.get((Ra, n))
        if ref:
            row["paper"] = dict(zip(("nu_vol", "nu_hot", "nu_cold", "re"), ref))
        runs.append(row)
        _log(f"{n}^3: {row}")
        cav.close()
    if save_file and prev is not None:
        np.savez(save_file, c=prev[0], **{k: v.astype(np.float16) for k, v in prev[1].items()})
    out = {"workload": f"3-D cavity Ra={Ra:g} Pr=0.71, erf meshes a=1.5, {storage}, coarsest "
                       "from rest, each finer mesh from the previous steady fields",
           "runs": runs}
    done = [r["n"] for r in runs]
    if len(done) >= 3:
        last = done[-3:]
        out["richardson_meshes"] = last
        out["richardson"] = {}
        for k in keys:
            try:
                p, finf, gci = richardson(*(vals[n][k] for n in last), 1.41)
            except (ValueError, ZeroDivisionError):     # not monotone in N, or equal
                p = finf = gci = None
            out["richardson"][k] = {"p": p, "extrapolated": finf, "gci_fine_pct": gci}
    return out


def validation_3d(n: int = 129, Ra: float = 1e5, max_steps: int = 1_200_000,
                  storage: str = "fp64") -> dict:
    """Steady 3-D cavity on the paper's erf mesh (a = 1.5) run to the Sec. 3
    steady criterion, against the Sec. 4 table values for the same mesh."""
    import paper_2509_01099_amd as pkg

    table = {(129, 1e5): {"nu_vol": 4.3406, "nu_hot": 4.3624, "nu_cold": 4.3624, "re": 39.4521}}
    sp = pkg.islbm_mesh_spacing("erf", n, 1.5)
    sp = sp / sp[0]
    cav = pkg.Cavity([sp, sp, sp], Ra, PR, storage=storage)
    steps, du, dT, secs = converge(cav, max_steps, check=20000, tag=f"{n}^3")
    st = cav.stats()
    cav.close()
    out = {"workload": f"3-D cavity Ra={Ra:g} Pr=0.71, {n}^3 erf mesh a=1.5, {storage}, from rest",
           "steps": steps, "du": du, "dT": dT, "seconds": round(secs, 1),
           "stats": {k: st[k] for k in ("nu_vol", "nu_hot", "nu_cold", "re_vol", "re_rms")}}
    ref = table.get((n, Ra))
    if ref:
        out["paper"] = ref
        out["rel_diff"] = {"nu_vol": st["nu_vol"] / ref["nu_vol"] - 1,
                           "nu_hot": st["nu_hot"] / ref["nu_hot"] - 1,
                           "nu_cold": st["nu_cold"] / ref["nu_cold"] - 1,
                           "re_rms": st["re_rms"] / ref["re"] - 1,
                           "re_vol": st["re_vol"] / ref["re"] - 1}
    return out


def throughput_table() -> dict:
    """MLUPS and algorithmic TB/s of every storage type on the 2-D benchmark
    mesh (1024^2 cosine, Ra 1e8), beyond the cache (4096^2) and on the 3-D
    meshes (256^3 and 384^3 tanh, Ra 1e7), with the uniform meshes of the same
    sizes; device events over the timed launches, from rest."""
    cases = [("cosine", (1024, 1024), st, k) for st, k in
             (("fp32", 3000), ("fp64", 1500), ("fp32sr", 1500), ("fp16", 3000), ("bf16", 3000))]
    cases.append(("uniform", (1024, 1024), "fp32", 3000))
    cases += [("cosine", (4096, 4096), st, k) for st, k in
              (("fp32", 300), ("fp64", 150), ("fp32sr", 300), ("fp16", 300), ("bf16", 300))]
    cases.append(("uniform", (4096, 4096), "fp32", 300))
    cases += [("tanh", (256, 256, 256), st, k) for st, k in
              (("fp32", 300), ("fp64", 150), ("fp32sr", 200), ("fp16", 300))]
    cases += [("uniform", (256, 256, 256), st, k) for st, k in (("fp32", 300), ("fp16", 300), ("bf16", 300))]
    cases += [("tanh", (384, 384, 384), st, k) for st, k in
              (("fp32", 100), ("fp64", 50), ("fp32sr", 60), ("fp16", 100), ("bf16", 100))]
    cases += [("uniform", (384, 384, 384), st, k) for st, k in (("fp32", 100), ("fp16", 100), ("bf16", 100))]
    rows = []
    for kind, shape, st, steps in cases:
        three = len(shape) == 3
        cav, _, _ = make_cavity(kind, shape, storage=st, Ra=1e7 if three else RA,
                                **({"u_f": 0.0} if three else {}))
        _, dev = time_run(cav, steps, 10)
        bad = cav.stats(allow_nonfinite=True)["nonfinite"]
        cav.close()
        nodes = math.prod(shape)
        mlups = nodes * steps / dev / 1e6
        rows.append({"mesh": kind, "shape": list(shape), "storage": st, "steps": steps,
                     "mlups": round(mlups, 1),
                     "algorithmic_TBs": round(mlups * 1e6 * BYTES_PER_LU[len(shape)][st] / 1e12, 3),
                     "nonfinite": bad})
        _log(f"{kind} {shape} {st}: {rows[-1]['mlups']} MLUPS")
    return {"study": "throughput of every storage type (one MI355X)", "rows": rows}


def _log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


# The paper's two performance cases (erf meshes, a = 2.1, Pr = 0.71, Ma = 0.1)
# with its wall-clock time per free-fall time on one A100 in FP64 (Sec. 3 and
# Sec. 4); steps timed per case.
PAPER_WCTPDT = ((2, 8193, 1e8, 1.5722e4, 400), (3, 400, 1e7, 1.456e3, 200))


def wctpdt_study(storages=("fp64", "fp32sr", "fp32", "fp16")) -> dict:
    """Wall-clock time per dimensionless time (Eq. 27) on the paper's two
    performance cases, with the uniform mesh of the same node count beside
    each.  One free-fall time t_f = H/u_f takes H_lu/u_f steps, so WCTpDT is
    the measured time per step (device events over the timed launches) times
    H_lu/u_f.  The cavities start at rest; the step's cost does not depend on
    the flow."""
    import paper_2509_01099_amd as pkg

    uf = 0.1 / 3 ** 0.5
    rows = []
    for dim, n, Ra, paper_s, steps in PAPER_WCTPDT:
        for st in storages:
            pair = {}
            for kind in ("erf", "uniform"):
                sp = pkg.islbm_mesh_spacing(kind, n, 2.1)
                sp = sp / sp[0]
                cav = pkg.Cavity([sp] * dim, Ra, PR, storage=st, u_f=uf)
                H = cav.info["H_lu"]
                _, dev = time_run(cav, steps, 20)
                bad = cav.stats(allow_nonfinite=True)["nonfinite"]
                cav.close()
                per = dev / steps
                nodes = n ** dim
                row = {"dim": dim, "n": n, "Ra": Ra, "mesh": kind, "storage": st,
                       "H_lu": round(H, 3), "steps_per_tf": round(H / uf, 1),
                       "ms_per_step": round(per * 1e3, 4),
                       "mlups": round(nodes / per / 1e6, 1),
                       "wctpdt_s": round(per * H / uf, 2), "nonfinite": bad}
                if kind == "erf":
                    row["paper_a100_fp64_s"] = paper_s
                    row["paper_over_ours"] = round(paper_s / row["wctpdt_s"], 2)
                pair[kind] = row
                rows.append(row)
                _log(f"{dim}-D {n}^{dim} {kind} {st}: {row['mlups']} MLUPS, "
                     f"WCTpDT {row['wctpdt_s']} s")
            pair["erf"]["mlups_over_uniform"] = round(pair["erf"]["mlups"] /
                                                      pair["uniform"]["mlups"], 3)
            pair["erf"]["wctpdt_over_uniform"] = round(pair["erf"]["wctpdt_s"] /
                                                       pair["uniform"]["wctpdt_s"], 3)
    return {"study": "WCTpDT on the paper's performance cases (erf a=2.1, Ma=0.1, "
                     "from rest; one MI355X)", "rows": rows}


def _ws_setup(n: int):
    from paper_2509_01099_amd import warmstart as W

    return W.mesh_spacing("erf", n, 1.5), W.draw_ra(40), 0.1 / 3 ** 0.5


def _ws_run(sp, ras, uf, steps, ids, st, t0, init=None, tag="cold"):
    """Runs the cavities of Ra indices `ids` concurrently (own streams) from
    rest or from the network's prediction; histories carry (step, Nu_hot,
    <Nu>, Re_rms, du, dT) every 20 000 steps."""
    import paper_2509_01099_amd as pkg
    from paper_2509_01099_amd import warmstart as W

    cavs = [pkg.Cavity([sp, sp], float(ras[i]), PR, storage=st, use_torch_buffers=False,
                       own_stream=True) for i in ids]
    init_nu = []
    if init is not None:
        for i, c in zip(ids, cavs):
            W.predict_init(init, c, sp, float(ras[i]), uf)
            init_nu.append(c.stats()["nu_hot"])

    def log(done, h):
        if done % 200000 == 0:
            _log(f"{tag} {st} Ra#{ids[0]}..{ids[-1]} step {done} t={time.perf_counter() - t0:.0f}s "
                 f"nu_hot={[round(x[-1][1], 4) for x in h]}")

    hs = W.run_concurrent(cavs, steps, 20000, log=log, steady_interval=2000)
    return cavs, hs, init_nu


def warmstart_cold(steps: int, n: int, ids, storage: str = "fp64", n_train: int = 32,
                   sub: int = 2, group: int = 16, out_path: str | None = None):
    """Cold solves from rest of the Ra indices `ids` (`group` at a time);
    returns their histories and, for training indices, the steady fields at
    every sub-th node (optionally written to out_path as .npz)."""
    import numpy as np

    from paper_2509_01099_amd import warmstart as W

    sp, ras, uf = _ws_setup(n)
    t0 = time.perf_counter()
    hist, fields = {}, {}
    for b in range(0, len(ids), group):
        part = list(ids[b:b + group])
        cavs, hs, _ = _ws_run(sp, ras, uf, steps, part, storage, t0)
        for i, c, h in zip(part, cavs, hs):
            hist[i] = h
            if i < n_train:
                fields[i] = W.fields_star(c, uf).reshape(n, n, 3)[::sub, ::sub].reshape(-1, 3)
            c.close()
    if out_path:
        tr = sorted(fields)
        np.savez_compressed(out_path, ids=np.array(sorted(hist)), n=n, steps=steps, sub=sub,
                            hist=np.array([hist[i] for i in sorted(hist)], dtype=np.float64),
                            train_ids=np.array(tr, dtype=np.int64),
                            fields=np.array([fields[i] for i in tr], dtype=np.float16))
    return hist, fields


def warmstart_study(steps: int, n: int = 257, n_train: int = 32, n_test: int = 8,
                    storage: str = "fp64", train_steps: int = 6000, sub: int = 2,
                    data_dir: str | None = None, warm_steps: int | None = None) -> dict:
    """Learned warm start on the 2-D cavity (n^2 erf mesh a = 1.5, Pr = 0.71,
    Ma = 0.1) at seeded log-uniform Ra in [1e6, 1e8].  Cold solves from rest
    (16 cavities at a time, each on its own stream) give the training fields
    (every sub-th node) and the steady Nusselt numbers; the network is
    trained on the first n_train; the n_test held-out cavities are then
    started from its prediction.  Criterion: steps until Nu_hot stays within
    1e-3 of the cold-start steady value.  The same held-out cases are also
    run with FP32 storage (cold and warm) against the same reference.  With
    data_dir, the cold solves are read from the .npz files that
    `--ws-phase cold` wrote there instead of being run.  warm_steps (default
    steps) bounds the warm runs; a run that never meets the criterion counts
    as `steps`."""
    import glob

    import numpy as np
    import torch

    from paper_2509_01099_amd import warmstart as W

    sp, ras, uf = _ws_setup(n)
    t0 = time.perf_counter()
    ids = list(range(n_train + n_test))
    if data_dir:
        hist, fields = {}, {}
        for path in sorted(glob.glob(os.path.join(data_dir, f"ws{n}_cold_*.npz"))):
            d = np.load(path)
            assert int(d["n"]) == n and int(d["steps"]) == steps and int(d["sub"]) == sub, path
            for i, h in zip(d["ids"], d["hist"]):
                hist[int(i)] = [tuple(r) for r in h]
            for i, f in zip(d["train_ids"], d["fields"]):
                fields[int(i)] = f.astype(np.float32)
        missing = [i for i in ids if i not in hist]
        assert not missing, f"cold solves missing for Ra indices {missing}"
    else:
        hist, fields = warmstart_cold(steps, n, ids, storage, n_train, sub)
    inputs = [W.node_inputs(sp, float(ras[i]), sub) for i in range(n_train)]
    targets = [fields[i] for i in range(n_train)]
    ref = {i: hist[i][-1][1] for i in ids}
    cold_steady = {i: W.steps_to_steady(hist[i]) for i in ids}
    # how settled the cold references are: change over the last 10 % of the run
    k10 = max(1, len(hist[0]) // 10)
    settle = max(abs(hist[i][-1][1] - hist[i][-1 - k10][1]) / abs(ref[i]) for i in ids)

    net = W.WarmStartMLP()
    inp = torch.tensor(np.concatenate(inputs), device="cuda")
    tgt = torch.tensor(np.concatenate(targets), device="cuda")
    t1 = time.perf_counter()
    losses = net.train(inp, tgt, steps=train_steps, batch=8192, log_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    _log(f"trained {train_steps} steps in {t_train:.1f}s, loss {losses[0][1]:.3e} -> {losses[-1][1]:.3e}")
    p = torch.tensor(W.node_inputs(sp, 1e7), device="cuda")
    net.predict(p)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(20):
        net.predict(p)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t2) / 20
    dims = net.dims
    flops = 2 * p.shape[0] * sum(dims[i] * dims[i + 1] for i in range(len(dims) - 1))

    test = ids[n_train:]
    runs, init_nu = {}, {}
    for st in (storage, "fp32"):
        if st != storage:
            cavs, hs, _ = _ws_run(sp, ras, uf, steps, test, st, t0, tag="cold")
            runs[(st, "cold")] = hs
            for c in cavs:
                c.close()
        else:
            runs[(st, "cold")] = [hist[i] for i in test]
        cavs, hs, init_nu[st] = _ws_run(sp, ras, uf, warm_steps or steps, test, st, t0, init=net,
                                        tag="warm")
        runs[(st, "warm")] = hs
        for c in cavs:
            c.close()
    rows = []
    for k, i in enumerate(test):
        row = {"Ra": float(ras[i]), "nu_hot_steady": ref[i]}
        for st in (storage, "fp32"):
            for how in ("cold", "warm"):
                h = runs[(st, how)][k]
                row[f"{st}_{how}_steps"] = W.steps_within([(r[0], r[1]) for r in h], ref[i])
                row[f"{st}_{how}_end_rel_err"] = abs(h[-1][1] - ref[i]) / ref[i]
                row[f"{st}_{how}_steady_steps"] = W.steps_to_steady(h)
                row[f"{st}_{how}_min_du_dT"] = [min(r[-2] for r in h), min(r[-1] for r in h)]
            row[f"{st}_warm_initial_rel_err"] = abs(init_nu[st][k] - ref[i]) / ref[i]
        rows.append(row)

    def total(st, how):
        return sum(r[f"{st}_{how}_steps"] or steps for r in rows)

    out = {"study": f"learned warm start, 2-D cavity {n}^2 erf (a=1.5), Pr 0.71, Ma 0.1, "
                    f"{n_train} training / {n_test} held-out Ra log-uniform in [1e6, 1e8]",
           "criterion": "steps until Nu_hot stays within 1e-3 of the cold-start steady value "
                        f"({storage} storage, {steps} cold / {warm_steps or steps} warm steps)",
           "cold_reference_settle_last10pct": settle,
           "steady_criterion": "Sec. 3: relative change of u and T over 2000 steps below 1e-9",
           "cold_steps_to_steady_criterion_all": [cold_steady[i] for i in ids],
           "seconds": round(time.perf_counter() - t0, 1),
           "train": {"samples": int(inp.shape[0]), "steps": train_steps, "batch": 8192,
                     "seconds": round(t_train, 1), "loss_first": losses[0][1],
                     "loss_last": losses[-1][1]},
           "inference": {"nodes": int(p.shape[0]), "ms": round(t_inf * 1e3, 3),
                         "gemm_tflops": round(flops / t_inf / 1e12, 2)},
           "held_out": rows}
    for st in (storage, "fp32"):
        out[f"{st}_cold_total_steps"] = total(st, "cold")
        out[f"{st}_warm_total_steps"] = total(st, "warm")
        out[f"{st}_speedup_steps"] = total(st, "cold") / total(st, "warm")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline and uniform lines (no copy ceiling, FP64 row, "
                         "HBM rows or warm-start block)")
    ap.add_argument("--precision", type=int, default=0, metavar="STEPS",
                    help="reduced-precision storage study instead of the headline line: "
                         "3-D 384^3 tanh cavity, Ra 1e7, FP64/FP32/FP16/BF16, STEPS steps "
                         "from rest, MLUPS and Nu/Re/peak-velocity errors against FP64")
    ap.add_argument("--warmstart", type=int, default=0, metavar="STEPS",
                    help="learned warm start study instead of the headline line: cold solves "
                         "of STEPS steps give the training fields, then warm and cold starts "
                         "are compared on held-out Rayleigh numbers")
    ap.add_argument("--ws-n", type=int, default=257, help="warm-start mesh size (erf, a=1.5)")
    ap.add_argument("--ws-phase", choices=["all", "cold", "eval"], default="all",
                    help="'cold' runs the cold solves of one batch of Ra indices and writes "
                         "<ws-dir>/ws<n>_cold_<batch>.npz; 'eval' reads those files from "
                         "--ws-dir and does training and the warm/cold comparison")
    ap.add_argument("--ws-batch", type=int, default=0)
    ap.add_argument("--ws-batch-size", type=int, default=8)
    ap.add_argument("--ws-dir", default=os.path.join(ROOT, "ws_out"),
                    help="directory of the cold-solve files of --ws-phase cold / eval")
    ap.add_argument("--ws-warm-steps", type=int, default=0,
                    help="steps of the warm runs (default: as many as the cold solves)")
    ap.add_argument("--convergence", type=float, default=0.0, metavar="RA",
                    help="grid-convergence study instead of the headline line: 2-D cavity at "
                         "this Ra on erf meshes 257/513/1025 (1e6) or 513/1025/2049, FP64, "
                         "run to the steady criterion; observed order and extrapolation")
    ap.add_argument("--throughput", action="store_true",
                    help="MLUPS of every storage type on the 2-D and 3-D benchmark meshes")
    ap.add_argument("--wctpdt", action="store_true",
                    help="wall-clock time per free-fall time on the paper's performance cases "
                         "(2-D 8193^2 Ra 1e8, 3-D 400^3 Ra 1e7, erf a=2.1) and their uniform "
                         "meshes, FP64 / FP32SR / FP32 / FP16")
    ap.add_argument("--convergence3d", type=float, default=0.0, metavar="RA",
                    help="3-D grid-convergence study at this Ra on the erf meshes of the paper's "
                         "3-D table (1e5: 129/181/257), FP32 storage with FP64 arithmetic")
    ap.add_argument("--c3-sizes", default="",
                    help="comma-separated mesh sizes of --convergence3d (default: the table's)")
    ap.add_argument("--c3-save", default="", metavar="NPZ",
                    help="--convergence3d: save the last mesh's steady fields (FP16) here")
    ap.add_argument("--c3-init", default="", metavar="NPZ",
                    help="--convergence3d: start the first mesh from fields saved by --c3-save")
    ap.add_argument("--c3-caps", default="",
                    help="--convergence3d: comma-separated step caps per mesh")
    ap.add_argument("--c3-prior", default="", metavar="JSON",
                    help="--convergence3d: an earlier output whose runs precede these meshes")
    ap.add_argument("--validation3d", action="store_true",
                    help="steady 3-D cavity (129^3 erf, Ra 1e5, FP64) against the paper's table")
    ap.add_argument("--profile-mesh", choices=sorted(PROFILE_MESHES), default="2d",
                    help="workload of --profile: 2d = the benchmark mesh (1024^2 cosine, Ra "
                         "1e8), 2d-4096 = 4096^2 cosine, 3d = 256^3 tanh (Ra 1e7), 3d-384 = "
                         "384^3 tanh, 3d-uniform = 256^3 uniform")
    ap.add_argument("--profile-storage", choices=["fp32", "fp64", "fp16", "bf16", "fp32sr"],
                    default="fp32", help="storage type of --profile")
    ap.add_argument("--profile", action="store_true",
                    help="short run of one workload's step kernel only, plus a 1 GiB copy for "
                         "counter calibration (for rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path, so --gpus "
              "must be 1", file=sys.stderr)
        return 2
    import torch

    import paper_2509_01099_amd as pkg

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    pkg.load()
    n = (N_CFG, N_CFG)
    nodes = N_CFG * N_CFG

    if args.convergence3d:
        sizes = tuple(int(v) for v in args.c3_sizes.split(",")) if args.c3_sizes else (
            (129, 181, 257) if args.convergence3d < 5e5 else (181, 257, 361))
        caps = (tuple(int(v) for v in args.c3_caps.split(",")) if args.c3_caps
                else (600_000, 500_000, 450_000)[:len(sizes)])
        prior = None
        if args.c3_prior:
            with open(args.c3_prior) as f:
                prior = json.loads(f.read().strip().splitlines()[-1])
        print(json.dumps(convergence_3d(args.convergence3d, sizes, max_steps=caps,
                                        init_file=args.c3_init, save_file=args.c3_save,
                                        prior=prior)))
        return 0
    if args.throughput:
        print(json.dumps(throughput_table()))
        return 0
    if args.wctpdt:
        print(json.dumps(wctpdt_study()))
        return 0
    if args.validation3d:
        print(json.dumps(validation_3d()))
        return 0
    if args.convergence:
        sizes = (257, 513, 1025) if args.convergence < 5e6 else (513, 1025, 2049)
        print(json.dumps(convergence_study(args.convergence, sizes)))
        return 0
    if args.warmstart:
        if args.ws_phase == "cold":
            ids = list(range(40))[args.ws_batch * args.ws_batch_size:
                                  (args.ws_batch + 1) * args.ws_batch_size]
            out_dir = args.ws_dir
            os.makedirs(out_dir, exist_ok=True)
            path = os.path.join(out_dir, f"ws{args.ws_n}_cold_{args.ws_batch}.npz")
            hist, _ = warmstart_cold(args.warmstart, args.ws_n, ids, out_path=path)
            print(json.dumps({"phase": "cold", "ids": ids, "file": path,
                              "final_nu_hot": [hist[i][-1][1] for i in ids]}))
            return 0
        print(json.dumps(warmstart_study(args.warmstart, n=args.ws_n,
                                         data_dir=args.ws_dir if args.ws_phase == "eval" else None,
                                         warm_steps=args.ws_warm_steps or None)))
        return 0
    if args.precision:
        print(json.dumps(precision_study(args.precision)))
        return 0

    if args.profile:
        kind, shape = PROFILE_MESHES[args.profile_mesh]
        cav, H, uf = make_cavity(kind, shape, storage=args.profile_storage,
                                 Ra=RA if len(shape) == 2 else 1e7)
        nodes = math.prod(shape)
        wall, dev = time_run(cav, args.steps, args.warmup)
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "steps": args.steps,
                          "mlups": nodes * args.steps / dev / 1e6,
                          "copy_bytes": 1 << 30}))
        return 0

    # headline: non-uniform (cosine) mesh, FP32
    cav, H, uf = make_cavity("cosine", n)
    wall, dev, dev_plain, dev_red = time_run_split(cav, args.steps, args.warmup)
    st = cav.stats(allow_nonfinite=True)
    cav.close()
    mlups = nodes * args.steps / wall / 1e6
    per_plain = dev_plain / (args.steps - 1) if args.steps > 1 else dev
    bpl = BYTES_PER_LU[2]["fp32"] * nodes
    achieved = bpl / per_plain / 1e9
    dig = kernel_digest()
    traffic = traffic_entry(dig)

    # same size, uniform mesh (plain-shift kernel)
    ucav, uH, uuf = make_cavity("uniform", n)
    uwall, udev, udev_plain, _ = time_run_split(ucav, args.steps, args.warmup)
    ucav.close()
    umlups = nodes * args.steps / uwall / 1e6
    uper = udev_plain / (args.steps - 1) if args.steps > 1 else udev

    copy = None if args.headline_only else copy_ceiling()
    cgbs = copy["copy_ceiling_GBs"] if copy else None
    rows, fp64_row, ws = [], None, None
    if not args.headline_only:
        fp64_row = step_row("2-D 1024^2 cosine, Ra 1e8 (FP64, the paper's precision)", "cosine",
                            n, "fp64", 2000, copy_GBs=cgbs)
        _log(f"fp64 row: {fp64_row}")
        for label, kind, shape, storage, k in HBM_ROWS:
            rows.append(step_row(label, kind, shape, storage, k, copy_GBs=cgbs))
            _log(f"hbm row: {rows[-1]}")
        ws = warmstart_block()

    cpu = None if args.no_cpu else cpu_baseline()
    out = {
        "metric": "MLUPS (non-uniform 1024^2 cosine mesh) with % HBM roofline; uniform mesh "
                  "of the same size alongside",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (cavity started at rest; no external data)",
        "config": {"workload": "2-D side-heated cavity, Ra=1e8, Pr=0.71, 1024x1024 "
                               "cosine-stretched mesh, D2Q9+D2Q5 MRT, FP32 populations in [z][y][pop][x] rows",
                   "u_f": uf, "H_lu": H, "nodes": nodes,
                   "wctpdt_s": round(wall / args.steps * H / uf, 3),
                   "nonfinite_nodes": st["nonfinite"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "step_kernel<2,Tile<64,4,1,1>,float> (plain launches)",
                     "cache_resident": True,
                     "note": "the two FP32 buffers of the 1024^2 mesh (117 MB) fit the 256 MB "
                             "last-level cache, so part of this traffic is served there; "
                             "hbm_rows holds the workloads beyond the cache",
                     "bytes_per_launch": bpl, "avg_launch_us": round(per_plain * 1e6, 3),
                     "reducing_launch_us": round(dev_red * 1e6, 3),
                     "mlups_plain_launches": round(nodes / per_plain / 1e6, 1)},
        "uniform": {"value": round(umlups, 1), "unit": "MLUPS",
                    "nonuniform_over_uniform": round(mlups / umlups, 4),
                    "plain_launch_us": round(uper * 1e6, 3),
                    "achieved_GBs": round(bpl / uper / 1e9, 1)},
        "cpu_baseline": cpu,
    }
    if copy:
        out["copy_ceiling_GBs"] = cgbs
        out["copies_GBs"] = copy["copies_GBs"]
    if fp64_row:
        out["fp64_row"] = fp64_row
    if rows:
        out["hbm_rows"] = rows
    if ws:
        out["warm_start"] = ws
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
