"""Benchmark of the particle-phase step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3-1m]

One "step" is prs_step_particles on the whole bed: clear the force field,
sort the spheres into cells, multi-direct forcing (interpolate + spread per
iteration), collision search and n_sub contact/Newton-Euler substeps, and the
write-back.  Inputs are synthetic and resident in HBM before timing starts.
Prints one JSON line: the particle-step rate and, beside it, the phase times,
the dominant kernel's roofline figures, the FP64 form, the FP32 + learned vs
FP64 plain comparison and the single-core oracle rate.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-step/s, markers/s, contacts/s; FP32+learned vs FP64 plain at 1e-6 slip"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def params_for(P, W, w, precision, **kw):
    ph = W.PHYS
    nx, ny, nz = w.grid
    d = dict(nx=nx, ny=ny, nz=nz, h=w.h, radius=0.5 * ph["D"], rho_p=ph["rho_p"],
             rho_f=ph["rho_f"], gravity=ph["g"], n_markers=w.n_markers, dt_f=ph["dt_f"],
             alpha=ph["alpha"], n_iter=w.n_iter, n_sub=ph["n_sub"], k_n=ph["k_n"], e_n=ph["e_n"],
             mu=ph["mu"], kt_ratio=ph["kt_ratio"], dt_ratio=ph["dt_ratio"], skin=0.1,
             precision=precision, max_particles=w.n)
    d.update(kw)
    return P.make_params(**d)


def touched_nodes(ctx, x, torch):
    """Grid nodes per component inside at least one marker stencil (spread of
    positive unit forces; every node in a stencil gets a positive weight)."""
    n = x.shape[0]
    F = torch.ones((n, ctx.p.n_markers, 3), dtype=ctx.dtype, device="cuda")
    f = [torch.zeros(s, dtype=ctx.dtype, device="cuda") for s in ctx.grid_shapes()]
    ctx.spread(x, F, f, accumulate=False)
    torch.cuda.synchronize()
    out = [int(torch.count_nonzero(a)) for a in f]
    del F, f
    torch.cuda.empty_cache()
    return out


def ib_bytes(w, n_touched, s):
    """Algorithmic bytes of one forcing iteration by the byte model of the
    method (per iteration: every touched node of each component read once
    for the interpolation and read-modify-written in f and in u** by the
    spreading, 5 s per node; every marker's correction written and read
    across the Jacobi barrier, 6 s per marker), split between the two
    kernels: interpolation N_T s + 3 M s, spreading 4 N_T s + 3 M s, with
    N_T the touched nodes summed over the three components and s the field
    word size."""
    M = w.n * w.n_markers
    NT = sum(n_touched)
    return NT * s + 3 * M * s, 4 * NT * s + 3 * M * s


def lean_bytes(w, n_touched, s, iters):
    """Bytes the library's own design moves per pass (no u** field: the
    first pass stores every node of f, later passes read-modify-write the
    touched nodes of f and read the step's recorded I[u-hat]), for
    comparison with the method's byte model."""
    M = w.n * w.n_markers
    NT = sum(n_touched)
    nx, ny, nz = w.grid
    nodes = nx * ny * nz * 2 + nx * (ny + 1) * nz
    interp = NT * s + M * 3 * s * 2 + w.n * (9 + 2) * 8
    f_bytes = (nodes * s + (iters - 1) * NT * 2 * s) / iters if iters > 0 else 0
    spread = M * 3 * s + f_bytes + w.n * 3 * 8 + w.n * 12 * 8 * 2
    return interp, spread


def dem_bytes(n, directed_contacts_per_substep):
    """Algorithmic bytes of one particle substep: per sphere its state read
    and written and its cell data (160 B), per directed contact its history
    slot read and written (72 B)."""
    return n * 160 + directed_contacts_per_substep * 72


def run_form(P, W, w, bed, precision, steps, warmup, torch, measure_touched=False):
    import numpy as np

    dt = torch.float32 if precision == P.F32 else torch.float64
    modes = W.flow_modes(w, bed.bed_top)
    t0 = time.time()
    uhat = W.fluid_field(w, modes, device="cuda", dtype=dt)
    log(f"field ({dt}) generated in {time.time() - t0:.1f}s")
    f = [torch.zeros_like(a) for a in uhat]
    x0 = torch.as_tensor(bed.x, device="cuda")
    u0 = torch.as_tensor(bed.u, device="cuda")
    om0 = torch.as_tensor(bed.om, device="cuda")
    res = {}
    with P.Context(params_for(P, W, w, precision)) as ctx:
        if measure_touched:
            res["touched"] = touched_nodes(ctx, x0, torch)
            log(f"touched nodes per component: {res['touched']}")
        x, u, om = x0.clone(), u0.clone(), om0.clone()
        # a settled bed starts from its contact history at rest
        H = P.History.from_host(bed.hist) if bed.hist is not None else P.History.zeros(w.n)
        Fh = torch.empty((w.n, 3), dtype=torch.float64, device="cuda")
        Th = torch.empty_like(Fh)
        for k in range(warmup):
            _, _, st = ctx.step(uhat, f, x, u, om, H, Fh, Th, zero_f=True)
            log(f"warmup {k + 1}/{warmup}: iterations {st['iterations']} slip {st['rel_slip']}")
        ctx.timing(True)
        ctx.read_timing(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        contacts = 0
        for k in range(steps):
            _, _, st = ctx.step(uhat, f, x, u, om, H, Fh, Th, zero_f=True)
            contacts += st["contacts"]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tm = ctx.read_timing(reset=True)
        ctx.timing(False)
        log(f"{steps} timed steps in {wall:.3f}s; last stats {st}")
    res.update(wall=wall, timing=tm, stats=st, contacts=contacts)
    del uhat, f
    torch.cuda.empty_cache()
    return res


def time_single_steps(P, ctx, uhat, bed, K, torch):
    """K identical steps from the bed's initial state (the state is copied
    before each step, outside the timed region); returns (ms per step,
    stats of the last step, phase timing per step, F_h of the last step)."""
    x0 = torch.as_tensor(bed.x, device="cuda")
    u0 = torch.as_tensor(bed.u, device="cuda")
    om0 = torch.as_tensor(bed.om, device="cuda")
    n = x0.shape[0]
    f = [torch.empty_like(a) for a in uhat]
    Fh = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    Th = torch.empty_like(Fh)
    H0 = P.History.from_host(bed.hist) if bed.hist is not None else P.History.zeros(n)
    total = 0.0
    ctx.timing(True)
    ctx.read_timing(reset=True)
    for _ in range(K):
        x, u, om = x0.clone(), u0.clone(), om0.clone()
        H = H0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, st = ctx.step(uhat, f, x, u, om, H, Fh, Th, zero_f=True)
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
    tm = ctx.read_timing(reset=True)
    ctx.timing(False)
    del f
    phases = {k[3:]: v / K for k, v in tm.items() if k.startswith("ms_")}
    return total / K * 1e3, st, phases, Fh


def learned_comparison(P, W, w, bed, torch, n_snap, K, tol=1e-6, max_iter=10):
    """FP32 + learned warm start against FP64 plain on the same bed and field,
    both to the relative slip tolerance tol with at most max_iter iterations.

    The network is trained first, on the GPU, on samples of the plain FP32
    forcing (30 iterations) of the 22k-sphere workload: n_snap (bed, flow
    time) snapshots, 2 % of the markers of each, Adam with batch 65,536 for
    2,000 iterations."""
    from paper_2108_01814_amd import learned as L

    res = {"tol": tol, "max_iter": max_iter}
    wt = W.WORKLOADS["c2-22k"]
    t0 = time.time()
    snaps = [(2000 + k // 10, k % 10) for k in range(n_snap)]
    S = L.collect(wt, snaps, n_iter=30, keep=0.02, seed=0,
                  progress=lambda k, st: (k + 1) % 25 == 0 and log(
                      f"training samples: snapshot {k + 1}/{n_snap}"))
    t_collect = time.time() - t0
    t0 = time.time()
    net, norm, losses = L.train(S, iters=2000, batch=65536, lr=1e-3, seed=0, log_every=500,
                                progress=lambda it, l: log(f"training: iteration {it} loss {l:.4f}"))
    torch.cuda.synchronize()
    t_train = time.time() - t0
    held = L.collect(wt, [(9000, 0)], n_iter=30, keep=0.02, seed=1)
    res["training"] = {"workload": wt.name, "snapshots": n_snap, "samples": int(S.X.shape[0]),
                       "adam_iterations": 2000, "batch": 65536, "collect_s": t_collect,
                       "train_s": t_train, "first_loss": losses[0][1], "final_loss": losses[-1][1],
                       "held_out_loss": L.validation_loss(net, held, norm)}
    del S, held
    torch.cuda.empty_cache()
    log(f"trained: {res['training']}")

    modes = W.flow_modes(w, bed.bed_top)
    fields = {P.F32: W.fluid_field(w, modes, device="cuda", dtype=torch.float32),
              P.F64: W.fluid_field(w, modes, device="cuda", dtype=torch.float64)}
    runs = {}

    def form(name, precision, learned, tol_, max_iter_):
        uhat = fields[precision]
        with P.Context(params_for(P, W, w, precision, tol_mode=1, tol=tol_,
                                  max_iter=max_iter_)) as ctx:
            if learned:
                ctx.set_learned(net)
            time_single_steps(P, ctx, uhat, bed, 1, torch)     # warm-up
            ms, st, ph, Fh = time_single_steps(P, ctx, uhat, bed, K, torch)
        torch.cuda.empty_cache()
        r = {"ms_per_step": ms, "iterations": st["iterations"], "rel_slip": st["rel_slip"],
             "rejected_learned": st["rejected_learned"], "phases_ms_per_step": ph}
        log(f"{name}: {ms:.1f} ms/step, {st['iterations']} iterations, "
            f"final slip {st['rel_slip'][-1]:.4g}, rejected {st['rejected_learned']}")
        runs[name] = r
        return r, Fh

    p64, Fh64 = form("fp64_plain", P.F64, False, tol, max_iter)
    Fh64 = Fh64.cpu()
    l32, Fh32 = form("fp32_learned", P.F32, True, tol, max_iter)
    Fh32 = Fh32.cpu()
    p32, _ = form("fp32_plain", P.F32, False, tol, max_iter)
    res.update(runs)
    res["tolerance_reached"] = {k: bool(r["rel_slip"][-1] < tol) for k, r in
                                (("fp64_plain", p64), ("fp32_learned", l32), ("fp32_plain", p32))}
    res["note"] = ("no form reaches the 1e-6 relative slip within the iteration cap (the Jacobi "
                   "multi-direct forcing stalls near 1e-2): times at the cap are at equal "
                   "iteration counts, and the comparisons at equal accuracy below stop each form "
                   "at the slip the other form ends at")
    res["speedup_at_cap"] = p64["ms_per_step"] / l32["ms_per_step"]
    # the learned gain alone: FP32 + learned to the slip FP32 plain ends at
    t32 = p32["rel_slip"][-1]
    e32, _ = form("fp32_learned_to_fp32_plain", P.F32, True, t32 * (1 + 1e-9), max_iter)
    ok32 = e32["rel_slip"][-1] < t32 * (1 + 1e-9)
    res["learned_vs_fp32_plain"] = {
        "target_slip": t32, "reached": bool(ok32),
        "fp32_learned_iterations": e32["iterations"], "fp32_plain_iterations": p32["iterations"],
        "fp32_learned_ms": e32["ms_per_step"], "fp32_plain_ms": p32["ms_per_step"],
        "speedup": p32["ms_per_step"] / e32["ms_per_step"] if ok32 else None}
    res.pop("fp32_learned_to_fp32_plain", None)
    # the precision gain alone: FP32 plain against FP64 plain, the same iterations
    res["fp32_plain_vs_fp64_plain"] = {"speedup": p64["ms_per_step"] / p32["ms_per_step"],
                                       "iterations": p32["iterations"],
                                       "final_slip_fp32": p32["rel_slip"][-1],
                                       "final_slip_fp64": p64["rel_slip"][-1]}
    # equal accuracy: the slip FP64 plain ends at, reached by FP32 + learned
    target = p64["rel_slip"][-1]
    eq, Fh_eq = form("fp32_learned_equal_accuracy", P.F32, True, target * (1 + 1e-9), max_iter)
    reached = eq["rel_slip"][-1] < target * (1 + 1e-9)
    res["equal_accuracy"] = {
        "target_slip": target, "reached": bool(reached),
        "fp32_learned_iterations": eq["iterations"], "fp64_plain_iterations": p64["iterations"],
        "fp32_learned_ms": eq["ms_per_step"], "fp64_plain_ms": p64["ms_per_step"],
        "speedup": p64["ms_per_step"] / eq["ms_per_step"] if reached else None}
    res.pop("fp32_learned_equal_accuracy", None)
    # a looser tolerance, reached by both forms
    a, _ = form("fp64_plain_1e-2", P.F64, False, 1e-2, max_iter)
    b, _ = form("fp32_learned_1e-2", P.F32, True, 1e-2, max_iter)
    c, _ = form("fp32_plain_1e-2", P.F32, False, 1e-2, max_iter)
    res["to_1e-2"] = {"fp64_plain_ms": a["ms_per_step"], "fp64_plain_iterations": a["iterations"],
                      "fp32_plain_ms": c["ms_per_step"], "fp32_plain_iterations": c["iterations"],
                      "fp32_learned_ms": b["ms_per_step"],
                      "fp32_learned_iterations": b["iterations"],
                      "speedup": a["ms_per_step"] / b["ms_per_step"],
                      "learned_vs_fp32_plain": c["ms_per_step"] / b["ms_per_step"]}
    for k in ("fp64_plain_1e-2", "fp32_learned_1e-2", "fp32_plain_1e-2"):
        res.pop(k, None)
    # accuracy: F_h of each form against FP64 plain run to 60 iterations
    ref, Fh_ref = form("fp64_plain_60", P.F64, False, 1e-12, 60)
    Fh_ref = Fh_ref.cpu()
    scale = float(Fh_ref.norm(dim=1).max())

    def err(F):
        return float((F - Fh_ref).norm(dim=1).max()) / scale

    res["force_error_vs_fp64_60_iterations"] = {
        "reference_final_slip": ref["rel_slip"][-1],
        "fp64_plain": err(Fh64), "fp32_learned": err(Fh32),
        "fp32_learned_equal_accuracy": err(Fh_eq.cpu())}
    res.pop("fp64_plain_60", None)
    del fields
    torch.cuda.empty_cache()
    return res


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c3-1m_f32.txt")
KERNEL_SOURCES = ("prs_ib.hip", "prs_stencil.h", "prs_device.h", "prs_internal.h")


def kernel_source_hash():
    """Hash of the kernel sources with comments and blank space removed (a
    change to a comment leaves the kernels, and their counters, as they were)."""
    import hashlib
    import re

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_01814_amd", "csrc", name)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel calibration), or None
    when there is none or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    meta = dict(l[2:].split("=", 1) for l in lines if l.startswith("# ") and "=" in l)
    if meta.get("source_hash") != kernel_source_hash():
        return None
    for l in lines:
        if l.startswith("#") or not l.strip():
            continue
        name, fetch, write = l.split("\t")[:3]
        if name == kernel:
            return float(fetch) + float(write)
    return None


def cpu_baseline(W, w, bed, width=12.0):
    """The FP64 oracle, single-threaded, on a window of the same bed: the
    spheres with centres in a width x Ly x width column, the fluid field on
    that column plus a margin (synthetic field in FP64), one full step."""
    import numpy as np

    import oracle

    ph = W.PHYS
    nx, ny, nz = w.grid
    h = w.h
    x0 = 0.5 * (w.domain[0] - width)
    z0 = 0.5 * (w.domain[2] - width)
    sel = ((bed.x[:, 0] >= x0) & (bed.x[:, 0] < x0 + width) &
           (bed.x[:, 2] >= z0) & (bed.x[:, 2] < z0 + width))
    xs, us, oms = (np.ascontiguousarray(a[sel]) for a in (bed.x, bed.u, bed.om))
    margin = 1.0
    wi0 = int(math.floor((x0 - margin) / h))
    wk0 = int(math.floor((z0 - margin) / h))
    wnx = int(math.ceil((width + 2 * margin) / h))
    wnz = wnx
    # the same generator, evaluated on the window's node columns only (host, FP64)
    modes = W.flow_modes(w, bed.bed_top)
    uh = [np.ascontiguousarray(t.numpy())
          for t in W.fluid_field(w, modes, window=(wi0, wnx, wk0, wnz))]
    po = oracle.make_params(nx=nx, ny=ny, nz=nz, h=h, wi0=wi0 % nx, wnx=wnx, wk0=wk0 % nz,
                            wnz=wnz, R=0.5 * ph["D"], nl=w.n_markers, g=ph["g"],
                            rho_p=ph["rho_p"], rho_f=ph["rho_f"], dt_f=ph["dt_f"],
                            alpha=ph["alpha"], n_iter=w.n_iter, n_sub=ph["n_sub"], k_n=ph["k_n"],
                            e_n=ph["e_n"], mu=ph["mu"], kt_ratio=ph["kt_ratio"],
                            dt_ratio=ph["dt_ratio"], use_cells=1)
    f = [np.zeros_like(a) for a in uh]
    H = oracle.History(len(xs))
    t0 = time.perf_counter()
    rc, out = oracle.step(po, uh, f, xs, us, oms, H)
    t = time.perf_counter() - t0
    return dict(value=len(xs) / t, unit="particle-step/s", cores=1, kind="oracle",
                sample=(f"{len(xs)} spheres ({len(xs) * w.n_markers} markers) with centres in a "
                        f"{width:g}D x {w.domain[1]:g}D x {width:g}D column of the same bed, "
                        f"one full step ({w.n_iter} forcing iterations, {ph['n_sub']} substeps), "
                        f"FP64, {t:.1f}s"), rc=rc, host=host_description())


def host_description():
    """CPU model, logical CPUs and memory of the host that ran the oracle."""
    model, mem_gb = None, None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    mem_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "mem_gib": mem_gb}


def copy_rate(torch, nbytes=2 << 30, reps=5):
    """Measured device-to-device copy rate (bytes read + written per second)
    of a plain torch copy of nbytes, best of reps: the achievable HBM rate
    beside the 8 TB/s specification."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (best / 1e3) / 1e9


def roofline_block(w, r, s, K, copy_gbs, tname):
    """Roofline figures of one form of the step (field word size s): each
    IB kernel's share of the method's byte model per launch over its mean
    launch time (HIP events on the library's stream), the forcing iteration,
    the particle substeps and the whole step against the HBM peak; the
    dominant kernel is the one with the larger time per step."""
    import paper_2108_01814_amd as P  # noqa: F401  (the library is loaded by the caller)
    from paper_2108_01814_amd import workloads as W

    tm = r["timing"]
    iters = r["stats"]["iterations"]
    n_sub = W.PHYS["n_sub"]
    b_interp, b_spread = ib_bytes(w, r["touched"], s)
    l_interp, l_spread = lean_bytes(w, r["touched"], s, iters)
    avg_interp = tm["ms_interp"] / max(tm["n_interp"], 1)
    avg_spread = tm["ms_spread"] / max(tm["n_spread"], 1)
    nb = 2 * math.ceil(0.5 * W.PHYS["D"] / w.h - 1e-9) + 4
    kern = {f"prs::k_interp<{tname}, 0, {nb}>": ("interpolation", b_interp, avg_interp,
                                                 tm["ms_interp"]),
            f"prs::k_spread_tiles<{tname}, 0, false>": ("spreading", b_spread, avg_spread,
                                                 tm["ms_spread"])}
    dom = max(kern, key=lambda k: kern[k][3])
    _, bts, ms, _ = kern[dom]
    # one forcing iteration: an interpolation and a spreading pass, plus its
    # share of the once-per-step tile records
    t_iter = ((tm["ms_interp"] + tm["ms_spread"] + tm.get("ms_record", 0.0)) / 1e3 / K / iters
              if iters else None)
    dcs = r["contacts"] / K / n_sub
    b_sub = dem_bytes(w.n, dcs)
    t_sub = tm["ms_substep"] / max(tm["n_substep"], 1) / 1e3
    t_step = r["wall"] / K
    b_step = iters * (b_interp + b_spread) + n_sub * b_sub + w.n * 120
    gbs = lambda b, t: b / t / 1e9 if t else None  # noqa: E731
    res = {"kernel": dom, "achieved": gbs(bts, ms / 1e3), "alg_bytes_per_launch": bts,
           "avg_launch_ms": ms,
           "byte_model": "per iteration 5 s per touched node (interpolation read; read-modify-"
                         "write of f and u** in the spreading) + 6 s per marker; per substep "
                         "160 B per sphere + 72 B per directed contact",
           "interp": {"alg_bytes": b_interp, "avg_ms": avg_interp,
                      "GBs": gbs(b_interp, avg_interp / 1e3),
                      "frac": gbs(b_interp, avg_interp / 1e3) / HBM_PEAK_GBS,
                      "lean_bytes": l_interp},
           "spread": {"alg_bytes": b_spread, "avg_ms": avg_spread,
                      "GBs": gbs(b_spread, avg_spread / 1e3),
                      "frac": gbs(b_spread, avg_spread / 1e3) / HBM_PEAK_GBS,
                      "lean_bytes": l_spread},
           "iteration": {"alg_bytes": b_interp + b_spread, "ms": t_iter * 1e3 if t_iter else None,
                         "frac": gbs(b_interp + b_spread, t_iter) / HBM_PEAK_GBS
                         if t_iter else None},
           "substep": {"alg_bytes": b_sub, "ms": t_sub * 1e3,
                       "frac": gbs(b_sub, t_sub) / HBM_PEAK_GBS if t_sub else None},
           "step": {"alg_bytes": b_step, "ms": t_step * 1e3,
                    "frac": gbs(b_step, t_step) / HBM_PEAK_GBS},
           "measured_copy_GBs": copy_gbs,
           "frac_of_measured_copy": gbs(bts, ms / 1e3) / copy_gbs}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3-1m")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the FP32 + learned vs FP64 plain comparison")
    ap.add_argument("--train-snapshots", type=int, default=200,
                    help="training snapshots of the learned warm start")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first stream a 1 GiB buffer into another three times (an elementwise "
                         "kernel of known traffic, the reference of the HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "form of the particle step is not built", file=sys.stderr)
        return 2

    import torch

    import paper_2108_01814_amd as P
    from paper_2108_01814_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    P.lib()
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)     # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
        log("calibration: 3 elementwise passes of 1 GiB in, 1 GiB out")
    w = W.WORKLOADS[args.workload]
    t0 = time.time()
    bed = W.make_bed(w)
    log(f"{w.name}: {w.n} spheres, grid {w.grid}, bed generated in {time.time() - t0:.1f}s")

    r32 = run_form(P, W, w, bed, P.F32, args.steps, args.warmup, torch, measure_touched=True)
    K = args.steps
    tm = r32["timing"]
    t_step = r32["wall"] / K
    M = w.n * w.n_markers
    iters = r32["stats"]["iterations"]
    n_sub = W.PHYS["n_sub"]
    t_ib = (tm["ms_interp"] + tm["ms_spread"] + tm.get("ms_record", 0.0)) / 1e3 / K
    t_dem = (tm["ms_search"] + tm["ms_substep"]) / 1e3 / K
    copy_gbs = copy_rate(torch)
    log(f"measured copy rate {copy_gbs:.0f} GB/s")
    out_roof = roofline_block(w, r32, 4, K, copy_gbs, "float")
    dom = out_roof["kernel"]
    out = {
        "metric": METRIC,
        "value": w.n / t_step,
        "unit": "particle-step/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n} equal spheres (D/h={w.d_over_h}, "
                               f"{w.n_markers} markers each) in {w.domain[0]:g}x{w.domain[1]:g}x"
                               f"{w.domain[2]:g} D, grid {w.grid[0]}x{w.grid[1]}x{w.grid[2]}",
                   "spheres": w.n, "markers": M, "grid": list(w.grid),
                   "forcing_iterations": iters, "substeps": n_sub,
                   "precision": "grid and marker arithmetic f32, sphere state f64",
                   "parallelism": "single GPU"},
        "markers_per_s": M * iters / t_ib if t_ib > 0 else None,
        "contacts_per_s": (r32["contacts"] / K) / t_dem if t_dem > 0 else None,
        "phases_ms_per_step": {k[3:]: v / K for k, v in tm.items() if k.startswith("ms_")},
        "touched_nodes": r32["touched"],
        "roofline": {"bound": "hbm", "achieved": out_roof["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": out_roof["achieved"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom), **{k: v for k, v in out_roof.items()
                                                         if k != "achieved"}},
    }
    if not args.no_fp64:
        K64 = max(1, min(K, 3))
        r64 = run_form(P, W, w, bed, P.F64, K64, 1, torch)
        t64 = r64["wall"] / K64
        tm64 = r64["timing"]
        r64["touched"] = r32["touched"]
        out["fp64_plain"] = {
            "value": w.n / t64, "unit": "particle-step/s", "ms_per_step": t64 * 1e3,
            "steps": K64, "forcing_iterations": r64["stats"]["iterations"],
            "phases_ms_per_step": {k[3:]: v / K64 for k, v in tm64.items() if k.startswith("ms_")},
            "fp32_speedup": t64 / t_step,
            "roofline": roofline_block(w, r64, 8, K64, copy_gbs, "double"),
        }
    if not args.no_learned:
        out["learned_vs_fp64"] = learned_comparison(P, W, w, bed, torch, args.train_snapshots,
                                                    max(1, min(K, 3)))
    if not args.no_cpu:
        cb = cpu_baseline(W, w, bed)
        cb.pop("rc", None)
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
