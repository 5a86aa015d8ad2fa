"""Benchmark of the batched MHD patch advance on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
                [--no-adjoint] [--adjoint-only]

Prints ONE JSON line.  `value` is useful cell-updates per second (one
interior cell advanced by one (sub)step) of the whole step with inputs
resident in HBM; the roofline object reports the dominant kernel (the flux
kernel: primitive recovery, minmod slopes, Hancock predictor and HLLD, or the
fused flux-update kernel when the launch configuration selects it) against
the FP64 vector peak, its duration measured live with HIP events on the
launch stream.  cpu_baseline times the FP64 oracle on a bounded sample of the
same workload on the host cores.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR_TFLOPS = 78.6   # MI355X FP64 vector
PEAK_FP32_VECTOR_TFLOPS = 157.3  # MI355X FP32 vector (packed); the kernels do not use packed FP32
PEAK_HBM_GBS = 8000.0

# Algorithmic work of the flux kernel, counted by running the oracle's own
# step on a flop-counting scalar (each +, -, *, /, sqrt = 1): Hancock
# predictor phase (primitive recovery, minmod slopes, face states, half-step
# increment, predicted states) per cell whose predicted states are formed,
# and one HLLD evaluation per face.  Checked against the oracle by a test.
FLOPS_PRED = {3: 912, 2: 612}
FLOPS_HLLD = 367
# The update's share, counted the same way: per updated cell (the hydro
# components, and B_z in 2-D), per updated face-centred B component, and per
# edge EMF (arithmetic mean of the four face EMFs).
FLOPS_UPD_CELL = {3: 55, 2: 48}
FLOPS_UPD_FACE = {3: 8, 2: 5}
FLOPS_EMF_EDGE = 4
GAMMA = 5.0 / 3.0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


KERNEL_SOURCES = {
    "k_flux": ("advance.hip", "advance_common.hpp", "mhd_device.hpp", "amr_internal.hpp", "emf.hpp", "tables.hip"),
    "k_fused": ("fused.hip", "launch_common.hpp", "advance_common.hpp", "mhd_device.hpp", "amr_internal.hpp",
                "emf.hpp", "tables.hip"),
}


def kernel_source_digest(kernel="k_flux"):
    """sha256 over the sources that define a kernel's memory traffic (the
    kernel and the host code that builds its work lists)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1110_1616_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, dtype, kernel="k_flux", launch_config=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE and WRITE_SIZE, each scaled by what
    the counter reads for a copy of known size), or None if there is none,
    it was taken in another launch configuration, or the kernel sources
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    # one record per profiled launch configuration
    for rec in data.get("records", [data]):
        if rec.get("source_sha256") != kernel_source_digest(kernel) or rec.get("dtype") != dtype:
            continue
        if launch_config is not None and rec.get("launch_config") != launch_config:
            continue
        return rec.get("traffic_bytes_per_launch")
    return None


def flux_kernel_flops(ndim, n, gv):
    """Algorithmic flops of one flux-kernel launch over a grid with interior n
    (per axis) advanced from valid band gv."""
    m = [x + 2 * gv - 2 for x in n[:ndim]]  # cells with predicted states
    cells = 1
    for x in m:
        cells *= x
    faces = 0
    for d in range(ndim):
        f = m[d] - 1
        for a in range(ndim):
            if a != d:
                f *= m[a]
        faces += f
    return FLOPS_PRED[ndim] * cells + FLOPS_HLLD * faces


def update_flops(ndim, n, gv):
    """Algorithmic flops of the update over a grid with interior n advanced
    from valid band gv: the updated box reaches gv - 2 cells into the band."""
    u = [x + 2 * gv - 4 for x in n[:ndim]]
    cells = 1
    for x in u:
        cells *= x
    faces = edges = 0
    for d in range(ndim):
        f = u[d] + 1
        e = u[d]
        for a in range(ndim):
            if a != d:
                f *= u[a]
                e *= u[a] + 1
        faces += f
        edges += e
    if ndim == 2:
        edges = (u[0] + 1) * (u[1] + 1)  # E_z only
    return FLOPS_UPD_CELL[ndim] * cells + FLOPS_UPD_FACE[ndim] * faces + FLOPS_EMF_EDGE * edges


def single_grid_workload(args):
    """Single 3D grid (the single-grid roofline workload)."""
    import numpy as np
    import torch

    from paper_1110_1616_amd import amr as A
    from paper_1110_1616_amd import inputs as I

    N = args.n
    dtype = args.dtype
    n = (N, N, N)
    ic = I.smooth_mhd(3, n, seed=2, v_rms=0.1, b_rms=0.3, jump=True)
    H = A.Hierarchy(3, n, [(0, (0, 0, 0), n)], ghost=4, dtype=dtype, dx0=ic["dx"], gamma=GAMMA, cfl=0.4,
                    emf=EMF[args.emf])
    U, V = H.new_state(), H.new_state()
    H.load_primitive(U, 0, ic["prim"], ic["b"])
    state = {"U": U, "V": V, "s": 0}

    def step():
        # one step of the single grid: band 4 is refilled every second step
        # (the two-substep patch mode), dt from the CFL reduction, advance
        s = state["s"]
        band = 4 if s % 2 == 0 else 2
        if band == 4:
            H.fill(0, A.AMR_FILL_SAME_LEVEL, state["U"])
        H.compute_dt(state["U"])
        H.advance(state["U"], state["V"], cycle=0, band=band)
        state["U"], state["V"] = state["V"], state["U"]
        state["s"] = s + 1

    flops_per_step_pair = flux_kernel_flops(3, n, 4) + flux_kernel_flops(3, n, 2)
    upd_per_step_pair = update_flops(3, n, 4) + update_flops(3, n, 2)
    info = {
        "workload": f"single 3D grid {N}^3 + 4-cell band, ideal MHD {dtype}, smooth Fourier-mode rho/v/A "
                    f"(|B| rms 0.3) with a 4:1 planar density jump, periodic, CFL 0.4",
        "cells": N ** 3,
        "ndim": 3,
        "dtype": dtype,
        "grids": 1,
    }

    def cpu_sample():
        import oracle as O
        steps = args.cpu_steps
        t = O.uniform_time(ic, GAMMA, 0.4, steps, g=4, fill_every=2)
        return {"seconds": t, "updates": float(N ** 3 * steps), "threads": O.max_threads(),
                "sample": f"oracle, same {N}^3 input, first {steps} steps (band 4 refilled every 2 steps)"}

    def tune():
        return H.autotune(state["U"], state["V"], 0, reps=5)

    return (H, step, (lambda k: flops_per_step_pair * k / 2.0), (lambda k: upd_per_step_pair * k / 2.0), info,
            cpu_sample, tune)


def amr_workload(args, deep=False):
    """Batched AMR hierarchy, 3D.  Default (3 levels, FP64): base 112^3 tiled
    by grids with even extents drawn from 8..32, each finer level covering
    12.5% of its parent (so every level carries about the same number of
    cells), band 4 so each fine grid runs its 2 substeps from one fill.
    deep (6 levels, FP32 by default): base 200^3, log-uniform extents 8..48,
    about 3600 grids and 48M cells."""
    import numpy as np
    import torch

    from paper_1110_1616_amd import amr as A
    from paper_1110_1616_amd import inputs as I

    if deep:
        N0 = (args.n0_deep,) * 3
        L = 6
        grids, fields = I.deep_hierarchy(args.n0_deep, seed=5)
        progress(f"deep hierarchy generated: {len(grids)} grids")
    else:
        N0 = (args.n0,) * 3
        L = 3
        grids = I.amr_hierarchy(3, N0, L, seed=3, ext=(8, 32))
        fields = I.amr_fields(3, N0, L, grids, seed=3, b_rms=0.3)
    H = A.Hierarchy(3, N0, grids, nlevels=L, ghost=4, dtype=args.dtype, emf=EMF[args.emf])
    Ua, Ub = H.new_state(), H.new_state()
    progress("hierarchy created; loading the initial state")
    for gi, f in enumerate(fields):
        H.load_primitive(Ua, gi, f["prim"], f["b"])
        if gi % 1000 == 999:
            progress(f"loaded {gi + 1} grids")
    cells = [0] * L
    for (l, lo, hi) in grids:
        cells[l] += int(np.prod([hi[a] - lo[a] for a in range(3)]))
    updates = sum(c * 2 ** l for l, c in enumerate(cells))
    # algorithmic flops of the flux kernel (fl) and of the update (ufl) per
    # coarse step
    fl = ufl = 0
    for (l, lo, hi) in grids:
        n = [hi[a] - lo[a] for a in range(3)]
        for k in range(2 ** l):
            gv = 2 if l == 0 else 4 - 2 * (k % 2)
            fl += flux_kernel_flops(3, n, gv)
            ufl += update_flops(3, n, gv)
    st = {"par": 0}
    stream = torch.cuda.Stream()

    def eager(mode):
        def f():
            with torch.cuda.stream(stream):
                st["par"] = H.coarse_step(Ua, Ub, st["par"], mode)
        return f

    def capture():
        with torch.cuda.stream(stream):
            H.graph_capture(Ua, Ub, st["par"], 0)

    def capture_per_grid():
        with torch.cuda.stream(stream):
            H.graph_capture(Ua, Ub, st["par"], 1)

    def graph_step():
        with torch.cuda.stream(stream):
            st["par"] = H.graph_launch(st["par"])

    def tune():
        # five passes per candidate (three on the deep hierarchy, whose pass
        # is 32 launch cycles long): the leading candidates differ by well
        # under 1%
        with torch.cuda.stream(stream):
            return H.autotune(Ua, Ub, st["par"], reps=3 if deep else 5)

    desc = (f"{L}-level AMR hierarchy, R=2, 3D ideal MHD {args.dtype}: base {N0[0]}^3, {len(grids)} grids of even "
            f"extents {'8..48 (log-uniform)' if deep else '8..32'} (levels {cells} cells), each level covering 12.5% "
            f"of its parent, 4-cell extended band (2 substeps per fill), smooth Fourier-mode rho/v/A (|B| rms 0.3), "
            f"periodic, CFL 0.4; one coarse step = fills + batched advance of R^(L-1) launch cycles "
            f"(finest level first) + reflux/EMF fix/restriction")
    info = {
        "workload": desc,
        "cells": updates,  # useful cell-updates per coarse step
        "ndim": 3,
        "dtype": args.dtype,
        "grids": len(grids),
        "level_cells": cells,
    }

    def cpu_sample():
        import oracle as O
        if deep:
            n0s = max(8, (args.n0_deep // 2) // 2 * 2)
            g2, f2 = I.deep_hierarchy(n0s, seed=5)
        else:
            n0s = max(8, (args.n0 // 2) // 2 * 2)
            g2 = I.amr_hierarchy(3, (n0s,) * 3, L, seed=3, ext=(8, 32))
            f2 = I.amr_fields(3, (n0s,) * 3, L, g2, seed=3, b_rms=0.3)
        c2 = [0] * L
        for (l, lo, hi) in g2:
            c2[l] += int(np.prod([hi[a] - lo[a] for a in range(3)]))
        u2 = sum(c * 2 ** l for l, c in enumerate(c2))
        steps = 1 if deep else args.cpu_steps
        nthr = O.max_threads()
        t = O.amr_time(3, (n0s,) * 3, L, 4, g2, f2, steps)
        # the same sample's first coarse step on one core
        O.set_threads(1)
        t1 = O.amr_time(3, (n0s,) * 3, L, 4, g2, f2, 1)
        O.set_threads(nthr)
        return {"seconds": t, "updates": float(u2 * steps), "threads": nthr, "seconds_1core": t1,
                "updates_1core": float(u2),
                "sample": f"oracle serial level cycle on the same generator at 1/8 volume (base {n0s}^3, "
                          f"{len(g2)} grids), {steps} coarse steps (1 on one core); OpenMP over the grids of a "
                          f"level"}

    def regrid_measure():
        """One regrid of level 2 from the level-1 flags of the current state:
        flags + clustering (amr_regrid), the new hierarchy's tables
        (amr_create + workspace), the (O)verlap of every level, then the
        coarse-step time of the regridded hierarchy (eager, batched)."""
        par = st["par"]
        cur = [H.current(Ua, Ub, par, l) for l in range(L)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            new = H.regrid(1, cur[1], cur[0], args.regrid_theta, efficiency=args.regrid_eff,
                           max_box=args.regrid_max_box)
        t1 = time.perf_counter()
        Hn = A.Hierarchy(3, N0, new, nlevels=L, ghost=4, dtype=args.dtype)
        # the regridded hierarchy steps in the launch configuration the
        # benchmark chose for the original one
        Hn.set_launch_config(*(A.amr_get_launch_config(H.h) + (A.amr_get_update_zchunk(H.h),)))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        with torch.cuda.stream(stream):
            Un = Hn.overlap_from(H, cur)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        Vn = Hn.new_state()
        p2 = 0
        with torch.cuda.stream(stream):
            p2 = Hn.coarse_step(Un, Vn, p2, 0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        with torch.cuda.stream(stream):
            for _ in range(3):
                p2 = Hn.coarse_step(Un, Vn, p2, 0)
        e1.record(stream)
        torch.cuda.synchronize()
        if Hn.error_flags()[0]:
            raise RuntimeError("non-physical state after the regrid")
        c2 = [0] * L
        for (l, lo, hi) in new:
            c2[l] += int(np.prod([hi[a] - lo[a] for a in range(3)]))
        return {"level": 2, "theta": args.regrid_theta, "efficiency": args.regrid_eff,
                "max_box": args.regrid_max_box, "grids_before": len(grids), "grids_after": len(new),
                "level_cells_after": c2, "regrid_ms": (t1 - t0) * 1e3, "create_ms": (t2 - t1) * 1e3,
                "overlap_ms": (t3 - t2) * 1e3,
                "coarse_step_ms_after": e0.elapsed_time(e1) / 3,
                "cell_updates_per_s_after": sum(c * 2 ** l for l, c in enumerate(c2)) / (e0.elapsed_time(e1) / 3e3)}

    return {"H": H, "stream": stream, "step": graph_step, "prepare": capture, "eager": eager(0),
            "per_grid": eager(1), "prepare_per_grid": capture_per_grid, "flux_flops": lambda k: fl * k,
            "update_flops": lambda k: ufl * k, "info": info, "cpu_sample": cpu_sample,
            "tune": tune, "regrid": None if deep else regrid_measure, "schedules": True}


def single_workload(args):
    H, step, flops, uflops, info, cpu, tune = single_grid_workload(args)
    return {"H": H, "stream": None, "step": step, "prepare": None, "eager": step, "per_grid": None,
            "flux_flops": flops, "update_flops": uflops, "info": info, "cpu_sample": cpu, "tune": tune}


EMF = {"mean": 0, "upwind": 1}

_T0 = time.perf_counter()


def progress(msg):
    """Phase line on stderr (stdout carries only the JSON result line)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


WORKLOADS = {"amr3": amr_workload, "single128": single_workload, "deep6": lambda a: amr_workload(a, deep=True)}


def adjoint_measure(reps=3):
    """Cost of the discrete adjoint on the differentiation workload: 64^3
    periodic FP64 grid, smooth Fourier-mode rho/v/A, 20 steps with step sizes
    frozen from a CFL-0.4 forward run, checkpoints every 5 steps.  forward =
    the differentiable advance (steps plus checkpoint copies); adjoint = its
    backward (recompute of each segment plus the reverse sweep)."""
    import numpy as np
    import torch

    from paper_1110_1616_amd import amr as A
    from paper_1110_1616_amd import autodiff as AD
    from paper_1110_1616_amd import inputs as I

    n = (64, 64, 64)
    ic = I.smooth_mhd(3, n, seed=4, v_rms=0.1, b_rms=0.3)
    H = A.Hierarchy(3, n, [(0, (0, 0, 0), n)], ghost=2, dtype="f64", dx0=ic["dx"], gamma=GAMMA)
    U, V = H.new_state(), H.new_state()
    H.load_primitive(U, 0, ic["prim"], ic["b"])
    U0 = [f.clone() for f in U.fields]
    dts = []
    for _ in range(20):
        H.fill(0, A.AMR_FILL_SAME_LEVEL, U)
        H.compute_dt(U)
        dts.append(float(H.dt0.item()))
        H.advance(U, V, cycle=0, band=2)
        U, V = V, U
    gen = torch.Generator(device="cuda").manual_seed(4)
    seed = [torch.randn(H.state_elems, dtype=torch.float64, device="cuda", generator=gen) for _ in range(8)]
    fwd, bwd = [], []
    for _ in range(reps + 1):
        x = [f.clone().requires_grad_(True) for f in U0]
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record()
        out = AD.advance(H, 0, dts, x, every=5)
        e1.record()
        torch.autograd.grad(out, x, grad_outputs=seed)
        e2.record()
        torch.cuda.synchronize()
        fwd.append(e0.elapsed_time(e1))
        bwd.append(e1.elapsed_time(e2))
    f, b = float(np.median(fwd[1:])), float(np.median(bwd[1:]))
    return {"workload": "64^3 periodic FP64, smooth Fourier-mode rho/v/A, 20 steps, checkpoints every 5",
            "forward_ms": f, "adjoint_ms": b, "adjoint_over_forward": b / f}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="amr3", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--n0", type=int, default=112)
    ap.add_argument("--n0-deep", type=int, default=200)
    ap.add_argument("--per-grid-steps", type=int, default=3)
    ap.add_argument("--dtype", default=None, choices=["f64", "f32"],
                    help="default f64 (f32 for the deep6 workload)")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--emf", default="mean", choices=sorted(EMF),
                    help="edge EMF of constrained transport: arithmetic mean or upwinded (Gardiner-Stone)")
    ap.add_argument("--no-regrid", action="store_true", help="skip the regrid measurement (3-level workload)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "0", "1"],
                    help="launch-cycle schedule: window start (0), predictive eta balance (1), or the faster")
    ap.add_argument("--regrid-theta", type=float, default=0.03,
                    help="flag threshold of the measured regrid (relative centred density jump)")
    ap.add_argument("--regrid-eff", type=float, default=0.5, help="clustering efficiency of the measured regrid")
    ap.add_argument("--regrid-max-box", type=int, default=32,
                    help="largest box extent of the measured regrid, in level-1 cells")
    ap.add_argument("--launch-config", default=None,
                    help="tile_policy,zchunk,launch_mode[,update_zchunk]: set this launch configuration instead "
                         "of autotuning (launch_mode bit 0 persistent queue, bit 1 one item chunk per XCD, bit 2 persistent flux kernel only, bit 3 fused flux-update kernel, bits 4-5 log2 of the work items per block claim)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device-to-device once (a plain copy kernel of known size that "
                         "calibrates HBM byte counters)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the adjoint of the 64^3 differentiation workload and print that object")
    args = ap.parse_args()
    if args.dtype is None:
        args.dtype = "f32" if args.workload == "deep6" else "f64"

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(it shards by grid in design only); rerun with --gpus 1", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch
    from paper_1110_1616_amd import amr as A

    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        # an elementwise kernel that reads and writes exactly N bytes each
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_measure(reps=max(1, args.steps))}), flush=True)
        return
    progress(f"building workload {args.workload}")
    W = WORKLOADS[args.workload](args)
    H, info = W["H"], W["info"]
    progress(f"workload ready: {info['grids']} grids")

    def timed(fn, k):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        stream = W["stream"] or torch.cuda.current_stream()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(k):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    # warm-up (eager), then capture the coarse step as HIP graphs if the
    # workload uses them
    for _ in range(args.warmup):
        W["eager"]()
    torch.cuda.synchronize()
    tuned = None
    if args.launch_config:
        vals = [int(v) for v in args.launch_config.split(",")]
        pol, zc, per = vals[:3]
        uz = vals[3] if len(vals) > 3 else None
        H.set_launch_config(pol, zc, per, uz)
        tuned = {"chosen": {"tile_policy": pol, "zchunk": zc, "launch_mode": per,
                            "update_zchunk": A.amr_get_update_zchunk(H.h)}, "set_by": "--launch-config"}
    elif W.get("tune") and not args.no_autotune:
        progress("autotuning the launch configuration")
        chosen, table = W["tune"]()
        torch.cuda.synchronize()
        tuned = {"chosen": {"tile_policy": table[chosen][0], "zchunk": table[chosen][1],
                            "launch_mode": table[chosen][2], "update_zchunk": table[chosen][4]},
                 "candidates_ms": [[t[0], t[1], t[2], t[4], round(t[3], 4)] for t in table]}
        for _ in range(2):
            W["eager"]()
        torch.cuda.synchronize()
    sched = None
    progress("warm-up and launch configuration done")
    if W.get("schedules"):
        # launch-cycle schedule: window start (0) or the predictive eta
        # balance (1); both compute the same bits, the faster one is timed
        ncyc = 2 ** (H.nlevels - 1)
        cand = [0, 1] if args.schedule == "auto" else [int(args.schedule)]
        ms = {}
        for sc in cand:
            H.set_schedule(sc)
            W["eager"]()
            ms[sc] = timed(W["eager"], 3) / 3
        best = min(ms, key=ms.get)
        H.set_schedule(best)
        _, work = A.amr_get_schedule(H.h, ncyc)
        sched = {"chosen": best, "eager_ms": {str(k): round(v, 4) for k, v in ms.items()},
                 "predicted_cycle_work": [round(x) for x in work]}
    if W["prepare"]:
        W["prepare"]()
        torch.cuda.synchronize()
        for _ in range(2):
            W["step"]()

    # timed region: K steps of the production path
    progress(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    gpu_ms = timed(W["step"], args.steps)
    wall = time.perf_counter() - t0

    # per-kernel durations over K eager steps of the same batched work (HIP
    # events on the launch stream around each flux and update launch)
    A.amr_set_kernel_timing(H.h, True)
    eager_ms = timed(W["eager"], args.steps)
    flux_ms, upd_ms, nl = A.amr_kernel_times(H.h)
    A.amr_set_kernel_timing(H.h, False)

    per_grid = per_grid_graph = per_grid_cfg = None
    if W["per_grid"] is not None and args.per_grid_steps > 0:
        # the serial per-grid order (one launch per grid) under the batched
        # path's launch configuration and under short z-chunks with one
        # block per item (more blocks per grid); the faster one is the
        # baseline
        progress("timing the per-grid path")
        keep = A.amr_get_launch_config(H.h) + (A.amr_get_update_zchunk(H.h),)
        best = None
        for cfg in (keep, (1, 8, 8 if args.emf == "mean" else 0, keep[3]), (1, 8, 0, keep[3])):
            H.set_launch_config(*cfg)
            W["per_grid"]()
            ms_ = timed(W["per_grid"], args.per_grid_steps)
            if best is None or ms_ < best[0]:
                best = (ms_, cfg)
        pg_ms, per_grid_cfg = best
        per_grid = float(info["cells"]) * args.per_grid_steps / (pg_ms / 1e3)
        H.set_launch_config(*per_grid_cfg)
        if W.get("prepare_per_grid"):
            # the same serial per-grid order replayed from a captured graph
            # (no host launch overhead); replaces the batched graphs
            progress("capturing and timing the per-grid path as a HIP graph")
            W["prepare_per_grid"]()
            torch.cuda.synchronize()
            W["step"]()
            pgg_ms = timed(W["step"], args.per_grid_steps)
            per_grid_graph = float(info["cells"]) * args.per_grid_steps / (pgg_ms / 1e3)
        H.set_launch_config(*keep)

    flags, _ = H.error_flags()
    if flags:
        print("non-physical state flagged during the benchmark", file=sys.stderr)
        sys.exit(3)

    seconds = gpu_ms / 1e3
    updates = float(info["cells"]) * args.steps
    value = updates / seconds
    # the dominant kernel: the flux kernel, or the fused flux-update kernel
    # (launch mode bit 3), whose event pair then covers the whole advance
    pol, zc, mode = A.amr_get_launch_config(H.h)
    fused = bool(mode & 8) and args.emf == "mean"
    kname = "k_fused" if fused else "k_flux"
    fl = W["flux_flops"](args.steps) + (W["update_flops"](args.steps) if fused else 0.0)
    peak = PEAK_FP64_VECTOR_TFLOPS if info["dtype"] == "f64" else PEAK_FP32_VECTOR_TFLOPS
    achieved = fl / (flux_ms / 1e3) / 1e12
    cfg = f"{pol},{zc},{mode}"
    esize = 8 if info["dtype"] == "f64" else 4
    out = {
        "metric": "MHD cell-updates/s (useful interior cell-updates per second of the batched advance)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": info["dtype"],
        "data": "synthetic",
        "config": {"workload": info["workload"] + ("; upwinded (Gardiner-Stone) CT EMF" if args.emf == "upwind" else ""),
                   "grids": info["grids"],
                   "useful_cell_updates_per_step": info["cells"], "parallelism": "single GPU"},
        "roofline": {"kernel": kname, "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(args.workload, info["dtype"], kname, cfg),
                     "avg_launch_ms": flux_ms / max(nl, 1), "launches": nl, "launch_config": cfg,
                     "flops_per_launch": fl / max(nl, 1)},
        "kernels_ms_per_step": ({"k_fused": flux_ms / args.steps} if fused else
                                {"k_flux": flux_ms / args.steps, "k_update": upd_ms / args.steps}),
        "eager_value": updates / (eager_ms / 1e3),
        "hbm_algorithmic_GBps": updates * 16 * esize / seconds / 1e9,
        "wall_s": wall,
    }
    if per_grid is not None:
        out["per_grid_value"] = per_grid
        out["batched_over_per_grid"] = value / per_grid
        out["per_grid_launch_config"] = ",".join(str(v) for v in per_grid_cfg)
    if per_grid_graph is not None:
        out["per_grid_graph_value"] = per_grid_graph
        out["batched_over_per_grid_graph"] = value / per_grid_graph
    if tuned is not None:
        out["autotune"] = tuned
    if sched is not None:
        out["schedule"] = sched
    if W.get("regrid") and not args.no_regrid:
        progress("measuring a regrid")
        out["regrid"] = W["regrid"]()
    if not args.no_adjoint:
        progress("measuring the adjoint")
        out["adjoint"] = adjoint_measure()
    if not args.no_cpu_baseline:
        progress("timing the CPU oracle sample")
        cs = W["cpu_sample"]()
        out["cpu_baseline"] = {"value": cs["updates"] / cs["seconds"], "unit": "cell-updates/s",
                               "cores": cs["threads"], "kind": "oracle", "sample": cs["sample"],
                               "cpu_model": cpu_model(), "nproc": os.cpu_count()}
        if "seconds_1core" in cs:
            out["cpu_baseline"]["value_1core"] = cs["updates_1core"] / cs["seconds_1core"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
