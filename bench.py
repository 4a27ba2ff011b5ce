"""Throughput of the BTDF-IB-LBM step on one MI355X.

Default workload: the particle-laden periodic lattice, 8192 x 8192 nodes,
2000 fixed cylinders of D = 24 (75 markers each, 150 000 markers), uniform
body force, FP32 populations, cosine 4-point delta with drs = 2.6 dh. One
step = the marker kernel (interpolation, direct force, per-body force and
torque) + the lattice kernel (streaming, spread gather, collision). Inputs
are synthetic and seeded; everything is resident in HBM before timing.

Prints one JSON line: MLUPS (whole job), ms per step, the roofline of the
lattice kernel (72 algorithmic bytes per lattice update against 8 TB/s,
timed with HIP events on the library's stream over the timed region), the
batched mode on 256 uneven channel cases beside the same cases run one
after another, the cost of the adjoint sweep beside the forward run, and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10000)
    p.add_argument("--warmup", type=int, default=200)
    p.add_argument("--workload", choices=["particles", "shedding", "channel"], default="particles")
    p.add_argument("--delta", choices=["cos4", "roma3", "peskin4"], default="cos4")
    p.add_argument("--variant", type=int, default=-1, help="lattice launch shape (-1: library default)")
    p.add_argument("--graph-chunk", type=int, default=0)
    p.add_argument("--row-pad", type=int, default=0)
    p.add_argument("--interior", type=int, default=-1, help="1/0: uniform-base path for interior waves (-1: library default)")
    p.add_argument("--blocking", type=int, default=-1,
                   help="steps per pass away from the bodies: 0 off, 1 deepest, 2 or 3 (-1: library default)")
    p.add_argument("--split-steps", type=int, default=3000,
                   help="steps of the separate per-kernel timing run (HIP events around each launch)")
    p.add_argument("--plane-pad", type=int, default=0)
    p.add_argument("--row-align", type=int, default=-1, help="row alignment in bytes (-1: library default)")
    p.add_argument("--copy-probe-mb", type=int, default=0,
                   help="before timing, copy a tensor of this size once (counter calibration)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-batched", action="store_true", help="skip the batched-mode figures")
    p.add_argument("--only-batched", action="store_true", help="print the batched-mode figures alone")
    p.add_argument("--batched-steps", type=int, default=5000)
    p.add_argument("--batched-variant", type=int, default=-1,
                   help="batch launch shape (-1: autotuned; a fixed one keeps counter runs to one shape)")
    p.add_argument("--batched-graph-chunk", type=int, default=50)
    p.add_argument("--seq-steps", type=int, default=200,
                   help="steps per case when timing the sequential single-case runs (0: skip them)")
    p.add_argument("--cpu-budget-s", type=float, default=20.0)
    p.add_argument("--cpu-one-core-budget-s", type=float, default=10.0,
                   help="host seconds for the one-thread oracle sample (0: skip it)")
    p.add_argument("--repeats", type=int, default=5,
                   help="timed blocks of --steps steps each; value and ms_per_step are their median")
    p.add_argument("--no-adjoint", action="store_true", help="skip the adjoint figures")
    p.add_argument("--only-adjoint", action="store_true", help="print the adjoint figures alone")
    p.add_argument("--adjoint-steps", type=int, default=5000)
    p.add_argument("--no-shedding", action="store_true",
                   help="skip the 2000x800 Re 200 shedding run (100 000 steps, Table 3)")
    p.add_argument("--no-other-delta", action="store_true",
                   help="skip timing the particle-laden lattice with the other delta (3-point / cosine)")
    p.add_argument("--no-validation", action="store_true",
                   help="skip the 1601^2 cylinder check at Re 40 (Table 3)")
    return p.parse_args()


def timed_blocks(sim, steps, repeats, fused_tiles):
    """`repeats` timed blocks of exactly `steps` steps, each bracketed by
    device synchronisations: wall seconds, the blocked pass's per-launch ms
    (HIP events around its launches only: events around every launch would
    add about 2% to a step) and, without blocking, the split kernel times."""
    import torch
    walls, passes, splits = [], [], []
    for _ in range(max(1, repeats)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if fused_tiles > 0:
            ms_pass, split = sim.step_timed_pass(steps), None
        else:
            split = sim.step_timed_split(steps)
            ms_pass = split[2]
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        passes.append(ms_pass)
        splits.append(split)
        sim.forces()  # surfaces an instability as an error
    return walls, passes, splits


def pass_kernel(depth):
    """Name of the blocked pass's kernel for a pass of depth steps."""
    return "lbm%d_kernel" % depth if depth <= 3 else "lbmd_kernel"


def bench_other_delta(args, kind_name):
    """The particle-laden lattice with the other delta of the pair the
    workload names (3-point with thickening 1.9, 4-point cosine with 2.6):
    the same steps and timed blocks, the whole step's MLUPS and the blocked
    pass's fraction of HBM at its compulsory bytes."""
    import btdf_workloads as W
    from paper_1806_09403_amd import Sim, _lib
    kind = {"cos4": W.COS4, "roma3": W.ROMA3, "peskin4": W.PESKIN4}[kind_name]
    case = W.c3(kind=kind)
    sim = Sim.from_case(case, precision=4, set_init=False)
    try:
        fused = sim.get_option(_lib.OPT_FUSED_TILES)
        depth = sim.get_option(_lib.OPT_STEPS_PER_PASS)
        sim.step(max(0, args.warmup - depth))
        if fused > 0:
            sim.step_timed_pass(depth)
        walls, passes, splits = timed_blocks(sim, args.steps, min(args.repeats, 3), fused)
        order = sorted(range(len(walls)), key=lambda i: walls[i])
        med = order[len(order) // 2]
        wall = walls[med]
        out = {"workload": case.name, "delta": kind_name, "thickening": case.thickening, "steps": args.steps,
               "ms_per_step": round(wall * 1e3 / args.steps, 5),
               "value": round(case.nodes * args.steps / wall / 1e6, 2), "unit": "MLUPS",
               "ms_per_step_repeats": [round(w * 1e3 / args.steps, 5) for w in walls]}
        if fused > 0:
            launch_ms = depth * passes[med]
            ach = sim.get_option(_lib.OPT_FUSED_NODES) * 9 * 2 * 4 / (launch_ms * 1e-3) / 1e9
            out[pass_kernel(depth)] = {"launch_ms": round(launch_ms, 5), "achieved": round(ach, 1),
                                           "frac": round(ach / HBM_PEAK_GBS, 4)}
        return out
    finally:
        sim.close()


def bench_shedding(args):
    """Unsteady shedding behind the D = 80 cylinder in the 2000x800 channel
    at Re 200 (FP32, cosine delta): 100 000 steps, the last 40 000 recorded.
    C_D as mean and half swing, the lift's half swing and the Strouhal
    number, beside Table 3's Re 200 row (a 40D x 40D domain there, 10%
    blockage here: a loose comparison)."""
    import btdf_workloads as W
    from paper_1806_09403_amd import validation
    t0 = time.perf_counter()
    case = W.c2()
    r = validation.run_unsteady(case, warmup=60_000, window=40_000)
    return {"workload": case.name, "delta": "cos4", "thickening": case.thickening, "Re": 200,
            "steps": r["steps"], "window": 40_000, "Cd": round(r["Cd"], 4), "Cd_dev": round(r["Cd_dev"], 4),
            "Cl_dev": round(r["Cl_dev"], 4), "St": round(r["St"], 4),
            "paper": {"Cd": 1.364, "Cd_dev": 0.042, "Cl_dev": 0.699, "St": 0.195},
            "seconds": round(time.perf_counter() - t0, 1)}


def make_case(args):
    import btdf_workloads as W
    kind = {"cos4": W.COS4, "roma3": W.ROMA3, "peskin4": W.PESKIN4}[args.delta]
    if args.workload == "particles":
        return W.c3(kind=kind), 4
    if args.workload == "shedding":
        return W.c2(kind=kind), 4
    return W.c1(kind=kind), 8


def cpu_sample(case, budget_s):
    """The FP64 oracle on the same lattice and bodies: one step to size the
    sample, then as many more as fit the budget (none if the first step
    already took it). Returns (MLUPS, steps, seconds)."""
    import numpy as np
    from oracle import oracle
    o = oracle.OracleSim(case.nx, case.ny, case.bc, case.tau, case.kind, case.thickening, case.G,
                         case.inflow, case.init)
    for b in case.bodies:
        o.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
    if case.init_uy is not None:
        ux, uy = case.init_fields()
        o.init_equilibrium(ux, uy, np.full((case.ny, case.nx), case.init[0]))
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter()
    k = int((budget_s - (t1 - t0)) / max(t1 - t0, 1e-9))
    if k > 0:
        o.step(k)
    t2 = time.perf_counter()
    steps = 1 + max(k, 0)
    o.close()
    return case.nodes * steps / (t2 - t0) / 1e6, steps, t2 - t0


def cpu_baseline(case, budget_s, one_core_budget_s):
    """The unmodified FP64 oracle on the host: all its OpenMP threads, then
    one thread."""
    from oracle import oracle
    cores = oracle.num_threads()
    mlups, steps, secs = cpu_sample(case, budget_s)
    what = "%s: %%d FP64 oracle steps of the full %dx%d lattice with all %d bodies (%%.1f s)" % (
        case.name, case.nx, case.ny, len(case.bodies))
    out = {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": what % (steps, secs)}
    if one_core_budget_s > 0:
        oracle.set_num_threads(1)
        m1, s1, t1 = cpu_sample(case, one_core_budget_s)
        oracle.set_num_threads(cores)
        out["one_core"] = {"value": round(m1, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
                           "sample": what % (s1, t1)}
    return out


def copy_probe(mb):
    """One plain device copy of known size: the reference dispatch against
    which the HBM byte counters of the kernels are scaled."""
    import torch
    nbytes = mb << 20
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dst.copy_(src)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print("copy probe: %d MiB read + %d MiB written in %.3f ms (%.1f GB/s)"
          % (mb, mb, (t1 - t0) * 1e3, 2 * nbytes / (t1 - t0) / 1e9), file=sys.stderr, flush=True)
    del src, dst


def bench_batched(args):
    """The 256 uneven channel cases: one batch (autotuned launch shape, graph
    replay) against the same cases run one after another as single cases
    (graph replay too). Cases that trip the instability guard in the batched
    run are left out of both sums (their work before stopping is not counted)."""
    import torch
    import btdf_workloads as W
    from paper_1806_09403_amd import BatchSim, Sim, _lib

    cases = W.c4()
    t_setup = time.perf_counter()
    opts = {}
    if args.row_align >= 0:
        opts[_lib.OPT_ROW_ALIGN] = args.row_align
    b = BatchSim(cases, precision=4, options=opts)
    if args.batched_variant >= 0:
        best = args.batched_variant
        b.set_option(_lib.OPT_LBM_VARIANT, best)
    else:
        best = b.autotune(steps_per_trial=5)
    b.set_option(_lib.OPT_GRAPH_CHUNK, args.batched_graph_chunk)
    b.step(100)
    torch.cuda.synchronize()
    print("batched setup + tune + warmup %.1f s" % (time.perf_counter() - t_setup), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    b.step(args.batched_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    unstable, _ = b.status()
    ms_ib, ms_lbm = b.step_timed(201)
    b_align = b.get_option(_lib.OPT_ROW_ALIGN)
    depth = b.get_option(_lib.OPT_STEPS_PER_PASS)
    blocked_nodes = b.get_option(_lib.OPT_FUSED_NODES)
    b.close()
    del b
    traffic = None
    key = "batched-v%d-a%d%s" % (best, b_align, "-p3" if depth == 3 else "")
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            t = json.load(f).get(key)
        if t:
            traffic = round(t["bytes_per_step"] / (ms_lbm * 1e-3) / 1e9, 1)
    stable = [k for k in range(len(cases)) if not unstable[k]]
    nodes = sum(cases[k].nodes for k in stable)
    mlups = nodes * args.batched_steps / wall / 1e6
    # algorithmic bytes of the lattice work per step: 72 B per node stepped
    # singly, 72 / depth per node in the blocked pass (all cases stable)
    bytes_per_step = 72 * (nodes - blocked_nodes) + 72 / depth * blocked_nodes if len(stable) == len(cases) \
        else 72 * nodes
    achieved = bytes_per_step / (ms_lbm * 1e-3) / 1e9
    print("batched: %d of %d cases stable, %.1f MLUPS" % (len(stable), len(cases), mlups), file=sys.stderr, flush=True)

    t_seq = 0.0
    for k in (stable if args.seq_steps > 0 else []):
        s = Sim.from_case(cases[k], precision=4)
        s.set_option(_lib.OPT_GRAPH_CHUNK, args.batched_graph_chunk)
        s.step(args.batched_graph_chunk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.seq_steps)
        torch.cuda.synchronize()
        t_seq += (time.perf_counter() - t0) / args.seq_steps
        s.close()
    seq_mlups = nodes / t_seq / 1e6 if t_seq > 0 else None
    if seq_mlups:
        print("sequential: %.1f MLUPS" % seq_mlups, file=sys.stderr, flush=True)
    return {"workload": "256 uneven single-cylinder channels (W 128..1024, H = W/2, D 8..48, Re 0.1..200), FP32",
            "cases": len(cases), "stable_cases": len(stable), "nodes": nodes, "steps": args.batched_steps,
            "value": round(mlups, 2), "unit": "MLUPS", "ms_per_step": round(wall * 1e3 / args.batched_steps, 5),
            "sequential_mlups": round(seq_mlups, 2) if seq_mlups else None,
            "speedup_vs_sequential": round(mlups / seq_mlups, 3) if seq_mlups else None,
            "sequential_sample": "each stable case alone, %d graph-replayed steps" % args.seq_steps,
            "lbm_variant": best, "graph_chunk": args.batched_graph_chunk, "row_align": b_align,
            "steps_per_pass": depth, "blocked_nodes_frac": round(blocked_nodes / nodes, 4),
            "kernel_ms": {"ib_batch_kernel": round(ms_ib, 5), "lbm_batch_kernel": round(ms_lbm, 5)},
            "kernel_ms_note": "per step; lbm_batch_kernel: the lattice launches of a step (with blocking: the "
                              "near tiles' steps and the blocked pass, a third of each triple)",
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                         "kernel": "lbm_batch_kernel" if depth == 1 else "lbm3_batch_kernel+lbm_batch_kernel",
                         "bytes_per_step": int(bytes_per_step)}}


def bench_adjoint(args):
    """Cost of the reverse sweep on the 800x400 Re = 100 channel (126
    markers, FP32): gradient of the mean drag coefficient over the horizon,
    with sqrt(N) checkpoints and with a full tape, against the forward run
    alone (replayed from graphs of 50 steps, its fastest form)."""
    import numpy as np
    import torch
    import btdf_workloads as W
    from paper_1806_09403_amd import Sim, _lib

    c = W.c5(precision=4)
    n = args.adjoint_steps
    b = c.bodies[0]

    def make():
        s = Sim(c.nx, c.ny, c.tau, c.kind, c.thickening, c.bc, c.inflow, c.G, c.init, 4, history_capacity=n)
        s.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
        return s

    s = make()
    s.set_option(_lib.OPT_GRAPH_CHUNK, 50)
    s.step(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(n)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3
    s.close()
    hbar = np.zeros((n, 1, 3))
    hbar[:, 0, 0] = 2.0 / (c.U * c.U * c.D) / n
    out = {"workload": "800x400 channel, D = 40, 126 markers, Re 100, FP32; J = mean Cd over %d steps" % n,
           "steps": n, "forward_ms_per_step": round(fwd_ms / n, 5)}
    grads = {}
    for name, K in (("sqrt_checkpoints", 0), ("tape", n)):
        s = make()
        s.adjoint(min(n, 60), hbar[:min(n, 60)], checkpoint_every=K)  # first launches, graph paths
        s.close()
        s = make()
        nbytes = _lib.load().btdf_adjoint_workspace_bytes(s._workspace(), n, K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g, ms = s.adjoint(n, hbar, checkpoint_every=K)
        wall = (time.perf_counter() - t0) * 1e3
        if K == 0:
            grads[4] = c5_gradient_terms(c, s, g, n)
        s.close()
        rev = ms[2]
        out[name] = {"checkpoint_every": K if K else int(np.ceil(np.sqrt(n))), "workspace_gb": round(nbytes / 1e9, 3),
                     "forward_pass_ms": round(ms[0], 2), "recompute_ms_overlapped": round(ms[1], 2),
                     "reverse_sweep_ms": round(ms[2], 2), "call_wall_ms": round(wall, 1),
                     "adjoint_over_forward": round(rev / fwd_ms, 3)}
        print("adjoint %s: forward pass %.1f ms, recompute %.1f ms (overlapped), reverse sweep %.1f ms; "
              "sweep / forward = %.2f" % (name, ms[0], ms[1], ms[2], rev / fwd_ms), file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    out["gradient_check"] = c5_gradient_check(c, n, grads[4])
    return out


C5_UV_SAMPLES = ((0, 0), (16, 1), (31, 1), (70, 0))


def c5_gradient_terms(c, s, g, n):
    """dJ/dU, dJ/dx_c and sampled dJ/dU_b from one adjoint call's gradients,
    J the mean drag coefficient over the n steps the call ran."""
    import numpy as np
    U, D = c.U, c.D
    hist = s.force_history(n)
    J = float(np.mean(2.0 * hist[:, 0, 0] / (U * U * D)))
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    dfeq = w * (3.0 * ex + 9.0 * ex * ex * U - 3.0 * U)  # d/dU of feq_q(1, (U, 0)), the initial state
    dU = g["inflow"][0] + float(np.einsum("qyx,q->", g["populations"], dfeq)) - 2.0 * J / U
    dx = float(np.sum(g["marker_xy"][:, 0]) + g["centres"][0, 0])
    return {"J": J, "dU": dU, "dx": dx, "uv": [float(g["marker_uv"][l, k]) for l, k in C5_UV_SAMPLES]}


def c5_gradient_check(c, n, g32):
    """FP32 (the timed call) and FP64 adjoint gradients against FP64 central
    differences of the GPU forward run, h = 1e-4: relative errors of dJ/dU,
    dJ/dx_c and three marker velocities' dJ/dU_b."""
    import numpy as np
    from paper_1806_09403_amd import Sim
    b = c.bodies[0]
    U, D, h = c.U, c.D, 1e-4

    def make(prec, u=U, dx=0.0, uv=None):
        s = Sim(c.nx, c.ny, c.tau, c.kind, c.thickening, c.bc, (u, 0.0), c.G, (1.0, u, 0.0), prec, history_capacity=n)
        s.add_body(b.xy + np.array([dx, 0.0]), b.uv if uv is None else uv, b.cx + dx, b.cy, b.ds)
        return s

    def J(u=U, **kw):  # the coefficient's normalisation moves with the inflow speed
        s = make(8, u=u, **kw)
        s.step(n)
        hist = s.force_history(n)
        s.close()
        return float(np.mean(2.0 * hist[:, 0, 0] / (u * u * D)))

    s = make(8)
    hbar = np.zeros((n, 1, 3))
    hbar[:, 0, 0] = 2.0 / (U * U * D) / n
    g, _ = s.adjoint(n, hbar, checkpoint_every=0)
    g64 = c5_gradient_terms(c, s, g, n)
    s.close()
    fd = {"dU": (J(u=U + h) - J(u=U - h)) / (2 * h), "dx": (J(dx=h) - J(dx=-h)) / (2 * h), "uv": []}
    for l, k in C5_UV_SAMPLES:
        duv = np.zeros_like(b.xy)
        duv[l, k] = h
        fd["uv"].append((J(uv=duv) - J(uv=-duv)) / (2 * h))

    def rel(a, r):
        return float("%.3g" % abs(a / r - 1.0))

    out = {"reference": "FP64 central differences of the GPU forward run, h = 1e-4", "target_rel": 1e-4,
           "J_fp32_vs_fp64_rel": rel(g32["J"], g64["J"])}
    for name, a in (("fp32", g32), ("fp64", g64)):
        out[name] = {"dJ_dU_rel": rel(a["dU"], fd["dU"]), "dJ_dxc_rel": rel(a["dx"], fd["dx"]),
                     "dJ_dUb_rel": [rel(x, r) for x, r in zip(a["uv"], fd["uv"])]}
    out["dUb_samples"] = [list(t) for t in C5_UV_SAMPLES]
    print("gradient check: %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def bench_validation(args):
    """The paper's cylinder case at its own size (Section 5.2), Re 40:
    drag coefficient and wake length against Table 3's row of the method."""
    import btdf_workloads as W
    from paper_1806_09403_amd import validation
    t0 = time.perf_counter()
    case = W.v40(40.0)
    r = validation.run_steady(case, max_steps=40_000)
    return {"workload": case.name, "delta": "roma3", "thickening": case.thickening, "Re": 40,
            "steps": r["steps"], "Cd": round(r["Cd"], 5), "Lw": round(r["Lw"], 4),
            "boundary_error": float("%.4g" % r["boundary_error"]),
            "paper": {"Cd": 1.551, "Lw": 2.40}, "seconds": round(time.perf_counter() - t0, 1)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1806_09403_amd import Sim, _lib

    if args.only_adjoint:
        print(json.dumps(bench_adjoint(args)), flush=True)
        return
    if args.only_batched:
        if args.copy_probe_mb:
            copy_probe(args.copy_probe_mb)
        print(json.dumps(bench_batched(args)), flush=True)
        return
    case, prec = make_case(args)
    t_setup = time.perf_counter()
    sim = Sim.from_case(case, precision=prec, set_init=False)
    if args.row_pad:
        sim.set_option(_lib.OPT_ROW_PAD, args.row_pad)
    if args.row_align >= 0:
        sim.set_option(_lib.OPT_ROW_ALIGN, args.row_align)
    if args.plane_pad:
        sim.set_option(_lib.OPT_PLANE_PAD, args.plane_pad)
    if case.init_uy is not None:
        import numpy as np
        ux, uy = case.init_fields()
        sim.init_equilibrium(ux, uy, np.full((case.ny, case.nx), case.init[0]))
    if args.variant >= 0:
        sim.set_option(_lib.OPT_LBM_VARIANT, args.variant)
    if args.graph_chunk:
        sim.set_option(_lib.OPT_GRAPH_CHUNK, args.graph_chunk)
    if args.interior >= 0:
        sim.set_option(_lib.OPT_INTERIOR_PATH, args.interior)
    if args.blocking >= 0:
        sim.set_option(_lib.OPT_TEMPORAL_BLOCKING, args.blocking)
    fused_tiles = sim.get_option(_lib.OPT_FUSED_TILES)
    depth = sim.get_option(_lib.OPT_STEPS_PER_PASS)
    # warmup: plain steps, then one timed call (untimed here) that creates the
    # handle's HIP events, so the timed region creates none
    pre = min(args.warmup, depth)
    sim.step(args.warmup - pre)
    if pre > 0:
        if fused_tiles > 0:
            sim.step_timed_pass(pre)
        else:
            sim.step_timed_split(pre)
    torch.cuda.synchronize()
    if args.copy_probe_mb:
        copy_probe(args.copy_probe_mb)
    print("setup + warmup %.1f s" % (time.perf_counter() - t_setup), file=sys.stderr, flush=True)

    # the timed region, repeated: each block is exactly --steps steps,
    # bracketed by stream synchronisations; value and ms_per_step are the
    # median block
    walls, passes, splits = timed_blocks(sim, args.steps, args.repeats, fused_tiles)
    order = sorted(range(len(walls)), key=lambda i: walls[i])
    med = order[len(order) // 2]
    wall, ms_pass = walls[med], passes[med]
    if fused_tiles <= 0:
        ms_ib, ms_single, _ = splits[med]
    split_steps = args.steps
    if fused_tiles > 0:
        # the other kernels' times: events around every launch, in a separate
        # run after the timed region
        split_steps = max(depth, min(args.steps, args.split_steps) // depth * depth)
        ms_ib, ms_single, _ = sim.step_timed_split(split_steps)
        sim.forces()

    n = case.nodes
    ms_step = wall * 1e3 / args.steps
    mlups = n * args.steps / wall / 1e6
    node_bytes = 9 * 2 * prec  # one read and one write of the 9 populations
    variant = sim.get_option(_lib.OPT_LBM_VARIANT)
    if fused_tiles > 0:
        # dominant kernel: the blocked pass, depth updates per node per launch of node_bytes
        launch_nodes = sim.get_option(_lib.OPT_FUSED_NODES)
        launch_ms = depth * ms_pass
        kernel, bytes_per_update = pass_kernel(depth), node_bytes / depth
        key = "%s-%s-v%d-p%d" % (args.workload, args.delta, variant, depth)
    else:
        launch_nodes, launch_ms = n, ms_single
        kernel, bytes_per_update = "lbm_kernel", node_bytes
        key = "%s-%s-v%d-i%d" % (args.workload, args.delta, variant, sim.get_option(_lib.OPT_INTERIOR_PATH))
    achieved = launch_nodes * node_bytes / (launch_ms * 1e-3) / 1e9
    # measured HBM bytes per launch (profiles/traffic.json, counter runs of this
    # exact configuration) over the same live duration: GB/s like `achieved`
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        if key in t:
            traffic = round(t[key]["bytes_per_launch"] / (launch_ms * 1e-3) / 1e9, 1)
    nb, nm, _ = sim.counts()
    line = {
        "metric": "MLUPS (D2Q9+BTDF-IB)",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": case.name, "nx": case.nx, "ny": case.ny, "bodies": nb, "markers": nm,
                   "delta": args.delta, "thickening": case.thickening, "tau": case.tau,
                   "lbm_variant": sim.get_option(_lib.OPT_LBM_VARIANT),
                   "row_pad": args.row_pad, "plane_pad": args.plane_pad,
                   "interior_path": sim.get_option(_lib.OPT_INTERIOR_PATH),
                   "graph_chunk": args.graph_chunk,
                   "temporal_blocking": sim.get_option(_lib.OPT_TEMPORAL_BLOCKING),
                   "steps_per_pass": depth,
                   "blocked_tiles": fused_tiles,
                   "blocked_nodes_frac": round(launch_nodes / n, 4) if fused_tiles else 0.0},
        "kernel_ms": dict([("ib_kernel", round(ms_ib, 5)), ("lbm_kernel", round(ms_single, 5))] +
                          ([(kernel, round(launch_ms, 5))] if fused_tiles > 0 else [])),
        "kernel_ms_note": ("%s: per launch (%d steps), HIP events around its launches over the timed steps; "
                           "ib_kernel and lbm_kernel: per step, events around every launch over %d further steps"
                           % (kernel, depth, split_steps)) if fused_tiles > 0 else
                          "ib_kernel and lbm_kernel: per step, HIP events around every launch over the timed steps",
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_ratio": round(traffic / achieved, 4) if traffic else None,
                     "kernel": kernel, "bytes_per_update": bytes_per_update,
                     "nodes_per_launch": launch_nodes, "launch_ms": round(launch_ms, 5),
                     # the same launches priced at one read and one write of
                     # the 9 populations per lattice update (72 B in FP32),
                     # as if every update went through HBM, and the whole
                     # step (immersed boundary included) at that price
                     "single_step_accounting": {
                         "bytes_per_update": node_bytes,
                         "kernel_achieved": round(launch_nodes * depth * node_bytes / (launch_ms * 1e-3) / 1e9, 1),
                         "kernel_frac": round(launch_nodes * depth * node_bytes / (launch_ms * 1e-3) / 1e9
                                              / HBM_PEAK_GBS, 4),
                         "step_achieved": round(n * node_bytes / (ms_step * 1e-3) / 1e9, 1),
                         "step_frac": round(n * node_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}},
        "repeats": len(walls),
        "ms_per_step_repeats": [round(w * 1e3 / args.steps, 5) for w in walls],
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if args.workload == "particles" and args.delta in ("cos4", "roma3") and not args.no_other_delta:
        other = "roma3" if args.delta == "cos4" else "cos4"
        line["other_delta"] = bench_other_delta(args, other)
        torch.cuda.empty_cache()
    if not args.no_batched:
        line["batched"] = bench_batched(args)
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        line["adjoint"] = bench_adjoint(args)
        torch.cuda.empty_cache()
    if not args.no_validation:
        line["validation"] = bench_validation(args)
        torch.cuda.empty_cache()
    if not args.no_shedding:
        line["shedding"] = bench_shedding(args)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_budget_s, args.cpu_one_core_budget_s)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
