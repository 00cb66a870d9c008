"""SDC zone-updates/s on one MI355X (Castro, Sec. 2, Eq. 2).

    python bench.py [--steps K] [--warmup W] [--workload net3d] [--precision both]

Default workload: the 3D 256^3 grid with the 13-species / 20-reaction seeded
network, 3 Gauss-Lobatto nodes (Simpson), K = 4 SDC iterations per step,
MC slopes and local Rusanov speeds, CFL time step.  A step is one full pass of
the hot path: 4 iterations x 2 node transitions (fused quadrature, explicit
update and per-zone Newton) plus the advective term at every new node.  Inputs
are resident in HBM before the timed region, which brackets exactly K steps
with device synchronisation and no per-launch instrumentation.  Prints one
JSON line.

The FP64 path gives `value`; the mixed path (FP32 Newton matrix and LU) is
reported beside it, and so are the 2D 512^2 workload (7 species), the
batched-box workload (plain launches and captured graphs, with its Newton
iteration histogram) and the adjoint/forward time ratio.  After the timed
steps, the same number of steps runs again with HIP events around every
launch (on the launch stream): `kernels` lists each kernel's summed and mean
launch time, share and fraction of the HBM and FP64 ceilings, and `roofline`
covers the kernel with the largest summed time, against the ceiling its
algorithmic bytes and flops make binding; `traffic` is the HBM bytes per
launch from the committed counter summary when that was taken on the same
kernel source.  `cpu_baseline` times the CPU oracle on sub-blocks of the same
workload, one process per core the job may use.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import sdc_inputs as si  # noqa: E402

PEAK_FP64_TFLOPS = 78.6  # MI355X vector FP64 (FMA counts 2)
PEAK_HBM_GBS = 8000.0


def kernel_model(h, stats, dim):
    """Algorithmic FP64 bytes and flops per zone of each kernel launch.

    Bytes: every state, advective, source and correction array a kernel reads
    or writes, once each, 8 bytes per value.  Flops: a Newton iteration costs
    the residual/matrix assembly, the LU and the triangular solves of the
    generated network code (exp and log count one each) plus 2 n_x for the
    update and the test; a solve adds one R(x) at the root and the explicit
    update (about 4 n_c); the quadrature of the m = 0 transition adds
    2 (M+1)(n_c + n_x) per correction term.  The advective term counts, per
    direction, the reconstruction and Rusanov flux of every component
    ((9 n_c + 40 + 3 n_c) per face) and the divergence (2 n_c).  The Newton
    count is the measured mean over the timed steps.
    """
    cm = h.cost_model()
    nx, nc, M = h.nreact_vars, h.ncomp, h.n_nodes - 1
    per_iter = cm["residual_matrix"] + cm["lu"] + cm["solve"] + 2 * nx
    per_solve = cm["source"] + 4 * nc
    nu = stats["iters"] / max(stats["solves"] - stats["failed"], 1)
    newton = nu * per_iter + per_solve
    words = {
        "transition_first": 3 * nc + (nc + nx),
        "transition_node0": (M + 1) * (nc + nx) + 2 * nc + (nc + nx) + (M - 1) * nc,
        "transition_later": 4 * nc + (nc + nx),
        "advect": 2 * nc,
        "source": nc + nx,
    }
    flops = {
        "transition_first": newton + 2 * nc,
        "transition_node0": newton + 2 * (M + 1) * (nc + nx) * M,
        "transition_later": newton + 3 * nc,
        "advect": ((9 * nc + 40 + 3 * nc) + 2 * nc) * dim,
        "source": cm["source"],
    }
    return {k: 8.0 * v for k, v in words.items()}, flops, per_iter, per_solve


def kernel_model4(h, stats, dim):
    """Algorithmic bytes (and flops where counted) per zone of each kernel kind
    of the fourth-order method.  The advective term counts what an evaluation
    must move (read U, write A: 2 n_c values), spread over its 3 dim launches
    (face averages, face fluxes and their divergence per direction); the transition kinds
    are the right-hand-side kernels (state, advective, correction and source
    inputs, the rhs and the Newton guess out); `order4` averages the
    zone-centre Newton-input kernel (rhs in; rho_c and b_c out) and the average
    store (R_c, rhs in; U, <R> out); `solve` is the per-zone Newton kernel
    (rho, b, guess in; root, R and iteration count out); `source` averages the
    centre-source and conversion kernels."""
    cm = h.cost_model()
    nx, nc, M = h.nreact_vars, h.ncomp, h.n_nodes - 1
    per_iter = cm["residual_matrix"] + cm["lu"] + cm["solve"] + 2 * nx
    nu = stats["iters"] / max(stats["solves"] - stats["failed"], 1)
    words = {
        "advect": 2 * nc / (3 * dim),
        "transition_first": 4 * nc + nx,
        "transition_node0": 2 * nc + (M + 1) * (nc + nx) + (M - 1) * nc + nc + nx,
        "transition_later": 5 * nc + nx,
        "order4": 0.5 * ((nc + nx + 1) + 4 * nx),
        "solve": 4 * nx + 1.5,
        "source": 0.5 * (nc + 3 * nx),
    }
    flops = {"solve": nu * per_iter + cm["source"]}
    return {k: 8.0 * v for k, v in words.items()}, flops, per_iter, cm["source"]


def roofline(bytes_per_zone, flops_per_zone, zones, avg_s):
    """Roofline of one kernel from its algorithmic bytes and flops per launch
    and its measured mean launch time: the binding ceiling is the larger of
    bytes / HBM peak and flops / FP64 peak."""
    B, F = bytes_per_zone * zones, flops_per_zone * zones
    t_hbm, t_alu = B / (PEAK_HBM_GBS * 1e9), F / (PEAK_FP64_TFLOPS * 1e12)
    hbm = dict(achieved=B / avg_s / 1e9, peak=PEAK_HBM_GBS, unit="GB/s", frac=t_hbm / avg_s)
    alu = dict(achieved=F / avg_s / 1e12, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s", frac=t_alu / avg_s)
    bound = "hbm" if t_hbm >= t_alu else "alu"
    main = hbm if bound == "hbm" else alu
    return dict(bound=bound, **main, bytes_per_launch=B, flops_per_launch=F, avg_launch_ms=1e3 * avg_s,
                hbm_frac=hbm["frac"], alu_frac=alu["frac"], alu_TFLOPs=alu["achieved"], hbm_GBs=hbm["achieved"])


def kernel_name(kind, dim, sched, precision, order=2):
    """Name of the kernel that a profiled kind stands for under a schedule."""
    if order == 4:
        return {"advect": "sdc_faceavg4_d+sdc_flux4_d+sdc_div4_d", "order4": "sdc_newton_inputs4+sdc_average_store4",
                "solve": "sdc_reaction_solve" + ("_o2" if sched["occ2"] else ""),
                "source": "sdc_source4_centre+sdc_convert4"}.get(kind, "sdc_rhs4_" + kind.split("_")[-1])
    if kind == "advect":
        return "sdc_advect_rows" if dim == 3 else "sdc_advect"
    if kind == "order4":
        return "sdc_newton_inputs4+sdc_average_store4"
    if kind.startswith("transition_"):
        return "sdc_" + kind + ("_o2" if sched["occ2"] else "")
    return "sdc_" + kind


def recorded_traffic(h, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summaries
    (profiles/hbm_traffic_*.md), if one was taken on this kernel and on the
    source this handle compiled (else None).  A summary's machine-readable
    record holds `source_sha256_16` and one `traffic_bytes_per_launch[<kernel>]`
    line per kernel."""
    import glob
    import hashlib
    digest = hashlib.sha256(h.generated_source().encode()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md"))):
        rec = {}
        with open(path) as f:
            for line in f:
                if line.startswith("- ") and ": " in line:
                    k, v = line[2:].split(": ", 1)
                    rec[k.strip()] = v.strip().strip("`")
        key = f"traffic_bytes_per_launch[{kernel}]"
        if rec.get("source_sha256_16") == digest and key in rec:
            return float(rec[key]), digest
    return None, digest


def make_handle(w, precision, schedule, graph=0):
    """'auto': the handle tunes its schedule on its first step (or reads the
    choice cached on disk for this kernel source and size); otherwise the
    comma-separated schedule (occupancy variant, iteration cap, split batches,
    advection tile).  graph=1: every step replays a captured HIP graph."""
    from paper_1910_12578_amd import SDC, config_from_workload
    h = SDC(config_from_workload(w, precision=precision, autotune=int(schedule == "auto"), graph=graph),
            w["network"])
    if schedule != "auto":
        vals = [int(v) for v in schedule.split(",")]
        h.set_schedule(*vals)
    return h


def warm(h, dt, U, work, warmup, schedule):
    """Untimed warmup steps; the first one includes the schedule tuning."""
    import torch
    t0 = time.perf_counter()
    if warmup > 0:
        h.step(dt, warmup, U, work)
    elif schedule == "auto":
        h.autotune(dt, U, work)
    torch.cuda.synchronize()
    occ2, cap, split, zchunk = h.schedule()
    return dict(occ2=occ2, cap=cap, split=split, zchunk=zchunk, mode=schedule,
                warmup_s=round(time.perf_counter() - t0, 3))


def kernel_table(h, w, st, prof, sched, precision):
    """Per-kernel summary of a profiled pass: summed and mean launch time,
    share of the kernel time, algorithmic bytes per launch and the fraction of
    the HBM and FP64 ceilings each reaches; the dominant kernel (largest summed
    time) and its roofline."""
    Z = w["U0"][0].size
    model = kernel_model4 if w.get("space_order", 2) == 4 else kernel_model
    bpz, fpz, per_iter, per_solve = model(h, st, w["dim"])
    total = sum(v[0] for v in prof.values())
    table = {}
    for k, (ms, n) in prof.items():
        if not n:
            continue
        row = dict(ms=round(ms, 3), launches=n, avg_ms=round(ms / n, 4), share=round(ms / total, 4))
        if k in bpz:
            r = roofline(bpz[k], fpz.get(k, 0.0), Z, ms * 1e-3 / n)
            # flops are counted only where the model has them (null otherwise)
            row.update(bytes_per_zone=bpz[k], hbm_frac=round(r["hbm_frac"], 4),
                       fp64_frac=round(r["alu_frac"], 4) if k in fpz else None)
        table[k] = row
    dom = max(table, key=lambda k: table[k]["ms"])
    roof = roofline(bpz[dom], fpz.get(dom, 0.0), Z, prof[dom][0] * 1e-3 / prof[dom][1])
    if dom not in fpz:
        roof.update(alu_frac=None, alu_TFLOPs=None)
    kname = kernel_name(dom, w["dim"], sched, precision, w.get("space_order", 2))
    roof["traffic"], digest = recorded_traffic(h, kname)
    roof["kernel"] = kname
    roof["share"] = table[dom]["share"]
    step_bytes = sum(bpz[k] * Z * prof[k][1] for k in bpz if prof[k][1])
    return table, roof, step_bytes, digest, per_iter, per_solve


def run_gpu(w, precision, steps, warmup, schedule="auto", graph=0):
    """Timed steps with profiling off (value, ms_per_step), then the same
    number of steps with HIP events around every launch (per-kernel table and
    roofline of the dominant kernel)."""
    import torch
    h = make_handle(w, precision, schedule, graph=graph)
    nc = w["U0"].shape[0]
    U0 = torch.from_numpy(w["U0"].reshape(nc, -1)).to("cuda")
    U = U0.clone()
    work = h.alloc_nodes()
    dt = w["dt"]
    stream = torch.cuda.current_stream()
    sched = warm(h, dt, U, work, warmup, schedule)
    # the timed steps start from the initial state
    U.copy_(U0)
    h.stats_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.step(dt, steps, U, work, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = h.stats()
    check = h.check()[0]
    ok = bool(torch.isfinite(U).all().item())
    Z = w["U0"][0].size
    U.copy_(U0)  # the profiled pass repeats the same steps
    h.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.step(dt, steps, U, work, stream=stream)
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t1
    prof = h.profile_read()
    h.profile(False)
    table, roof, step_bytes, digest, per_iter, per_solve = kernel_table(h, w, st, prof, sched, precision)
    res = dict(
        elapsed=elapsed, ms_per_step=1e3 * elapsed / steps, zone_updates=Z * steps / elapsed,
        zone_sweeps=Z * steps * w["n_iters"] / elapsed,
        ms_per_step_profiled=1e3 * elapsed_prof / steps,
        stats=st, mean_newton=st["iters"] / max(st["solves"] - st["failed"], 1), finite=ok, check=check,
        kernels=table, roofline=roof, step_hbm_frac=step_bytes / elapsed_prof / (PEAK_HBM_GBS * 1e9),
        flops_per_newton_iteration=per_iter, flops_per_solve=per_solve,
        cost_model=h.cost_model(), schedule=sched, source_sha256_16=digest,
    )
    h.close()
    del U, U0, work
    torch.cuda.empty_cache()
    return res


def run_adjoint_ratio(nsteps=20):
    """Forward vs backward time of the adjoint workload (256^2, 7 species,
    smooth mode): forward = nsteps SDC steps keeping one checkpoint per step;
    backward = nsteps step adjoints (replay + reverse sweeps)."""
    import torch
    from paper_1910_12578_amd import SDC, config_from_workload
    w = si.workload("adjoint2d")
    h = SDC(config_from_workload(w), w["network"])
    nc = w["U0"].shape[0]
    U0 = torch.from_numpy(w["U0"].reshape(nc, -1)).to("cuda")
    work = h.alloc_nodes()
    dt = w["dt"]
    seed = torch.zeros_like(U0)
    seed[2 + w["dim"]:2 + w["dim"] + w["network"]["nspec"]] = -torch.tensor(
        w["network"]["q"], device="cuda")[:, None] * float(np.prod(w["dx"]))
    thetabar = torch.zeros(2 * h.nreact, dtype=torch.float64, device="cuda")

    def forward():
        U = U0.clone()
        ck = []
        for _ in range(nsteps):
            ck.append(U.clone())
            h.step(dt, 1, U, work)
        return U, ck

    def backward(ck):
        Ub = seed.clone()
        for U_n in reversed(ck):
            Ub, _ = h.step_adjoint(dt, U_n, Ub, None, thetabar)
        return Ub

    _, ck = forward()
    backward(ck)  # warm (allocates the adjoint workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, ck = forward()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    backward(ck)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    h.close()
    return dict(workload=f"adjoint2d 256x256, 7 species / 10 reactions, smooth mode, {nsteps} steps",
                forward_ms=1e3 * (t1 - t0), backward_ms=1e3 * (t2 - t1), ratio=(t2 - t1) / (t1 - t0))


def run_boxes(w, steps, warmup, precision, schedule="auto", graphs=(0, 1)):
    """Batched boxes: independent periodic boxes of uneven size, one launch per
    kernel over all boxes; then the same steps replayed from captured HIP
    graphs (one per buffer-rotation phase of a step).  The timed steps start
    from the initial state, whose hot tail (the lognormal temperature) burns
    in the first steps and spreads the Newton counts."""
    import torch
    Z = w["U0"].shape[1]
    out = {}
    U0 = torch.from_numpy(w["U0"]).to("cuda")
    for graph in graphs:
        h = make_handle(w, precision, schedule, graph=graph)
        U = U0.clone()
        work = h.alloc_nodes()
        sched = warm(h, w["dt"], U, work, max(warmup, 1) if graph else warmup, schedule)
        U.copy_(U0)
        h.stats_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.step(w["dt"], steps, U, work)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = h.stats()
        if graph:
            out["graph"] = dict(zone_updates=Z * steps / el, ms_per_step=1e3 * el / steps)
        else:
            out.update(zone_updates=Z * steps / el, ms_per_step=1e3 * el / steps,
                       mean_newton=st["iters"] / max(st["solves"] - st["failed"], 1), failed=st["failed"],
                       nonfinite=st["nonfinite"], newton_hist={i: v for i, v in enumerate(st["hist"]) if v},
                       schedule=sched)
        h.close()
        del U, work
        torch.cuda.empty_cache()
    del U0
    torch.cuda.empty_cache()
    return out


def run_amr(w, patches, steps, warmup):
    """Two-level hierarchy: the single-grid workload as the coarse level and
    `patches` (lo, ext in coarse zones) refined by 2 with subcycling.  The
    timed coarse steps start from the initial state with interpolated patches;
    zone-updates count every coarse zone once and every patch zone (ghosts
    excluded) twice per coarse step."""
    import torch
    from paper_1910_12578_amd import AMR, config_from_workload
    a = AMR(config_from_workload(w, autotune=1), w["network"], patches)
    nc = w["U0"].shape[0]
    U0 = torch.from_numpy(w["U0"].reshape(nc, -1)).to("cuda")
    Uc = U0.clone()
    Uf = torch.empty((nc, a.zf), dtype=torch.float64, device="cuda")
    a.fill_patches(Uc, Uf)
    if warmup:
        a.step(w["dt"], warmup, Uc, Uf)
    Uc.copy_(U0)
    a.fill_patches(Uc, Uf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.step(w["dt"], steps, Uc, Uf)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    fine = sum(int(np.prod([2 * e for e in ext])) for _, ext in patches)
    updates = (w["U0"][0].size + 2 * fine) * steps
    st = a.stats()
    a.close()
    del U0, Uc, Uf
    torch.cuda.empty_cache()
    return dict(zone_updates=updates / el, ms_per_step=1e3 * el / steps, coarse_zones=w["U0"][0].size,
                patch_zones=fine, patches=[dict(lo=list(lo), ext=list(ext)) for lo, ext in patches],
                failed=st[0]["failed"] + st[1]["failed"], nonfinite=st[0]["nonfinite"] + st[1]["nonfinite"])


def _oracle_block(args):
    """One oracle step on one sub-block (runs in a worker process)."""
    light, U0, dt = args
    from threadpoolctl import threadpool_limits
    from oracle import sdc as osdc
    prob = osdc.Problem.from_workload(light)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        osdc.run(U0, dt, 1, prob)
        return time.perf_counter() - t0


def _warm_worker(_):
    from oracle import sdc as osdc  # noqa: F401  (import cost outside the timed map)
    return 0


def host_cores():
    """Cores this job may use: the CPU affinity set, bounded by OMP_NUM_THREADS
    when the environment sets it (the CPU share given to a one-GPU job)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(omp))) if omp.isdigit() and int(omp) > 0 else n


def cpu_baseline(w, edge, procs):
    """The oracle, one step of edge^3 sub-blocks of the same initial state:
    `procs` worker processes (one thread each) on distinct blocks at once,
    and one block alone on one thread."""
    import multiprocessing as mp
    dim = w["dim"]
    light = {k: v for k, v in w.items() if k != "U0"}
    light["shape"] = (edge,) * dim
    nb = w["shape"][0] // edge
    blocks = []
    for i in range(procs):
        o = (i % nb, (i // nb) % nb, (i // nb // nb) % nb)[:dim]
        sl = (slice(None),) + tuple(slice(c * edge, (c + 1) * edge) for c in o)
        blocks.append((light, np.ascontiguousarray(w["U0"][sl]), w["dt"]))
    zones = edge ** dim
    t1 = _oracle_block(blocks[0])
    out = dict(value=zones / t1, unit="zone-updates/s", cores=1, kind="oracle",
               sample=f"one step of a {edge}^{dim} block of the same initial state ({zones} zones, same dt, "
                      f"network and iteration counts), NumPy FP64, one thread: {t1:.1f} s")
    if procs > 1:
        ctx = mp.get_context("spawn")
        with ctx.Pool(procs) as pool:
            pool.map(_warm_worker, range(procs))
            t0 = time.perf_counter()
            ts = pool.map(_oracle_block, blocks, chunksize=1)
            wall = time.perf_counter() - t0
        out = dict(value=procs * zones / wall, unit="zone-updates/s", cores=procs, kind="oracle",
                   sample=f"{procs} processes of one thread, each one step of a different {edge}^{dim} block "
                          f"of the same initial state ({zones} zones each, same dt, network and iteration "
                          f"counts), NumPy FP64, wall {wall:.1f} s (slowest block {max(ts):.1f} s)",
                   single_thread=out)
    return out


def workload_label(w):
    grid = "x".join(map(str, w["shape"])) if w.get("shape") else f"{len(w['box_n'])} boxes"
    nodes = "Radau" if w.get("node_type") == "radau" else "Gauss-Lobatto"
    order = ", fourth order in space" if w.get("space_order", 2) == 4 else ""
    return (f"{w['name']} {grid}, {w['network']['nspec']} species / {w['network']['nreact']} reactions, "
            f"{w['n_nodes']} {nodes} nodes, K={w['n_iters']}{order}")


def advect_probe(edges):
    """The advective term of the net3d recipe on small cubic grids, six
    evaluations each (the row kernel), then a 1 GiB device copy: a program for
    counter runs that compare the bytes the kernel fetches from beyond L2 with
    the bytes it reads once (n_c x 8 per zone) on grids that fit in L2."""
    import torch
    from paper_1910_12578_amd import SDC, config_from_workload
    for n in edges:
        w = si.workload("net3d", shape=(n, n, n))
        nc = w["U0"].shape[0]
        U = torch.from_numpy(w["U0"].reshape(nc, -1)).to("cuda")
        with SDC(config_from_workload(w), w["network"]) as h:
            A = h.advective_term(U)
            for _ in range(5):
                h.advective_term(U, A)
            torch.cuda.synchronize()
        print(json.dumps(dict(grid=n, zones=n ** 3, bytes_read_once=n ** 3 * nc * 8, evaluations=6)), flush=True)
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=8 << 27)), flush=True)


def gpu_leg(w, steps, warmup, schedule, precisions=("fp64", "mixed")):
    """FP64 and mixed runs of one single-grid workload, summarised."""
    out = {}
    for name in precisions:
        prec = 0 if name == "fp64" else 1
        print(f"[bench] {w['name']} {name}: warmup {warmup}, timed {steps} steps", file=sys.stderr, flush=True)
        out[name] = run_gpu(w, prec, steps, warmup, schedule)
        print(f"[bench] {w['name']} {name}: {out[name]['zone_updates']:.4e} zone-updates/s "
              f"({out[name]['ms_per_step']:.2f} ms/step)", file=sys.stderr, flush=True)
    return out


def summary(r):
    return dict(value=r["zone_updates"], ms_per_step=r["ms_per_step"],
                ms_per_step_profiled=r["ms_per_step_profiled"], mean_newton_iterations=r["mean_newton"],
                newton_failed=r["stats"]["failed"], schedule=r["schedule"],
                roofline={k: r["roofline"][k] for k in ("kernel", "share", "bound", "frac", "achieved", "unit",
                                                        "avg_launch_ms", "hbm_frac", "alu_frac", "traffic")},
                step_hbm_frac=r["step_hbm_frac"], kernels=r["kernels"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="net3d")
    ap.add_argument("--shape", default=None, help="override grid, e.g. 64,64,64")
    ap.add_argument("--precision", default="both", choices=("fp64", "mixed", "both"))
    ap.add_argument("--cpu-edge", type=int, default=48)
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle worker processes for cpu_baseline, one thread each (0: every core the job may use)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward time ratio")
    ap.add_argument("--no-boxes", action="store_true", help="skip the batched-box workload")
    ap.add_argument("--no-net2d", action="store_true", help="skip the 2D 512^2 workload")
    ap.add_argument("--no-order4", action="store_true", help="skip the fourth-order-in-space leg")
    ap.add_argument("--no-amr", action="store_true", help="skip the refined-patch (two-level) leg")
    ap.add_argument("--space-order", type=int, default=2, choices=(2, 4), help="spatial order of the main workload")
    ap.add_argument("--node-type", default="lobatto", choices=("lobatto", "radau"), help="nodes of the main workload")
    ap.add_argument("--schedule", default="auto",
                    help="schedule: 'auto' (tuned on the first warmup step) or 'OCC2,CAP[,SPLIT[,ZCHUNK]]', e.g. 0,0,0,16")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--advect-probe", default="",
                    help="only evaluate the advective term six times on each of these cubic grids (e.g. "
                         "16,24,32,64; small enough to stay in L2) and copy 1 GiB, for byte-counter runs")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); multi-GPU sharding is a design "
              f"note, not a measured path", file=sys.stderr)
        sys.exit(2)
    if a.advect_probe:
        advect_probe([int(v) for v in a.advect_probe.split(",")])
        return
    shape = tuple(int(v) for v in a.shape.split(",")) if a.shape else None
    print(f"[bench] generating {a.workload} {shape or ''}", file=sys.stderr, flush=True)
    w = si.workload(a.workload, shape=shape)
    w["space_order"] = a.space_order
    w["node_type"] = a.node_type
    Z = w["U0"][0].size
    precs = ("fp64", "mixed") if a.precision == "both" else (a.precision,)
    runs = gpu_leg(w, a.steps, a.warmup, a.schedule, precs)
    head = runs.get("fp64") or runs["mixed"]
    label = workload_label(w)
    out = dict(
        metric=f"SDC zone-updates/s, {label}, {'FP64' if 'fp64' in runs else 'mixed'} "
               f"(mixed precision, other workloads and adjoint/forward time beside it)",
        value=head["zone_updates"],
        unit="zone-updates/s",
        n_gpus=1, steps=a.steps, warmup=a.warmup,
        ms_per_step=head["ms_per_step"],
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64" if "fp64" in runs else "f64+f32lu",
        data="synthetic",
        config=dict(workload=label, zones=Z, dt=w["dt"]),
        roofline=dict(head["roofline"]),
        step_hbm_frac=head["step_hbm_frac"],
        zone_sweeps_per_s=head["zone_sweeps"],
        ms_per_step_profiled=head["ms_per_step_profiled"],
        schedule=head["schedule"],
        mean_newton_iterations=head["mean_newton"],
        newton_failed=head["stats"]["failed"],
        newton_hist={i: v for i, v in enumerate(head["stats"]["hist"]) if v},
        kernels=head["kernels"],
    )
    if "mixed" in runs and "fp64" in runs:
        out["mixed"] = summary(runs["mixed"])
        out["mixed"]["speedup_vs_fp64"] = runs["mixed"]["zone_updates"] / runs["fp64"]["zone_updates"]
    others = {}
    if not a.no_net2d and a.workload != "net2d" and shape is None:
        w2 = si.workload("net2d")
        r2 = gpu_leg(w2, a.steps, a.warmup, a.schedule, precs)
        others["net2d"] = dict(workload=workload_label(w2), zones=w2["U0"][0].size,
                               **{k: summary(v) for k, v in r2.items()})
        del w2
    if not a.no_order4 and a.space_order == 2 and shape is None and w["dim"] == 3:
        w4 = dict(w, space_order=4)
        r4 = gpu_leg(w4, a.steps, a.warmup, a.schedule, ("fp64",))
        others["order4"] = dict(workload=workload_label(w4), zones=Z, **{k: summary(v) for k, v in r4.items()})
        del w4
    if not a.no_amr and a.space_order == 2 and a.node_type == "lobatto" and shape is None and w["dim"] == 3:
        # x extents of 62 coarse zones: padded patch rows of 128 fine zones fill the row kernel's blocks
        patches = [((32, 40, 48), (62, 64, 64)), ((150, 130, 120), (62, 64, 80))]
        print("[bench] refined patches", file=sys.stderr, flush=True)
        r = run_amr(w, patches, a.steps, a.warmup)
        others["amr"] = dict(workload=workload_label(w) + " coarse level, patches refined by 2 with subcycling", **r)
        print(f"[bench] refined patches: {r['zone_updates']:.4e} zone-updates/s ({r['ms_per_step']:.1f} ms per "
              f"coarse step)", file=sys.stderr, flush=True)
    if not a.no_boxes and shape is None:
        print("[bench] generating batched boxes", file=sys.stderr, flush=True)
        wb = si.boxes_workload()
        Zb = wb["U0"].shape[1]
        box = dict(workload=workload_label(wb) + f", {Zb} zones, dt {wb['dt']:.3e}", zones=Zb)
        for name in precs:
            print(f"[bench] boxes {name}", file=sys.stderr, flush=True)
            box[name] = run_boxes(wb, a.steps, a.warmup, 0 if name == "fp64" else 1, a.schedule)
            print(f"[bench] boxes {name}: {box[name]['zone_updates']:.4e} zone-updates/s", file=sys.stderr, flush=True)
        others["boxes"] = box
        del wb
    if others:
        out["workloads"] = others
    if not a.no_adjoint:
        print("[bench] adjoint/forward ratio", file=sys.stderr, flush=True)
        out["adjoint"] = run_adjoint_ratio()
    if a.copy_probe_mib:
        import torch
        n = a.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 8 * n
        del src, dst
    if not a.no_cpu_baseline:
        procs = a.cpu_procs or host_cores()
        print(f"[bench] cpu baseline (oracle, {procs} processes)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_edge, procs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
