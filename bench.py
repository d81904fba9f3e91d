#!/usr/bin/env python3
"""Benchmark of the parareal-with-splitting hot path on one MI355X.

Workload (default): 2D u_t = div(a grad u), a = 1 + 0.5 sin(2 pi x) cos(2 pi y),
1023 x 1023 interior nodes, FP64, N = 64 slices, s = 64 fine FIE steps per
slice, one coarse FIE step, synthetic seeded u0 (16 sine modes).

One timed step = one parareal iteration = the fine propagator on all 64 slices
(pr_fine_propagate: 64 x 64 FIE steps = 4.29e9 point-updates) plus the serial
coarse sweep fused with the correction and the increment (pr_coarse_sweep).
value = fine point-updates per second over the whole step, in Gpts/s.

Also reported: the fine sweep kernel's roofline (algorithmic bytes per launch
over its mean launch time from hipEvents on the work stream, one event pair
around each step's loop of sweeps, so the mean includes the gaps between
launches), the oracle timed
on a bounded sample on the host, and the parareal wall time to tolerance
against the sequential fine solve on the same GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fine-propagator Gpts/s + % HBM roofline; parareal wall time vs plain loop"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def oracle_problem(w):
    import oracle
    if w.theta is not None:
        ax, ay = oracle.faces_from_theta(w.nx, w.ny, w.theta, dim=w.dim)
    else:
        ax, ay = w.ax, w.ay
    return oracle.Problem(dim=w.dim, nx=w.nx, ny=w.ny, T=w.T, n_slices=w.n_slices,
                          fine_steps=w.fine_steps, split=w.split, ax=ax, ay=ay, rho=w.rho)


def covered_nodes(w):
    """Nodes each colour's substep solves for (its components: runs of faces with rho > 0,
    node range [first face - 1, last face]); the other nodes are untouched."""
    tot = []
    for r in w.rho:
        pos = r > 0
        cover = np.zeros(w.nx, bool)
        cover |= pos[1:]      # face f+1 > 0 touches node f
        cover |= pos[:-1]     # face f > 0 touches node f (f < n)
        tot.append(int(cover.sum()))
    return tot


def dd2_strips(w):
    """Strips (colour, first column, width) of the 2D strip decomposition: maximal runs of
    columns where the colour's weight is nonzero on the node or an x-face."""
    out = []
    for k, r in enumerate(w.rho):
        act = (r[0:-1:2] > 0) | (r[1::2] > 0) | (r[2::2] > 0)
        i = 0
        while i < w.nx:
            if not act[i]:
                i += 1
                continue
            j = i
            while j < w.nx and act[j]:
                j += 1
            out.append((k, i, j - i))
            i = j
    return out


def dd2_substep_bytes(w, N):
    """Algorithmic bytes of one colour substep of the strip solver, averaged over the
    colours: every dense w x w block the block cyclic reduction stores at levels >= 1
    (padded to W, a multiple of 16) read once; at level 0 the LU of each eliminated
    row read twice (3 vectors forward and back, plus its 2 coupling vectors in the
    back substitution) and the 2 coupling vectors of each kept row; plus one read
    and one write of every node of the colour's strips for each slice."""
    ny = w.ny
    tot = []
    for k in range(len(w.rho)):
        b = 0.0
        for kk, i0, ws in dd2_strips(w):
            if kk != k:
                continue
            Wp = (ws + 15) // 16 * 16
            mats = 0
            l = 1
            while (ny >> l) > 0:
                n = ny >> l
                for a in range(n):
                    mats += (1 + (a >= 1) + (a + 1 < n)) if a % 2 == 0 else (1 + (a + 1 < n))
                l += 1
            vecs = 8 * ((ny + 1) // 2) + 2 * (ny // 2)
            b += 8.0 * Wp * (Wp * mats + vecs) + 16.0 * ws * ny * N
        tot.append(b)
    return float(np.mean(tot))


def measured_traffic(kernel_src, summary):
    """HBM bytes per launch from the committed byte-counter summary, or None when the
    kernel source has changed since the counters were taken (or no summary exists)."""
    import hashlib
    try:
        fig = json.load(open(summary))
        h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
    except (OSError, ValueError):
        return None
    return fig["traffic_bytes_per_launch"] if fig.get("source_sha256_16") == h else None


def sweep_label(prob):
    """Name and form of the fine sweep kernel the handle launches."""
    tw, gr, m = (prob.get_option(k) for k in ("twisted", "grouped", "fine_chunk"))
    if prob.get_option("partitioned_used") > 0:
        return "k_part_sweep (one workgroup per line, parts of up to 24 positions per lane)"
    ins = prob.instances[0]
    lanes = max(8, min(64, 1 << (ins["n_slices"] - 1).bit_length()))
    if ins["fine"] == 1:  # Douglas-Rachford sweeps use the short chunk
        return f"k_fine_sweep ({'two waves' if tw else 'one wave'} per line, chunk 16, DR)"
    if tw and gr and lanes == 64 and m in (20, 24):
        return f"k_fine_sweep_g (four lines per workgroup, two waves per line, chunk {m})"
    return f"k_fine_sweep ({'two waves' if tw else 'one wave'} per line, chunk {m})"


def cpu_baseline(w, budget_s):
    """Oracle (serial FP64 C, one thread) on a bounded sample of the same workload:
    the fine propagator on one slice for as many fine steps as fit the budget."""
    P = oracle_problem(w)
    dt = w.T / w.n_slices / w.fine_steps
    u = np.ascontiguousarray(w.u0)
    t0 = time.perf_counter()
    u = P.fie_step(u, dt)
    one = time.perf_counter() - t0
    steps = max(1, int(budget_s / max(one, 1e-6)))
    t0 = time.perf_counter()
    for _ in range(steps):
        u = P.fie_step(u, dt)
    el = time.perf_counter() - t0
    pts = w.nx * w.ny * steps
    shape = f"{w.nx}x{w.ny}" if w.dim == 2 else f"{w.nx}-node"
    return {"value": pts / el / 1e9, "unit": "Gpts/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle FIE steps on one {shape} slice: {steps} fine steps "
                      f"({pts:.3g} point-updates) in {el:.2f} s",
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}


def cpu_baseline_dd2(w):
    """Oracle on a bounded sample of the strip workload: one FIE step of a grid the size
    of the workload's widest strip with a single colour (rho = 1), i.e. one strip solve
    (banded elimination, factor and solve, as the oracle does every substep)."""
    import oracle
    ws = max(width for _, _, width in dd2_strips(w))
    P = oracle.Problem(dim=2, nx=ws, ny=w.ny, T=w.T, n_slices=1, fine_steps=1, split="dd",
                       ax=np.ones((w.ny, ws + 1)), ay=np.ones((w.ny + 1, ws)),
                       rho=np.ones((1, 2 * ws + 1)))
    u = np.ascontiguousarray(w.u0[:, :ws])
    t0 = time.perf_counter()
    P.fie_step(u, w.T / w.n_slices / w.fine_steps)
    el = time.perf_counter() - t0
    pts = ws * w.ny
    return {"value": pts / el / 1e9, "unit": "Gpts/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle solve of one {ws}x{w.ny} strip (the widest strip of the "
                      f"workload, one colour substep of one component) in {el:.2f} s",
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_batch(args):
    """Batched parareal over uneven instances in one handle (grouped fine sweeps,
    batched coarse sweeps, graph-captured corrections, per-instance convergence)
    against the plain loop: one single-instance handle per instance, direct
    launches, the same per-instance iteration count (so the same accuracy)."""
    import torch
    import paper_2502_08370_amd as pr
    import workloads as W
    ws = W.config4(n_instances=args.instances)
    dev = torch.device("cuda:0")

    def inst(w):
        return dict(dim=2, nx=w.nx, ny=w.ny, T=w.T, n_slices=w.n_slices,
                    fine_steps=w.fine_steps, theta=w.theta)

    t0 = time.perf_counter()
    P = pr.Problem([inst(w) for w in ws])
    P.set_option("partitioned", args.partitioned)
    torch.cuda.synchronize()
    log(f"batch handle: {len(ws)} instances, created in {time.perf_counter() - t0:.2f} s, "
        f"{P.get_option('partitioned_used')} with partitioned sweeps")
    tune = P.autotune() if args.autotune else None
    if tune:
        log(f"autotune: {tune}")
    u0 = P.pack_u0([w.u0 for w in ws])
    kmax = max(w.n_slices for w in ws)
    U = P.new_states()
    P.parareal_iterate(u0, U, k_max=1, tol=0.0)  # warm-up (graph capture)
    torch.cuda.synchronize()
    time.sleep(0.1)  # an idle gap that marks the timed region in kernel traces
    t0 = time.perf_counter()
    k, inc = P.parareal_iterate(u0, U, k_max=kmax, tol=ws[0].tol)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    pts = sum(w.nx * w.ny * w.n_slices * w.fine_steps * ki for w, ki in zip(ws, k))
    log(f"batched: {t_batch:.3f} s, iterations per instance {min(k)}..{max(k)}, "
        f"{pts / t_batch / 1e9:.1f} Gpts/s")
    del P, U, u0
    torch.cuda.empty_cache()
    # the plain loop: one single-instance handle per instance, the same per-instance
    # iteration count, with direct launches and with each handle's own captured graph
    # (captured in an untimed first call, as the batched handle's was)
    loops = {}
    max_diff = 0.0
    for use_graph in ((0, 1) if not args.no_loop else ()):
        t_loop = 0.0
        for i, w in enumerate(ws):
            Pi = pr.Problem([inst(w)])
            Pi.set_option("partitioned", args.partitioned)
            Pi.set_option("graph", use_graph)
            ui = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()
            Ui = Pi.new_states()
            if use_graph or i == 0:
                Pi.parareal_iterate(ui, Ui, k_max=1, tol=0.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ki, inci = Pi.parareal_iterate(ui, Ui, k_max=k[i], tol=0.0)
            torch.cuda.synchronize()
            t_loop += time.perf_counter() - t0
            max_diff = max(max_diff, abs(inci[0] - inc[i]) / max(abs(inc[i]), 1e-300))
            del Pi, Ui
        loops[use_graph] = t_loop
        log(f"loop of single-instance handles ({'graph' if use_graph else 'direct launches'}): "
            f"{t_loop:.3f} s ({t_loop / t_batch:.2f}x the batched time)")
    if loops:
        log(f"last-increment relative agreement with the batched run {max_diff:.1e}")
    t_loop = loops.get(0)
    result = {
        "metric": METRIC, "value": round(pts / t_batch / 1e9, 3), "unit": "Gpts/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * t_batch, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch{len(ws)}_2d_uneven", "instances": len(ws),
                   "grids": "n in {63,127,255,511}", "slices": "N in {16,32,64}",
                   "fine_steps": ws[0].fine_steps, "tol": ws[0].tol,
                   "step": "parareal to tolerance on every instance"},
        "batched_wall_s": round(t_batch, 4),
        "loop_wall_s": None if args.no_loop else round(loops[0], 4),
        "loop_graph_wall_s": None if args.no_loop else round(loops[1], 4),
        "batched_speedup_vs_loop": None if args.no_loop else round(loops[0] / t_batch, 3),
        "batched_speedup_vs_loop_graph": None if args.no_loop else round(loops[1] / t_batch, 3),
        "iterations": {"min": min(k), "max": max(k), "mean": round(float(np.mean(k)), 2)},
        "fine_point_updates": pts, "autotune": tune,
    }
    print(json.dumps(result), flush=True)


def bench_adjoint(args):
    """Gradient of 0.5 ||u(T) - u_obs||^2 with respect to u0 and theta on the
    differentiation workload (511^2, N = 32, s = 32): the serial adjoint (one
    reverse chain of N*s steps, per-slice recompute) against the parallel-in-time
    adjoint (boundary adjoints by the transposed problem, exact or by backward
    parareal to a tolerance, then every slice's recompute and reverse steps at
    once). value = differentiated fine point-updates per second of the parallel
    adjoint with exact boundary adjoints."""
    import torch
    import paper_2502_08370_amd as pr
    import workloads as W
    w = W.config5()
    dev = torch.device("cuda:0")
    n, N, s = w.nx, w.n_slices, w.fine_steps
    P = pr.Problem([dict(dim=2, nx=n, ny=n, T=w.T, n_slices=N, fine_steps=s, theta=w.theta)])
    Pstar = pr.Problem([dict(dim=2, nx=n, ny=n, T=w.T, n_slices=N, fine_steps=s,
                             theta=w.extra["theta_star"])])
    u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()
    Us = Pstar.new_states()
    Pstar.sequential_fine(u0, Us)
    Uf = P.new_states()
    P.sequential_fine(u0, Uf)
    npts = n * n
    lam = (Uf[N * npts:] - Us[N * npts:]).contiguous()  # dL/du(T)
    out = {}
    for name, kw in (("serial", None), ("parallel_exact", dict(k_max=0)),
                     ("parallel_parareal", dict(k_max=N, tol=1e-8 * lam.abs().max().item()))):
        g0 = torch.empty(npts, dtype=torch.float64, device=dev)
        gc = torch.empty((n + 2) ** 2, dtype=torch.float64, device=dev)
        times = []
        for rep in range(1 + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = None
            if kw is None:
                P.adjoint(u0, lam, g0, gc)
            else:
                k = P.adjoint_parallel(u0, lam, g0, gc, **kw)
            torch.cuda.synchronize()
            if rep:
                times.append(time.perf_counter() - t0)
        out[name] = (min(times), g0.clone(), gc.clone(), k)
        log(f"{name}: {1e3 * min(times):.1f} ms" + (f", backward corrections {k}" if k else ""))
    ref = out["serial"][2]
    agree = {k: (v[2] - ref).abs().max().item() / ref.abs().max().item() for k, v in out.items()}
    t_par = out["parallel_exact"][0]
    pts = npts * N * s
    result = {
        "metric": METRIC, "value": round(pts / t_par / 1e9, 3), "unit": "Gpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(1e3 * t_par, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{n}x{n}", "slices": N, "fine_steps": s,
                   "step": "gradient of a terminal misfit wrt u0 and theta (forward checkpoints, "
                           "boundary adjoints, per-slice recompute and reverse steps)"},
        "adjoint_ms": {k: round(1e3 * v[0], 3) for k, v in out.items()},
        "backward_parareal_corrections": out["parallel_parareal"][3],
        "theta_gradient_rel_diff_vs_serial": agree,
        "speedup_parallel_exact_vs_serial": round(out["serial"][0] / t_par, 3),
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["varcoef2d", "dd1d", "dd2d", "batch", "manufactured",
                                           "adjoint"],
                    default="varcoef2d",
                    help="varcoef2d: 2D variable coefficient 1023^2, N=64, s=64 (default); "
                         "dd1d: 1D domain decomposition 2^20 nodes, 8 components, N=32, s=128; "
                         "batch: 256 uneven 2D instances, batched parareal vs a loop of "
                         "single-instance launches; manufactured: the paper's test problem "
                         "(h = 1e-3, DT = 0.05, dt = 2.5e-3, T = 1, source term), errors "
                         "against the exact solution; dd2d: the same problem split into two "
                         "subdomains of q = 2 vertical strips with overlap 1/16 (the paper's 2D "
                         "domain-decomposition runs); adjoint: serial vs parallel-in-time "
                         "adjoint on 511^2, N=32, s=32")
    ap.add_argument("--fine", choices=["fie", "dr"], default="fie",
                    help="fine propagator (eq. FIE_method or eq. DR_method)")
    ap.add_argument("--instances", type=int, default=256)
    ap.add_argument("--copy-probe-mib", type=int, default=512,
                    help="size of a plain device-to-device copy timed in the same run (0: skip)")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--partitioned", type=int, choices=[0, 1, 2], default=1,
                    help="partitioned fine sweeps: 1 few slices (default), 2 wherever a line fits "
                         "one workgroup, 0 chunked sweeps only")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1023)
    ap.add_argument("--slices", type=int, default=64)
    ap.add_argument("--fine-steps", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-parareal", action="store_true",
                    help="skip the parareal-to-tolerance vs sequential comparison")
    ap.add_argument("--no-loop", action="store_true",
                    help="batch workload: skip the loop of single-instance handles")
    args = ap.parse_args()
    if args.gpus != 1:
        log(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
            "(slices would shard across GPUs with one state handed forward per coarse sweep; "
            "not built).")
        sys.exit(2)

    import torch
    import workloads as W
    import paper_2502_08370_amd as pr

    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "dd1d":
        w = W.config3()
    elif args.workload == "manufactured":
        w = W.manufactured2d(999, 20, 20)
    elif args.workload == "dd2d":
        w = W.dd2_manufactured(999, 20, 20, q=2, beta=1.0 / 16)
    else:
        w = W.config2(n=args.n, n_slices=args.slices, fine_steps=args.fine_steps)
    w.fine = args.fine
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = (cpu_baseline_dd2(w) if (w.split == "dd" and w.dim == 2)
               else cpu_baseline(w, args.cpu_seconds))
        log(f"  {cpu['sample']}: {cpu['value']:.4f} Gpts/s")

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    N, s, npts = w.n_slices, w.fine_steps, w.nx * w.ny
    inst = dict(dim=w.dim, nx=w.nx, ny=w.ny, T=w.T, n_slices=N, fine_steps=s, split=w.split,
                fine=w.fine)
    if w.theta is not None:
        inst["theta"] = w.theta
    else:
        inst["ax"], inst["ay"] = w.ax, w.ay
    if w.rho is not None:
        inst["rho"] = w.rho
    if w.forcing is not None:
        inst["forcing"] = w.forcing
    t_setup = time.perf_counter()
    prob = pr.Problem([inst])
    prob.set_option("partitioned", args.partitioned)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    log(f"problem set-up (factorisations) {t_setup:.3f} s")
    u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()
    U = prob.new_states()
    G = prob.new_slices()
    F = prob.new_slices()
    inc = torch.zeros(1, dtype=torch.float64, device=dev)
    U[:npts].copy_(u0)
    prob.coarse_sweep(None, G, U, inc)  # initial guess

    def step():
        prob.fine_propagate(U[:N * npts], F)
        prob.coarse_sweep(F, G, U, inc)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    prob.profile(2)
    # span mode: one event pair around each loop of fine sweeps and each coarse
    # sweep (per-launch events would add their own queue time to the step)
    prob.profile(3)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_host = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    prob.profile(0)
    ms_step = e0.elapsed_time(e1) / args.steps
    phases = prob.profile_read()
    log(f"step {ms_step:.3f} ms (host {1e3 * t_host / args.steps:.3f} ms); phases: "
        + ", ".join(f"{k} {v[0] / args.steps:.3f} ms/{v[1] // args.steps}" for k, v in phases.items()))

    fine_pts = npts * N * s
    value = fine_pts / (ms_step * 1e-3) / 1e9
    sweep_ms, sweep_n = phases["fine_sweep"]
    sweep_avg_ms = sweep_ms / sweep_n
    dd2 = w.split == "dd" and w.dim == 2
    if dd2:
        bytes_per_sweep = dd2_substep_bytes(w, N)
    elif w.split == "dd":
        # one colour substep reads and writes each node of that colour's components once
        bytes_per_sweep = 16.0 * float(np.mean(covered_nodes(w))) * N
    elif w.fine == "dr":
        # a Douglas-Rachford substep reads and writes the value and the term S = dt A_y U
        bytes_per_sweep = 32.0 * npts * N
    else:
        bytes_per_sweep = 16.0 * npts * N  # one substep: read + write one FP64 per point per slice
    achieved = bytes_per_sweep / (sweep_avg_ms * 1e-3) / 1e9
    traffic = None
    tb = None
    csrc = os.path.join(ROOT, "paper_2502_08370_amd", "csrc")
    if w.split != "dd" and (w.nx, w.n_slices, w.fine_steps) == (1023, 64, 64):
        tb = measured_traffic(os.path.join(csrc, "pr_kernels_dim.hip"),
                              os.path.join(ROOT, "profiles", "pmc_fine_sweep_varcoef2d_1023_N64_s64.json"))
    elif (w.split != "dd" and w.fine == "fie" and (w.nx, w.n_slices, w.fine_steps) == (999, 20, 20)
          and prob.get_option("partitioned_used") > 0):
        tb = measured_traffic(os.path.join(csrc, "pr_kernels_dim.hip"),
                              os.path.join(ROOT, "profiles", "pmc_fine_sweep_manufactured2d_999_N20_s20.json"))
    elif dd2 and (w.nx, w.n_slices, w.fine_steps) == (999, 20, 20):
        tb = measured_traffic(os.path.join(csrc, "pr_kernels_dd2.hip"),
                              os.path.join(ROOT, "profiles", "pmc_dd2_substep_dd2d_999_M2_q2_N20_s20.json"))
    elif w.split == "dd" and (w.nx, w.n_slices, w.fine_steps) == (1 << 20, 32, 128):
        tb = measured_traffic(os.path.join(csrc, "pr_kernels_dd.hip"),
                              os.path.join(ROOT, "profiles", "pmc_dd_substep_dd1d_1048576_M2_N32_s128.json"))
    if tb is not None:
        traffic = {"gbs": round(tb / (sweep_avg_ms * 1e-3) / 1e9, 1), "bytes_per_launch": tb,
                   "over_algorithmic": round(tb / bytes_per_sweep, 4)}
    fine_ms = (phases["fine_sweep"][0] + phases.get("fine_transpose", (0, 0))[0]) / args.steps
    coarse_ms = (phases.get("coarse_sweep", (0, 0))[0] + phases.get("coarse_x", (0, 0))[0]
                 + phases.get("coarse_y", (0, 0))[0]) / args.steps

    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpts/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{w.nx}x{w.ny}" if w.dim == 2 else f"{w.nx}",
                   "slices": N, "fine_steps": s, "coarse_steps": 1,
                   "split": ("domain decomposition, vertical strips" if dd2 else
                             "domain decomposition" if w.split == "dd" else "dimensional"),
                   "integrators": "FIE/" + w.fine.upper(),
                   "step": "one parareal iteration: F^s on all slices + serial coarse sweep "
                           "with correction and increment"},
        "roofline": {"bound": "hbm",
                     "kernel": ("dd2 substep (k_dd2_solve phases + k_dd2_tri0s + k_dd2_kup0)" if dd2 else
                                "dd substep (k_dd_local_run + k_dd_runscan)" if w.split == "dd"
                                else sweep_label(prob)),
                     "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic["gbs"] if traffic else None,
                     "traffic_detail": traffic, "bytes_per_launch": bytes_per_sweep,
                     "mean_launch_ms": round(sweep_avg_ms, 5), "launches": int(sweep_n)},
        "fine_propagator": {"gpts": round(fine_pts / (fine_ms * 1e-3) / 1e9, 3),
                            "ms": round(fine_ms, 4)},
        "coarse_sweep_ms": round(coarse_ms, 4),
        "setup_s": round(t_setup, 3),
        "cpu_baseline": cpu,
    }

    if args.copy_probe_mib > 0:
        # plain copy of known size: achievable bandwidth in this session, and the reference
        # for scaling hardware byte counters
        nbytes = args.copy_probe_mib << 20
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(5):
            b.copy_(a)
        c1.record()
        torch.cuda.synchronize()
        gbs = 2 * nbytes * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
        result["copy_probe"] = {"bytes_copied": nbytes, "read_plus_write_gbs": round(gbs, 1)}
        result["roofline"]["frac_of_copy_probe"] = round(achieved / gbs, 4)
        log(f"copy probe {args.copy_probe_mib} MiB: {gbs:.1f} GB/s read+write")
        del a, b

    if not args.no_parareal:
        # parareal to tolerance vs the sequential fine solve (the plain loop of fine steps)
        Ub = prob.new_states()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k, incv = prob.parareal_iterate(u0, Ub, k_max=N, tol=w.tol)
        torch.cuda.synchronize()
        t_par = time.perf_counter() - t0
        Us = prob.new_states()
        t0 = time.perf_counter()
        prob.sequential_fine(u0, Us)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        Ub3, Us3 = Ub.view(N + 1, -1), Us.view(N + 1, -1)
        err = ((Ub3 - Us3).abs().max() / Us3.abs().max()).item()
        result["parareal"] = {"iterations": k[0], "tol": w.tol, "last_increment": incv[0],
                              "wall_s": round(t_par, 4), "sequential_fine_wall_s": round(t_seq, 4),
                              "speedup_vs_sequential": round(t_seq / t_par, 3),
                              "rel_err_vs_sequential": err}
        log(f"parareal: {k[0]} iterations, {t_par:.3f} s; sequential fine {t_seq:.3f} s; "
            f"rel err vs sequential {err:.2e}")
        if "exact_space" in w.extra:
            # the paper's error measure: max over the coarse time levels of the discrete
            # 2-norm of the difference to the exact solution
            Sx = torch.as_tensor(w.extra["exact_space"], device=dev).reshape(-1)
            tn = torch.arange(N + 1, device=dev, dtype=torch.float64) * (w.T / N)
            ex = torch.sin(2 * torch.pi * tn)[:, None] * Sx[None, :]
            h = 1.0 / (w.nx + 1)
            e2 = lambda V: (((V - ex) ** 2).sum(dim=1).sqrt() * h).max().item()
            result["manufactured"] = {"error_parareal": e2(Ub3), "error_sequential_fine": e2(Us3),
                                      "h": h, "DT": w.T / N, "dt": w.T / N / s}
            log(f"error vs exact solution: parareal {e2(Ub3):.3e}, sequential fine {e2(Us3):.3e}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
