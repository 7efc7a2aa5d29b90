"""Throughput benchmark of the fused npFEM step on one MI355X.

Workload (default): 20 000 red blood cells (258 vertices) + 4 000 platelets (66 vertices) in
a seeded random interleave, 20 projective-dynamics iterations per step, external forces
N(0, 2 pN) with 5 % of the cells at 10x (seed 3). Inputs are resident in HBM before timing;
force arrays come from a pool of pre-generated steps that the steps cycle through.

Prints one JSON line: throughput in cell-PD-iterations/s over the timed steps, per-step
latency percentiles, the plain one-cell-at-a-time form on a subset for comparison, the
dominant kernel's roofline figures, the accuracy of the run against the FP64 oracle on
sampled cells, and the oracle's own CPU throughput on that sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-PD-iterations/s at ≤1e-4 diam error; p50/p99 step latency vs plain"
PEAK_FP32_VECTOR_TFLOPS = 157.3     # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
PEAK_FP16_MFMA_TFLOPS = 2500.0      # MI355X published dense fp16 matrix-core peak
# Algorithmic FLOP per cell per PD iteration (local projections + FP64 volume reductions +
# gather + banded-factor solve), and bytes per vertex per step (read x, v, F; write x, v).
FLOP_PER_ITER = {0: 3.2e5, 1: 6.9e4}
# the paper's viscoelastic parameters (parameter table): Rayleigh beta_D, position-based kappa
VISCO_BETA = 0.01
VISCO_KAPPA = 0.8
BYTES_PER_VERTEX_STEP = 60
FUSED_SRC = os.path.join(ROOT, "paper_1911_03062_amd", "csrc", "kernels_fused.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_step_large_24000_traffic.json")


# algorithmic HBM bytes of one contact-detection pass per vertex (FP32; see the packing leg)
DETECT_BYTES_PER_VERTEX = 36 + 8 + 32 + 16 + 4


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("kernels_fused.hip", "projections.h", "filters.h", "npfem_internal.h"):
        with open(os.path.join(ROOT, "paper_1911_03062_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """Per-launch HBM bytes from the committed counter summary, if it matches the source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


# All-cores oracle leg: forked workers (before anything touches the GPU) step disjoint parts
# of a cell sample with one BLAS thread each and return the sample's final states, which the
# accuracy block compares with a GPU run of the same steps. The oracle vectorises over the
# cells of a type; each worker steps its cells as one compact batch (the workload arrays are
# shared by the fork).
_ORACLE_JOB = {}


def host_cpu() -> dict:
    """The host's CPU model, core counts and BLAS/OpenMP thread settings."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    env = {k: os.environ[k] for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                      "MKL_NUM_THREADS", "MAX_JOBS") if k in os.environ}
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable,
            "thread_env": env}


def _oracle_worker(cells):
    import contextlib
    import oracle as O
    import npfem_inputs as I
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:                      # pragma: no cover
        limiter = contextlib.nullcontext()
    j = _ORACLE_JOB
    b, pool, K, steps = j["batch"], j["pool"], j["K"], j["steps"]
    cells = np.asarray(cells, dtype=np.int64)
    idx = np.concatenate([np.arange(b.offsets[c], b.offsets[c + 1]) for c in cells])
    types = b.types[cells]
    offsets = np.zeros(len(cells) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(b.offsets[cells + 1] - b.offsets[cells])
    forces = [np.ascontiguousarray(f[:, idx]) for f in pool]
    ot = {k: O.CellType(x_, t_, m_, I.DT) for k, (x_, t_, m_) in I.cell_type_inputs().items()}
    xo, vo = np.ascontiguousarray(b.x0[:, idx]), np.ascontiguousarray(b.v0[:, idx])
    with limiter:
        c0 = time.perf_counter()
        for s in range(steps):
            xo, vo = O.step_batch(ot, types, offsets, xo, vo, forces[s % len(forces)], K)
        wall = time.perf_counter() - c0
    return wall, cells, xo


def oracle_all_cores(w, K, steps, pool_n, n_random, max_procs=16):
    """The oracle over n_random seeded cells plus every strongly forced cell of workload w,
    `steps` steps from the initial state, on all usable host cores (at most max_procs, the
    CPU share of one GPU on the measurement hosts). Returns (baseline dict, cells, states)."""
    import multiprocessing as mp
    import npfem_inputs as I
    host = host_cpu()
    n_procs = max(1, min(max_procs, host["usable_cpus"] or 1))
    b = w.batch()
    _ORACLE_JOB.update(batch=b, pool=list(w.forces(b, n_steps=pool_n)), K=K, steps=steps)
    rng = np.random.default_rng(14)
    strong = I.strong_cells(b, w.seed, w.strong_fraction) if w.strong_fraction > 0 else []
    cells = np.unique(np.concatenate([rng.choice(b.n_cells, min(n_random, b.n_cells),
                                                 replace=False), strong])).astype(np.int64)
    # cost-balanced parts: red cells cost ~4.6 platelets per iteration
    cost = np.where(b.types[cells] == I.RBC, 4.6, 1.0)
    order = np.argsort(-cost, kind="stable")
    load = np.zeros(n_procs)
    parts = [[] for _ in range(n_procs)]
    for i in order:
        p = int(np.argmin(load))
        parts[p].append(int(cells[i]))
        load[p] += cost[i]
    parts = [sorted(pt) for pt in parts if pt]
    pool = mp.get_context("fork").Pool(len(parts))
    try:
        res = pool.map(_oracle_worker, parts)
    finally:
        pool.close()
        pool.join()
    _ORACLE_JOB.clear()
    wall = max(r[0] for r in res)
    states = {}
    for _, pc, xo in res:
        off = 0
        for c in pc:
            n = int(b.offsets[c + 1] - b.offsets[c])
            states[int(c)] = xo[:, off:off + n]
            off += n
    base = {
        "value": len(cells) * K * steps / wall, "unit": "cell-PD-iterations/s",
        "cores": len(parts), "kind": "oracle",
        "sample": f"{len(cells)} cells of {w.name} ({min(n_random, b.n_cells)} seeded random "
                  f"plus all {len(strong)} strongly forced), {steps} steps x {K} PD iterations "
                  f"from the initial state, NumPy FP64, {len(parts)} forked workers with 1 BLAS "
                  f"thread each, cells split by cost; slowest worker {wall:.1f} s",
        "host": host,
        "cap": f"workers = min({max_procs}, usable CPUs)",
    }
    return base, cells, states


LEGS = ("plain", "filter", "global", "visco", "contacts", "skalak", "packing", "serving")


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large_24000")
    ap.add_argument("--force-pool", type=int, default=4)
    ap.add_argument("--sample-cells", type=int, default=12,
                    help="cells of the one-core oracle leg (compared with the timed state)")
    ap.add_argument("--accuracy-cells", type=int, default=512,
                    help="seeded random cells of the all-cores oracle leg, which also takes "
                         "every strongly forced cell")
    ap.add_argument("--accuracy-steps", type=int, default=10,
                    help="steps of the all-cores oracle leg and of the GPU run it checks")
    ap.add_argument("--plain-cells", type=int, default=8)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (a known-size "
                         "kernel to scale HBM counters by)")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of each Poisson-arrival serving run (0 skips them)")
    ap.add_argument("--serve-budget-mb", type=int, default=8192,
                    help="HBM budget of the serving run's slot pool (x, v, F)")
    ap.add_argument("--serve-stress-mb", type=int, default=512,
                    help="HBM budget of a second, stressed serving run (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle leg (accuracy check and CPU baseline)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default fused layouts instead of timing them first")
    ap.add_argument("--cells-per-wave", default=None,
                    help="fused layouts as 'RBC,PLT' cells per wave (skips the autotuner)")
    ap.add_argument("--packing-steps", type=int, default=200,
                    help="timed steps of the packing leg (detection + step)")
    ap.add_argument("--eager", action="store_true",
                    help="time plain npfem_step calls instead of HIP-graph replays")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated legs to run besides the timed step: " + ",".join(LEGS))
    args = ap.parse_args()
    legs = set(x for x in args.legs.split(",") if x)
    unknown = legs - set(LEGS)
    if unknown:
        ap.error(f"unknown legs {sorted(unknown)}")

    def want(name):
        return name in legs
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the cells of a batch are independent: a multi-GPU run would give each GPU its "
              "own batch of cells, which this build does not do)", file=sys.stderr)
        sys.exit(2)

    import npfem_inputs as I
    cpu_all = None
    if not args.no_cpu_baseline:
        # before torch and the library are loaded: the workers are plain forks
        log("oracle on all host cores")
        w0 = I.WORKLOADS[args.workload]
        cpu_all, acc_cells, acc_states = oracle_all_cores(
            w0, w0.n_pd_iters, args.accuracy_steps,
            max(1, min(args.force_pool, args.warmup + args.steps)), args.accuracy_cells)
        log(f"oracle on all host cores: {cpu_all['sample']}")

    import torch
    from paper_1911_03062_amd import npfem as N

    torch.cuda.set_device(0)
    log(f"building workload {args.workload}")
    w = I.WORKLOADS[args.workload]
    b = w.batch()
    K = w.n_pd_iters
    n_steps_total = args.warmup + args.steps
    pool_n = max(1, min(args.force_pool, n_steps_total))
    pool_np = list(w.forces(b, n_steps=pool_n))

    types = {k: N.CellType(x, t, m, I.DT) for k, (x, t, m) in I.cell_type_inputs().items()}
    batch = N.Batch([types[int(t)] for t in b.types], precision=32, form="fused")
    x = torch.tensor(b.x0, dtype=torch.float32, device="cuda")
    v = torch.tensor(b.v0, dtype=torch.float32, device="cuda")
    pool = [torch.tensor(f, dtype=torch.float32, device="cuda") for f in pool_np]
    stream = torch.cuda.current_stream()
    present = {name: k for name, k in (("RBC", I.RBC), ("PLT", I.PLT)) if (b.types == k).any()}
    if args.cells_per_wave:
        for name, gw in zip(("RBC", "PLT"), args.cells_per_wave.split(",")):
            if name in present:
                batch.set_cells_per_wave(types[present[name]], int(gw))
    elif not args.no_autotune:
        log("autotuning the fused layouts (scratch state)")
        batch.autotune(K, reps=2)
    layouts = {name: batch.cells_per_wave(types[k]) for name, k in present.items()}
    log(f"cells per wave: {layouts}")
    # one single-step graph per force buffer, replayed in the same order as eager steps
    graphs = None if args.eager else [batch.graph(x, v, [f], I.DT, K) for f in pool]

    def step(s):
        if graphs is None:
            batch.step(x, v, pool[s % pool_n], I.DT, K)
        else:
            graphs[s % pool_n].launch(stream)

    log("inputs resident; warm-up")
    for s in range(args.warmup):
        step(s)
    batch.check()
    torch.cuda.synchronize()

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for s in range(args.steps):
        step(args.warmup + s)
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    batch.check()
    log(f"timed {args.steps} steps in {wall:.3f} s")
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])  # ms
    gpu_ms = float(lat.sum())
    elapsed_s = max(wall, gpu_ms * 1e-3)
    n_cells = b.n_cells
    value = n_cells * K * args.steps / elapsed_s

    # roofline of the fused kernel: one launch per step
    n_rbc = int(np.sum(b.types == I.RBC))
    n_plt = n_cells - n_rbc
    flop_launch = K * (n_rbc * FLOP_PER_ITER[I.RBC] + n_plt * FLOP_PER_ITER[I.PLT])
    avg_launch_s = float(np.mean(lat)) * 1e-3
    achieved_tflops = flop_launch / avg_launch_s / 1e12
    alg_bytes = BYTES_PER_VERTEX_STEP * b.v_total
    traffic = measured_traffic()

    # the other launch path on copies of the state (the state above must keep exactly the
    # warm-up + timed steps for the accuracy check)
    xc, vc = x.clone(), v.clone()
    other = None
    if graphs is None:
        other_graphs = [batch.graph(xc, vc, [f], I.DT, K) for f in pool]
        run_other = lambda s: other_graphs[s % pool_n].launch(stream)
    else:
        run_other = lambda s: batch.step(xc, vc, pool[s % pool_n], I.DT, K)
    run_other(0)
    torch.cuda.synchronize()
    oe0, oe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    oe0.record(stream)
    for s in range(5):
        run_other(s)
    oe1.record(stream)
    torch.cuda.synchronize()
    other = oe0.elapsed_time(oe1) / 5
    del xc, vc

    # the all-cores oracle leg's check: the same steps from the initial state on the same
    # launch path, in place (the timed state is kept on the host for the one-core leg)
    xg_timed = x.double().cpu().numpy()
    acc_all = None
    if cpu_all is not None:
        x.copy_(torch.tensor(b.x0, dtype=torch.float32))
        v.copy_(torch.tensor(b.v0, dtype=torch.float32))
        for s in range(args.accuracy_steps):
            step(s)
        torch.cuda.synchronize()
        batch.check()
        xa = x.double().cpu().numpy()
        errs, disp, strong_err = [], [], 0.0
        strong_set = set(int(c) for c in I.strong_cells(b, w.seed, w.strong_fraction)) \
            if w.strong_fraction > 0 else set()
        for c in acc_cells:
            sl = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
            xo_c = acc_states[int(c)]
            e = np.linalg.norm(xa[:, sl] - xo_c, axis=0).max() / I.DIAMETER[int(b.types[c])]
            errs.append(e)
            disp.append(np.linalg.norm(xo_c - b.x0[:, sl], axis=0).max())
            if int(c) in strong_set:
                strong_err = max(strong_err, e)
        errs = np.array(errs)
        acc_all = {"max_err_over_diam": float(errs.max()), "median_err_over_diam": float(np.median(errs)),
                   "max_err_strongly_forced": strong_err, "gate": 1e-4,
                   "passes": bool(errs.max() <= 1e-4), "sampled_cells": int(len(acc_cells)),
                   "strongly_forced_cells": int(len(strong_set & set(int(c) for c in acc_cells))),
                   "steps_compared": args.accuracy_steps,
                   "oracle_max_displacement_um": float(max(disp)),
                   "launch": "eager npfem_step" if graphs is None else "hipGraph replays"}
        log(f"accuracy over {len(acc_cells)} cells: max {errs.max():.3e}, median {np.median(errs):.3e}")

    if args.copy_calibration_mb > 0:
        nbytes = args.copy_calibration_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    plain_ms = None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-PD-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {n_rbc} RBC (258 vertices) + {n_plt} platelets (66 vertices), "
                        f"interleaved, {K} PD iterations/step, forces N(0, {w.sigma} pN), "
                        f"{int(w.strong_fraction * 100)}% of cells at 10x",
            "n_cells": n_cells, "n_vertices": b.v_total, "n_pd_iters": K,
            "form": "fused", "dt_us": I.DT, "force_pool": pool_n,
            "reductions": "fp64 (volume, area)",
            "cells_per_wave": layouts,
            "autotuned": not (args.no_autotune or args.cells_per_wave),
            "launch": "eager npfem_step" if graphs is None else
                      "hipGraph replays (one single-step graph per force buffer)",
        },
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(np.mean(lat))},
        ("eager_ms_per_step" if graphs is not None else "graph_ms_per_step"): other,
        "roofline": {
            "bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_VECTOR_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP32_VECTOR_TFLOPS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "hbm_achieved_GBs": alg_bytes / avg_launch_s / 1e9,
            "hbm_frac": alg_bytes / avg_launch_s / 1e9 / PEAK_HBM_GBS,
            "kernel": "k_fused_step", "flop_per_launch": flop_launch,
            "avg_launch_ms": avg_launch_s * 1e3,
        },
        "kernel_source_hash": kernel_source_hash(),
    }

    if want("plain"):
        # plain one-cell-at-a-time form on a subset, same state recipe
        rng = np.random.default_rng(11)
        pcells = np.sort(rng.choice(n_cells, size=min(args.plain_cells, n_cells), replace=False))
        idx = np.concatenate([np.arange(b.offsets[c], b.offsets[c + 1]) for c in pcells])
        pbatch = N.Batch([types[int(b.types[c])] for c in pcells], precision=32, form="plain")
        px = torch.tensor(np.ascontiguousarray(b.x0[:, idx]), dtype=torch.float32, device="cuda")
        pv = torch.tensor(np.ascontiguousarray(b.v0[:, idx]), dtype=torch.float32, device="cuda")
        pf = torch.tensor(np.ascontiguousarray(pool_np[0][:, idx]), dtype=torch.float32, device="cuda")
        pbatch.step(px, pv, pf, I.DT, K)
        torch.cuda.synchronize()
        pe0, pe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pe0.record(stream)
        p_steps = 3
        for _ in range(p_steps):
            pbatch.step(px, pv, pf, I.DT, K)
        pe1.record(stream)
        torch.cuda.synchronize()
        plain_ms = pe0.elapsed_time(pe1) / p_steps
        plain_value = len(pcells) * K / (plain_ms * 1e-3)
        out["plain_gpu"] = {"value": plain_value, "unit": "cell-PD-iterations/s", "cells": len(pcells),
                             "ms_per_step": plain_ms, "launches_per_cell_step": 2 * K + 2,
                             "speedup_fused_over_plain": value / plain_value}
        log(f"plain form: {plain_ms:.2f} ms per step of {len(pcells)} cells")

    if want("filter"):
        # boundary filter: one-ring median of the whole batch's external forces (one launch)
        fout = torch.empty_like(pool[0])
        batch.filter_forces(pool[0], fout)
        torch.cuda.synchronize()
        me0, me1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        mf_reps = 20
        # a spin kernel ahead of the timed launches keeps the stream busy while the host enqueues
        # them, so the events bracket back-to-back filter kernels, not the host's call overhead
        torch.cuda._sleep(20_000_000)
        me0.record(stream)
        for _ in range(mf_reps):
            batch.filter_forces(pool[0], fout)
        me1.record(stream)
        torch.cuda.synchronize()
        mf_s = me0.elapsed_time(me1) / mf_reps * 1e-3
        mf_bytes = 2 * 3 * 4 * b.v_total
        del fout
        out["median_filter"] = {
            "kernel": "k_median_filter", "bound": "hbm", "avg_launch_us": mf_s * 1e6,
            "algorithmic_bytes_per_launch": mf_bytes, "achieved_GBs": mf_bytes / mf_s / 1e9,
            "frac": mf_bytes / mf_s / 1e9 / PEAK_HBM_GBS,
            "note": "F_ext of all cells in, filtered F_ext out (FP32, 24 B per vertex); "
                    "not part of the timed step",
        }

    if want("global"):
        # the global step alone over every cell (3 right-hand sides each): the dense L^-1 product
        # on the matrix cores, the dense L^-1 on the vector ALU and the banded Cholesky
        # substitution, on seeded N(0, 1) right-hand sides; sampled cells checked against the
        # oracle's FP64 solve
        import oracle as O
        g = torch.Generator(device="cuda").manual_seed(21)
        grhs = torch.randn((3, b.v_total), generator=g, device="cuda", dtype=torch.float32)
        gout = torch.empty_like(grhs)
        gcells = np.random.default_rng(22).choice(n_cells, 32, replace=False)
        rhs_np = grhs.double().cpu().numpy()
        ot_g = {k: O.CellType(x_, t_, m_, I.DT) for k, (x_, t_, m_) in I.cell_type_inputs().items()}
        gref = {}
        for c in gcells:
            sl = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
            gref[int(c)] = np.transpose(O.solve(ot_g[int(b.types[c])], np.transpose(rhs_np[:, sl])[None])[0])
        nnz = {}
        for k_, ct_ in ot_g.items():
            nnz[k_] = int(np.count_nonzero(np.abs(np.linalg.cholesky(ct_.L)) > 0))
        dense_flop = sum(3 * 2 * ot_g[int(t)].n ** 2 for t in b.types)
        # matrix-core work the dense form issues: per block of up to 16 same-type cells (as many
        # as fit 64 KB of LDS), pairs of 16-row tiles of L^-1 (the odd last one twice) times
        # every 16-column tile of the block's right-hand sides over 32-row k chunks, three fp16
        # products (split operands) each
        mfma_flop = 0
        for k_, ct_ in ot_g.items():
            n_t = ct_.n
            npad = max(32, -(-n_t // 4) * 4)
            cs = 3 * npad + (3 - 3 * npad) % 16   # the cell-block stride (3 mod 16)
            bc = min(16, max(1, 65536 // (4 * cs)))
            rt, nch = -(-n_t // 16), -(-(npad // 4) // 8)
            cols = -(-3 * bc // 16)
            cells_t = int(np.count_nonzero(b.types == k_))
            blocks = -(-cells_t // bc)
            mfma_flop += blocks * 3 * 2 * (16 * 2 * (-(-rt // 2))) * (32 * nch) * (16 * cols)
        band_flop = sum(3 * 4 * nnz[int(t)] for t in b.types)
        gres = {}
        for solve in ("dense", "banded", "gemv"):
            batch.global_solve(grhs, gout, solve=solve)
            torch.cuda.synchronize()
            xg = gout.double().cpu().numpy()
            err = 0.0
            for c in gcells:
                sl = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
                err = max(err, float(np.max(np.linalg.norm(xg[:, sl] - gref[int(c)], axis=1)
                                            / np.linalg.norm(gref[int(c)], axis=1))))
            ge0, ge1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            g_reps = 20
            torch.cuda._sleep(20_000_000)
            ge0.record(stream)
            for _ in range(g_reps):
                batch.global_solve(grhs, gout, solve=solve)
            ge1.record(stream)
            torch.cuda.synchronize()
            us = ge0.elapsed_time(ge1) / g_reps * 1e3
            flop = band_flop if solve == "banded" else dense_flop
            gres[solve] = {"avg_launch_us": us, "algorithmic_flop": flop,
                           "achieved_TFLOPs": flop / (us * 1e-6) / 1e12,
                           "max_rel_err_vs_oracle": err}
        mfma_tflops = mfma_flop / (gres["dense"]["avg_launch_us"] * 1e-6) / 1e12
        gres["dense"].update({"kernel": "k_global_dense_wide", "bound": "mfma",
                              "mfma_dtype": "fp16 split operands (hi + lo, three products), FP32 accumulation",
                              "mfma_flop_issued": mfma_flop, "mfma_TFLOPs": mfma_tflops,
                              "peak": PEAK_FP16_MFMA_TFLOPS, "frac": mfma_tflops / PEAK_FP16_MFMA_TFLOPS,
                              "flop_note": "algorithmic: 2 n^2 per column (dense L^-1 times one "
                                           "right-hand side); issued: the padded tiles, 3 fp16 products"})
        gres["banded"].update({"kernel": "k_global_banded", "bound": "alu", "peak": PEAK_FP32_VECTOR_TFLOPS,
                               "frac": gres["banded"]["achieved_TFLOPs"] / PEAK_FP32_VECTOR_TFLOPS,
                               "flop_note": "4 nnz(C) per column (forward and back substitution)"})
        gres["gemv"].update({"kernel": "k_global_gemv", "bound": "alu", "peak": PEAK_FP32_VECTOR_TFLOPS,
                             "frac": gres["gemv"]["achieved_TFLOPs"] / PEAK_FP32_VECTOR_TFLOPS,
                             "flop_note": "2 n^2 per column (dense L^-1 times one right-hand side, FP32 FMAs)"})
        out["global_step"] = {
            "config": f"every cell of {w.name}: {3 * n_rbc} RBC columns against the 258 x 258 "
                      f"inverse, {3 * n_plt} platelet columns against the 66 x 66 one; FP32, "
                      "inputs resident; error per column relative to the oracle's FP64 "
                      "prefactored solve, 32 sampled cells",
            "hbm_bytes_per_launch": 24 * b.v_total,
            **gres,
            "dense_over_banded_speed": gres["banded"]["avg_launch_us"] / gres["dense"]["avg_launch_us"],
            "autotune_choice": batch.global_solve_choice(),
        }
        log(f"global step: dense {gres['dense']['avg_launch_us']:.1f} us, banded "
            f"{gres['banded']['avg_launch_us']:.1f} us, gemv {gres['gemv']['avg_launch_us']:.1f} us")
        del grhs, gout

    if want("visco"):
        # the paper's viscoelastic configuration on the same batch and forces: Rayleigh beta_D and
        # position-based damping, fused form, autotuned, single-step graph replays
        vtypes = {k: N.CellType(x_, t_, m_.with_rayleigh(0.0, VISCO_BETA).with_kappa(VISCO_KAPPA), I.DT)
                  for k, (x_, t_, m_) in I.cell_type_inputs().items()}
        vbatch = N.Batch([vtypes[int(t)] for t in b.types], precision=32, form="fused")
        if not args.no_autotune:
            vbatch.autotune(K, reps=2)
        vlayouts = {name: vbatch.cells_per_wave(vtypes[k]) for name, k in present.items()}
        vx = torch.tensor(b.x0, dtype=torch.float32, device="cuda")
        vv = torch.tensor(b.v0, dtype=torch.float32, device="cuda")
        vgraphs = [vbatch.graph(vx, vv, [f], I.DT, K) for f in pool]
        for s_ in range(2):
            vgraphs[s_ % pool_n].launch(stream)
        torch.cuda.synchronize()
        ve0, ve1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        v_steps = 10
        ve0.record(stream)
        for s_ in range(v_steps):
            vgraphs[s_ % pool_n].launch(stream)
        ve1.record(stream)
        torch.cuda.synchronize()
        vbatch.check()
        visco_ms = ve0.elapsed_time(ve1) / v_steps
        del vgraphs, vbatch, vx, vv
        out["viscoelastic"] = {
            "config": f"Rayleigh beta_D = {VISCO_BETA} us (alpha_D = 0) and position-based damping "
                      f"kappa = {VISCO_KAPPA} on every cell; same batch, forces and K",
            "ms_per_step": visco_ms, "value": n_cells * K / (visco_ms * 1e-3),
            "unit": "cell-PD-iterations/s", "cells_per_wave": vlayouts,
            "cost_vs_undamped": visco_ms / (elapsed_s * 1e3 / args.steps),
        }

    if want("contacts"):
        # collision energies on the same batch: 5 % of the vertices in contact (projection points
        # within 0.1 um, w = 400 pN/um, their forces zeroed), fused form, eager steps
        crng = np.random.default_rng(13)
        cw_np = np.where(crng.random(b.v_total) < 0.05, 400.0, 0.0)
        cw = torch.tensor(cw_np, dtype=torch.float32, device="cuda")
        cpt = (x + 0.1 * torch.randn(x.shape, generator=torch.Generator(device="cuda").manual_seed(13),
                                     device="cuda")).contiguous()
        cf = torch.where(cw > 0, torch.zeros_like(pool[0]), pool[0]).contiguous()
        xc2, vc2 = x.clone(), v.clone()
        batch.step(xc2, vc2, cf, I.DT, K, contacts=(cpt, cw))
        torch.cuda.synchronize()
        ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c_steps = 5
        ce0.record(stream)
        for _ in range(c_steps):
            batch.step(xc2, vc2, cf, I.DT, K, contacts=(cpt, cw))
        ce1.record(stream)
        torch.cuda.synchronize()
        batch.check()
        contacts_ms = ce0.elapsed_time(ce1) / c_steps
        del xc2, vc2, cpt, cw, cf
        out["contacts"] = {
            "config": "5 % of the vertices in contact (w = 400 pN/um, projection points within "
                      "0.1 um, forces zeroed there); same batch and K, eager steps",
            "ms_per_step": contacts_ms, "value": n_cells * K / (contacts_ms * 1e-3),
            "unit": "cell-PD-iterations/s",
        }

    if want("skalak") and plain_ms is not None:
        # Skalak membrane with line search (plain form) on the plain comparator's cells
        stypes = {k: N.CellType(x_, t_, m_.with_membrane("skalak"), I.DT)
                  for k, (x_, t_, m_) in I.cell_type_inputs().items()}
        sbatch = N.Batch([stypes[int(b.types[c])] for c in pcells], precision=32, form="plain")
        sx, sv = px.clone(), pv.clone()
        sbatch.step(sx, sv, pf, I.DT, K)
        torch.cuda.synchronize()
        se0, se1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        se0.record(stream)
        for _ in range(p_steps):
            sbatch.step(sx, sv, pf, I.DT, K)
        se1.record(stream)
        torch.cuda.synchronize()
        sbatch.check()
        skalak_ms = se0.elapsed_time(se1) / p_steps
        del sbatch, sx, sv
        out["skalak_plain"] = {
            "config": f"Skalak membrane with line search, plain form, the same {len(pcells)} cells",
            "ms_per_step": skalak_ms, "value": len(pcells) * K / (skalak_ms * 1e-3),
            "unit": "cell-PD-iterations/s", "launches_per_cell_step": 3 * K + 2,
            "cost_vs_plain_pd": skalak_ms / plain_ms,
        }

    if want("skalak"):
        # Skalak membrane with its line search in the fused form, every cell of the workload:
        # the same batch, forces and K, autotuned layouts, single-step graph replays; the
        # timing covers whatever line-search trials the cells needed
        stypes_f = {k: N.CellType(x_, t_, m_.with_membrane("skalak"), I.DT)
                    for k, (x_, t_, m_) in I.cell_type_inputs().items()}
        fbatch = N.Batch([stypes_f[int(t)] for t in b.types], precision=32, form="fused")
        if not args.no_autotune:
            fbatch.autotune(K, reps=2)
        flayouts = {name: fbatch.cells_per_wave(stypes_f[k]) for name, k in present.items()}
        fx = torch.tensor(b.x0, dtype=torch.float32, device="cuda")
        fv = torch.tensor(b.v0, dtype=torch.float32, device="cuda")
        fgraphs = [fbatch.graph(fx, fv, [f], I.DT, K) for f in pool]
        for s_ in range(2):
            fgraphs[s_ % pool_n].launch(stream)
        torch.cuda.synchronize()
        fe0, fe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f_steps = 5
        fe0.record(stream)
        for s_ in range(f_steps):
            fgraphs[s_ % pool_n].launch(stream)
        fe1.record(stream)
        torch.cuda.synchronize()
        fbatch.check()
        skalak_fused_ms = fe0.elapsed_time(fe1) / f_steps
        del fgraphs, fbatch, fx, fv
        out["skalak_fused"] = {
            "config": f"Skalak membrane with line search on every cell of {w.name}, fused form, "
                      "same forces and K, single-step graph replays",
            "ms_per_step": skalak_fused_ms, "value": n_cells * K / (skalak_fused_ms * 1e-3),
            "unit": "cell-PD-iterations/s", "cells_per_wave": flayouts,
            "cost_vs_pd_fused": skalak_fused_ms / (elapsed_s * 1e3 / args.steps),
        }
        log(f"fused Skalak: {skalak_fused_ms:.2f} ms per step")

    if want("packing"):
        # cell packing: the workload's cells placed at random at hematocrit 0.4, interpenetrating;
        # each step finds the particle-in-kernel contacts of the current positions and then steps
        # with their collision energies and no external force (eager, the main run's layouts)
        log("packing run")
        PK = I.PACKING
        pk = I.packing_batch(b.types, seed=w.seed)
        kbatch = N.Batch([types[int(t)] for t in pk.types], precision=32, form="fused")
        for name, k in present.items():
            kbatch.set_cells_per_wave(types[k], layouts[name])
        kx = torch.tensor(pk.x0, dtype=torch.float32, device="cuda")
        kv = torch.zeros_like(kx)
        kf = torch.zeros_like(kx)
        kp = torch.empty_like(kx)
        kw = torch.empty((pk.v_total,), dtype=torch.float32, device="cuda")
        Kp = PK["n_pd_iters"]

        def pack_step():
            kbatch.detect_contacts(kx, PK["radius"], PK["separation"], PK["weight"], kp, kw, stream)
            kbatch.step(kx, kv, kf, I.DT, Kp, contacts=(kp, kw), stream=stream)

        kbatch.detect_contacts(kx, PK["radius"], PK["separation"], PK["weight"], kp, kw, stream)
        torch.cuda.synchronize()
        pack_frac0 = float((kw > 0).float().mean())
        de0, de1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        d_reps = 10
        de0.record(stream)
        for _ in range(d_reps):
            kbatch.detect_contacts(kx, PK["radius"], PK["separation"], PK["weight"], kp, kw, stream)
        de1.record(stream)
        pack_step()
        torch.cuda.synchronize()
        detect_ms = de0.elapsed_time(de1) / d_reps
        pk_steps = max(1, args.packing_steps)
        pe0, pe1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pe0.record(stream)
        for _ in range(pk_steps):
            pack_step()
        pe1.record(stream)
        torch.cuda.synchronize()
        kbatch.check()
        packing_ms = pe0.elapsed_time(pe1) / pk_steps
        pack_frac1 = float((kw > 0).float().mean())
        del kbatch, kx, kv, kf, kp, kw
        out["packing"] = {
            "config": f"the workload's cells at random rigid motions at hematocrit {PK['hematocrit']} "
                      f"(interpenetrating), no external force, K = {Kp}; per step: contact "
                      f"detection (kernel radius {PK['radius']} um, separation {PK['separation']} "
                      f"um, w = {PK['weight']} pN/um) then the step with the collision energies; "
                      f"{pk_steps + 1} steps, eager",
            "ms_per_step": packing_ms, "detect_ms": detect_ms,
            "detect_roofline": {
                "bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS,
                "algorithmic_bytes_per_pass": DETECT_BYTES_PER_VERTEX * pk.v_total,
                "achieved": DETECT_BYTES_PER_VERTEX * pk.v_total / (detect_ms * 1e-3) / 1e9,
                "frac": DETECT_BYTES_PER_VERTEX * pk.v_total / (detect_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                "note": "one detection pass (fill, count, scan, scatter, query): positions read "
                        "three times (36 B), bucket written and read (8 B), record written and "
                        "read (32 B), projection point and weight written (16 B), the vertex's "
                        "cell read (4 B), per vertex; candidate gathers are not algorithmic",
            },
            "value": n_cells * Kp / (packing_ms * 1e-3), "unit": "cell-PD-iterations/s",
            "contact_fraction_first_step": pack_frac0,
            "contact_fraction_last_step": pack_frac1,
        }

    if args.serve_seconds > 0 and want("serving"):
        from paper_1911_03062_amd import serving as S
        rest = {k: xx for k, (xx, tt, mm) in I.cell_type_inputs().items()}
        serving = {}
        for name, mb in (("serving", args.serve_budget_mb), ("serving_stress", args.serve_stress_mb)):
            if mb <= 0:
                continue
            log(f"{name}: {args.serve_seconds:g} s of arrivals, HBM budget {mb} MiB")
            reqs, sessions = S.poisson_workload(args.serve_seconds, rate=200.0, seed=5)
            spool = S.SlotPool(types, rest, hbm_budget_bytes=mb << 20)
            srv = S.StepServer(spool, n_pd_iters=10, sigma=1.0)
            st = srv.run(reqs, sessions)
            cells = st["cells_stepped"]
            serving[name] = {
                "arrivals": f"Poisson 200/s for {args.serve_seconds:g} s, 50-10000 cells "
                            "log-uniform, 80/20 RBC/PLT, K=10, sessions of up to 10 requests "
                            "(continue probability 0.8)",
                "requests": len(reqs), "sessions": len(sessions), "ticks": len(st["ticks"]),
                "latency": S.latency_summary(reqs),
                "throughput_cell_PD_iter_per_s": cells * 10 / st["wall_s"],
                "gpu_busy_frac": st["busy_ms"] * 1e-3 / st["wall_s"],
                "hbm_budget_bytes": mb << 20, "slot_capacity_cells": spool.cap,
                "admission_waits": st["admission_waits"],
                "moved_to_host": st["evictions"], "moved_back": st["restores"],
                "peak_cells_resident": st["peak_cells_resident"],
                "mean_cells_per_tick": float(np.mean([tk.n_cells for tk in st["ticks"]])),
            }
            del spool, srv
            torch.cuda.empty_cache()
        out.update(serving)

    if not args.no_cpu_baseline:
        import oracle as O
        import contextlib
        try:
            from threadpoolctl import threadpool_limits
            limiter = threadpool_limits(limits=1)
        except Exception:                      # pragma: no cover
            limiter = contextlib.nullcontext()
        ot = {k: O.CellType(x_, t_, m_, I.DT) for k, (x_, t_, m_) in I.cell_type_inputs().items()}
        strong = I.strong_cells(b, w.seed, w.strong_fraction)
        srng = np.random.default_rng(12)
        sample = np.unique(np.concatenate([srng.choice(n_cells, args.sample_cells - 2, replace=False),
                                           strong[:2]])).astype(np.int64)
        xo, vo = b.x0.copy(), b.v0.copy()
        with limiter:
            c0 = time.perf_counter()
            for s in range(n_steps_total):
                xo, vo = O.step_batch(ot, b.types, b.offsets, xo, vo, pool_np[s % pool_n], K,
                                      cells=sample)
                if s % 5 == 4:
                    log(f"oracle step {s + 1}/{n_steps_total}")
            cpu_s = time.perf_counter() - c0
        xg = xg_timed
        errs = []
        for c in sample:
            sl = slice(int(b.offsets[c]), int(b.offsets[c + 1]))
            errs.append(np.linalg.norm(xg[:, sl] - xo[:, sl], axis=0).max() / I.DIAMETER[int(b.types[c])])
        disp = max(np.linalg.norm(xo[:, int(b.offsets[c]):int(b.offsets[c + 1])]
                                  - b.x0[:, int(b.offsets[c]):int(b.offsets[c + 1])], axis=0).max()
                   for c in sample)
        acc_timed = {"max_err_over_diam": float(max(errs)), "gate": 1e-4,
                     "passes": bool(max(errs) <= 1e-4), "sampled_cells": int(len(sample)),
                     "steps_compared": n_steps_total, "oracle_max_displacement_um": float(disp),
                     "note": "the timed run's own state after warm-up + timed steps"}
        out["accuracy"] = dict(acc_all) if acc_all is not None else {}
        out["accuracy"]["timed_state"] = acc_timed
        out["accuracy"]["passes"] = bool(acc_timed["passes"] and
                                         (acc_all is None or acc_all["passes"]))
        out["cpu_baseline"] = {
            "value": len(sample) * K * n_steps_total / cpu_s, "unit": "cell-PD-iterations/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{len(sample)} sampled cells of {w.name} (incl. 2 strongly forced) for "
                      f"{n_steps_total} steps x {K} PD iterations, NumPy FP64, 1 BLAS thread, "
                      f"{cpu_s:.1f} s",
            "host": host_cpu(),
        }
        if cpu_all is not None:
            out["cpu_baseline_all_cores"] = cpu_all
        if not out["accuracy"]["passes"]:
            out["value_invalid_reason"] = "accuracy gate failed"
    try:
        import psutil
        kids = psutil.Process().children(recursive=True)
        if kids:
            log(f"child processes still running: {[(k.pid, k.name()) for k in kids]}")
    except Exception:                      # pragma: no cover
        pass
    print(json.dumps(out))


if __name__ == "__main__":
    main()
