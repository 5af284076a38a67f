#!/usr/bin/env python3
"""Benchmark of the cluster-pair non-bonded path on one MI355X.

Workload: 32 000 rigid SPC/E waters (96 000 atoms) in a 9.86 nm periodic box,
8x8 clusters, rc = 1.0 nm, rlist = 1.1 nm, Ewald beta = 3.12 /nm, forces and
LJ + Coulomb energies every step, pair list rebuilt every 10 steps.  Inputs
are synthetic (seeded random sequential addition of waters, Maxwell-Boltzmann
velocities at 300 K, ballistic positions x_k = x_0 + v k dt with dt = 2 fs),
resident in HBM before timing starts.

One step = one list lifetime: nb_grid_sort + nb_pairlist_build + 10 x
nb_forces (energies on).  value = pair interactions computed per second over
whole steps (listed cluster pairs x M x N per force call, the paper's
pairs-per-cycle convention); effective (r < rc) pairs/s are reported beside.

Roofline of the force kernel (bound: FP32 VALU ALU work, no MFMA):
algorithmic flops = 63 per interacting pair (full LJ + Ewald evaluation; FP32
VALU count of the built 8x8 force+energy kernel, FMA = 2) + 8 per listed pair
beyond rc (distance and cut-off test), divided by the force kernel's average
duration from HIP events on the library stream; peak = 157.3 TFLOP/s
(MI355X FP32 vector, 256 CUs x 2.4 GHz, counting packed FP32; code compiled
without packed FP32 reaches at most half of it).  roofline.traffic = measured HBM
bytes per force-kernel launch (scaled FETCH_SIZE + WRITE_SIZE counters, see
FORCE_TRAFFIC), null once the kernel sources differ from the profiled ones.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 63          # FP32 flops of one in-range pair evaluation (8x8 force+energy kernel)
FLOPS_PER_DISTANCE = 8       # FP32 flops of the distance and cut-off test of a listed pair
PEAK_FP32 = 157.3e12
# HBM traffic of one force-kernel launch on this workload: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# (KiB per dispatch), each scaled by what the same counter reads for a 256 MiB device-to-device copy
# (FETCH_SIZE x2.0, WRITE_SIZE x1.0).  Valid only for the kernel sources the counters were taken on.
FORCE_TRAFFIC = {"sources_sha1": "b2d8739c097e1351acc57e7d893ff20860a228f8", "fetch_kib": 16351.0,
                 "write_kib": 105339.7, "fetch_scale": 2.0, "write_scale": 1.0}
FORCE_SOURCES = ("paper_1306_1737_amd/csrc/forces.hip", "paper_1306_1737_amd/csrc/devptr.h",
                 "paper_1306_1737_amd/csrc/ewald_fit.h")
METRIC = "atom-pair interactions/s (FP32, ≤1e-5 rel force err) + % FP32 VALU peak"


def force_traffic_bytes():
    """Measured bytes per force-kernel launch, or None once the kernel sources changed since."""
    import hashlib
    h = hashlib.sha1()
    try:
        for f in FORCE_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    if h.hexdigest() != FORCE_TRAFFIC["sources_sha1"]:
        return None
    t = FORCE_TRAFFIC
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def cpu_baseline(box, w):
    """The FP64 oracle on the host cores, timed on the whole production box: the cell-list (binned) force and
    energy evaluation, and beside it the brute-force O(N^2) double loop (forces on every atom against all
    partners).  Rates count unique pairs within rc (half of N * 4/3 pi rc^3 rho), as the GPU's effective rate."""
    import numpy as np
    import oracle
    import synth
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ["OMP_NUM_THREADS"] = str(nthreads)
    rho = box.n / box.box.prod()
    pairs = 0.5 * box.n * 4.0 / 3.0 * np.pi * w.rc ** 3 * rho
    runs, t0 = 0, time.perf_counter()
    while runs < 3 or time.perf_counter() - t0 < 5.0:   # repeated for a stable rate (a few seconds in all)
        oracle.forces(box.xyz, box.q, box.type, box.box, box.excl_off, box.excl_idx, synth.lj_table_spce(), w.rc,
                      w.beta, synth.COULOMB_F, mode="binned")
        runs += 1
    dt_binned = (time.perf_counter() - t0) / runs
    sub = np.arange(box.n, dtype=np.int32)
    t0 = time.perf_counter()
    oracle.forces_subset(box.xyz, box.q, box.type, box.box, box.excl_off, box.excl_idx, synth.lj_table_spce(),
                         w.rc, w.beta, synth.COULOMB_F, sub)
    dt_brute = time.perf_counter() - t0
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": pairs / dt_binned, "unit": "pair interactions/s (unique pairs r < rc, FP64)", "cores": nthreads,
            "kind": "oracle",
            "sample": "whole %d-atom box, cell-list (binned) FP64 forces + energies, %.2f s per evaluation (mean of "
                      "%d); CPU %s" % (box.n, dt_binned, runs, cpu),
            "brute": {"value": pairs / dt_brute, "seconds": dt_brute,
                      "sample": "forces on all %d atoms, each by brute force over all partners" % box.n}}


def list_build_bytes(n_atoms, n_slots, n_ci, n_cj, entries):
    """Algorithmic bytes of one grid sort + pair-list build: the sort reads positions/charges (16 B) and the type
    (4 B) of every atom and writes per slot the sorted position (16 B), type, original index and image (4 B
    each), per atom its slot (4 B), and per cluster its bounding box (32 B, i- and j-clusters); the search reads
    the sorted positions and the boxes once and writes per entry 16 B plus its j-force row index (4 B)."""
    sort = 20 * n_atoms + 28 * n_slots + 4 * n_atoms + 32 * (n_ci + (n_cj if n_cj != n_ci else 0))
    search = 16 * n_slots + 32 * n_ci + 20 * entries
    return sort + search


def _gen_box(args):
    import synth
    nw, seed = args
    return synth.water_box(int(nw), synth.box_edge_for(int(nw)), seed=int(seed))


def bench_batched(args):
    """256 uneven water boxes (1 500-24 000 atoms, log-uniform, seeded), rc 1.0 / rlist 1.1 nm: one step =
    grid sort + list rebuild of every replica + 10 force steps, either as one replayed graph of the batched
    launches (one launch per stage for all replicas), or as per-replica nb_grid_sort / nb_pairlist_build /
    nb_forces calls."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import torch
    import synth
    import paper_1306_1737_amd as mxn
    from paper_1306_1737_amd import autotune
    sizes = synth.batched_sizes(256)
    print("[bench] generating %d replicas (%d atoms)" % (len(sizes), 3 * int(sizes.sum())), file=sys.stderr,
          flush=True)
    # the generator runs in C through ctypes, which releases the GIL: threads suffice
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as pool:
        boxes = list(pool.map(_gen_box, [(nw, 5000 + k) for k, nw in enumerate(sizes)]))
    dev = torch.device("cuda:0")
    rc, rlist, beta = 1.0, 1.1, 3.12
    ctx = mxn.nb_create(0)
    print("[bench] autotuning", file=sys.stderr, flush=True)
    tune = autotune.tune_batch(ctx, boxes, rc, rlist, beta, reps=3, cache=None)
    shape = tuple(tune["shape"]) if args.shape == "auto" else tuple(int(v) for v in args.shape.split("x"))
    group = tune["group"]
    reps = autotune.build_replicas(ctx, boxes, shape, rlist)
    lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
    params = mxn.make_params(rc, beta, synth.COULOMB_F, lj)
    n = len(reps)
    energy = torch.zeros(2 * n, dtype=torch.float64, device=dev)
    batch = mxn.nb_batch_create(ctx, [r["grid"] for r in reps], [r["lst"] for r in reps], [r["xyzq"] for r in reps],
                                [r["f"] for r in reps])
    mxn.nb_batch_set_group(batch, group)
    mxn.nb_batch_bind_topology(batch, [r["type"] for r in reps], [r["eo"] for r in reps], [r["ei"] for r in reps])
    mxn.nb_batch_capture_cycle(ctx, batch, 10, params, mxn.NB_ENERGY, energy)
    e1 = [torch.zeros(2, dtype=torch.float64, device=dev) for _ in reps]

    def step_graph():
        mxn.nb_batch_replay(ctx, batch)

    def step_loop():
        for r in reps:
            r["grid"] = mxn.nb_grid_sort(ctx, r["box"].box, r["xyzq"], r["type"], shape, r["grid"])
            r["lst"] = mxn.nb_pairlist_build(ctx, r["grid"], rlist, -1.0, r["eo"], r["ei"], mxn.NB_LIST_ASYNC, r["lst"])
        for _ in range(10):
            for k, r in enumerate(reps):
                mxn.nb_forces(ctx, r["grid"], r["lst"], r["xyzq"], params, mxn.NB_ENERGY, r["f"], e1[k])

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        mxn.nb_sync(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        mxn.nb_sync(ctx)
        return (time.perf_counter() - t0) * 1e3 / args.steps

    ms_graph = timed(step_graph)
    ms_loop = timed(step_loop)
    listed = sum(mxn.nb_list_info(r["lst"])[0] for r in reps) * shape[0] * shape[1]
    result = {"metric": "atom-pair interactions/s, batched replicas", "value": listed * 10 / (ms_graph * 1e-3),
              "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "ms_per_step": ms_graph, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "f32", "data": "synthetic",
              "config": {"workload": "water-256-replicas", "replicas": n, "atoms": int(sum(b.n for b in boxes)),
                         "shape": "%dx%d" % shape, "items_per_group": group, "rc": rc, "rlist": rlist,
                         "force_steps_per_step": 10},
              "per_replica_launches_ms_per_step": ms_loop, "speedup_vs_per_replica": ms_loop / ms_graph,
              "autotune": tune["table"]}
    mxn.nb_batch_free(batch)
    autotune.free_replicas(reps)
    mxn.nb_destroy(ctx)
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--shape", default="8x8")
    ap.add_argument("--variant", default="direct", choices=["direct", "super"])
    ap.add_argument("--list-order", default="canonical", choices=["canonical", "distance"])
    ap.add_argument("--coulomb", default="ewald", choices=["ewald", "rf", "table"],
                    help="Coulomb correction: Ewald (analytic), reaction field (eps_rf 78), Ewald from a table")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="production", choices=["production", "batched", "twostage", "rdf"])
    ap.add_argument("--rdf-bins", type=int, default=500, help="rdf: histogram bins up to rc")
    ap.add_argument("--outer-rlist", type=float, default=0.0, metavar="NM",
                    help="twostage: radius of the box-only outer list (default: the workload's rlist)")
    ap.add_argument("--outer-nstlist", type=int, default=0, metavar="STEPS",
                    help="twostage: lifetime of the outer list (default: the workload's nstlist)")
    ap.add_argument("--prune-every", type=int, default=2, metavar="STEPS", help="twostage: rolling prune interval")
    ap.add_argument("--r-inner", type=float, default=1.05, metavar="NM", help="twostage: rolling prune radius")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (calibrates memory-traffic counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.empty(args.copy_probe * (1 << 18), dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe, "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py: measures one GPU only; multi-GPU runs are not part of it "
              "(the path would shard by replica or by spatial domain, see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        if args.shape == "8x8":
            args.shape = "auto"
        return bench_batched(args)
    if args.workload == "twostage":
        return bench_twostage(args)
    if args.workload == "rdf":
        return bench_rdf(args)

    import numpy as np
    import torch
    import synth
    import paper_1306_1737_amd as mxn

    w = synth.PRODUCTION
    m, n = (int(v) for v in args.shape.split("x"))
    print("[bench] generating %d waters" % w.n_mol, file=sys.stderr, flush=True)
    box = synth.water_box(w.n_mol, w.L, seed=1306)
    vel = synth.velocities(box.mass, w.T, seed=1306)
    xs = synth.free_flight(box.xyz, vel, w.dt, w.nstlist)
    dev = torch.device("cuda:0")
    xq = [torch.from_numpy(box.xyzq(x)).to(dev) for x in xs]
    typ = torch.from_numpy(box.type).to(dev)
    eo = torch.from_numpy(box.excl_off).to(dev)
    ei = torch.from_numpy(box.excl_idx).to(dev)
    lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
    f = torch.zeros((box.n, 3), dtype=torch.float32, device=dev)
    e = torch.zeros(2, dtype=torch.float64, device=dev)
    ctx = mxn.nb_create(0)
    mxn.nb_set_force_variant(ctx, {"direct": mxn.NB_FORCE_DIRECT, "super": mxn.NB_FORCE_SUPER}[args.variant])
    coulomb = {"ewald": mxn.NB_COULOMB_EWALD, "rf": mxn.NB_COULOMB_RF, "table": mxn.NB_COULOMB_EWALD_TABLE}[args.coulomb]
    params = mxn.make_params(w.rc, w.beta, synth.COULOMB_F, lj, True, coulomb, 78.0)
    state = {"grid": None, "lst": None}

    order_flag = mxn.NB_LIST_BY_DISTANCE if args.list_order == "distance" else 0

    def step(list_flags, sample=-1):
        """One list lifetime; force call `sample` (if any) has HIP events around its force kernel."""
        list_flags |= order_flag
        state["grid"] = mxn.nb_grid_sort(ctx, box.box, xq[0], typ, (m, n), state["grid"])
        state["lst"] = mxn.nb_pairlist_build(ctx, state["grid"], w.rlist, -1.0, eo, ei, list_flags, state["lst"])
        for k in range(w.nstlist):
            if k == sample:
                mxn.nb_timing_enable(ctx, True, timers=[mxn.NB_TIMER_FORCE_KERNEL])
            mxn.nb_forces(ctx, state["grid"], state["lst"], xq[k], params, mxn.NB_ENERGY, f, e)
            if k == sample:
                mxn.nb_timing_enable(ctx, False)

    print("[bench] warmup", file=sys.stderr, flush=True)
    step(0)                                # sizes the list storage (one synchronisation)
    mxn.nb_sync(ctx)
    for _ in range(max(0, args.warmup - 1)):
        step(mxn.NB_LIST_ASYNC)
    mxn.nb_sync(ctx)
    mxn.nb_timing_read(ctx)
    # Timed region.  Each recorded HIP event costs a few microseconds of stream time, so the force
    # kernel is timed on one force call per step (the k-th of step k, cycling through the list lifetime).
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        step(mxn.NB_LIST_ASYNC, sample=s_ % w.nstlist)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mxn.nb_sync(ctx)                       # raises on list overflow or non-finite input
    tim = mxn.nb_timing_read(ctx)
    print("[bench] timed %d steps" % args.steps, file=sys.stderr, flush=True)
    # per-stage times from a few further steps with every timer on (not part of the timed region)
    mxn.nb_timing_enable(ctx, True)
    for _ in range(3):
        step(mxn.NB_LIST_ASYNC)
    stage = mxn.nb_timing_read(ctx)
    mxn.nb_timing_enable(ctx, False)
    # the force call with no timer in the stream: blocks of 30 calls on the current list, host clock around
    # each block (median of three)
    call_blocks = []
    for _ in range(3):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _r in range(3):
            for k in range(w.nstlist):
                mxn.nb_forces(ctx, state["grid"], state["lst"], xq[k], params, mxn.NB_ENERGY, f, e)
        torch.cuda.synchronize()
        call_blocks.append((time.perf_counter() - tb) * 1e6 / (3 * w.nstlist))
    # the list build (grid sort + asynchronous pair list) the same way: blocks of 10, host clock
    build_blocks = []
    for _ in range(3):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _r in range(10):
            state["grid"] = mxn.nb_grid_sort(ctx, box.box, xq[0], typ, (m, n), state["grid"])
            state["lst"] = mxn.nb_pairlist_build(ctx, state["grid"], w.rlist, -1.0, eo, ei,
                                                 mxn.NB_LIST_ASYNC | order_flag, state["lst"])
        torch.cuda.synchronize()
        build_blocks.append((time.perf_counter() - tb) * 1e6 / 10)
    mxn.nb_sync(ctx)

    # pair counts per force call (averaged over the 10 positions of a list lifetime)
    listed, real, inr, exc = 0, 0, 0, 0
    for k in range(w.nstlist):
        c = mxn.nb_list_stats(ctx, state["grid"], state["lst"], xq[k], w.rc)
        listed += c[0]; real += c[1]; inr += c[2]; exc += c[3]
    listed /= w.nstlist; real /= w.nstlist; inr /= w.nstlist; exc /= w.nstlist
    ms_step = (t1 - t0) * 1e3 / args.steps
    calls = w.nstlist
    value = listed * calls / (ms_step * 1e-3)
    eff = inr * calls / (ms_step * 1e-3)
    fk_ms, fk_n = tim["force_kernel"]
    fk_avg = fk_ms / max(fk_n, 1) * 1e-3
    # the flop count per pair is the analytic-Ewald kernel's; other Coulomb variants report no roofline
    alg_flops = FLOPS_PER_PAIR * (inr + exc) + FLOPS_PER_DISTANCE * (listed - inr - exc)
    achieved = alg_flops / fk_avg
    paper_conv = FLOPS_PER_PAIR * listed / fk_avg
    gs_ms, gs_n = stage["grid_sort"]
    pl_ms, pl_n = stage["pairlist"]
    fc_ms, fc_n = stage["force_call"]
    gi = mxn.nb_grid_info(state["grid"])
    n_entries = mxn.nb_list_info(state["lst"])[0]
    lb_bytes = list_build_bytes(box.n, gi["n_slots"], gi["n_ci"], gi["n_cj"], n_entries)
    lb_us = float(np.median(build_blocks))   # no timer in the stream
    lb_us_timed = gs_ms / max(gs_n, 1) * 1e3 + pl_ms / max(pl_n, 1) * 1e3
    result = {
        "metric": METRIC, "value": value, "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "n_atoms": box.n, "box_nm": w.L, "shape": "%dx%d" % (m, n), "rc": w.rc,
                   "rlist": w.rlist, "beta": w.beta, "nstlist": w.nstlist, "energies": "every step",
                   "force_calls_per_step": calls, "force_kernel": args.variant, "list_order": args.list_order,
                   "coulomb": args.coulomb},
        "roofline": ({"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                      "frac": achieved / PEAK_FP32, "traffic": force_traffic_bytes(),
                      "convention": "strict: %d flops per pair within rc + %d per other listed pair"
                                    % (FLOPS_PER_PAIR, FLOPS_PER_DISTANCE),
                      "flops_per_call": alg_flops,
                      "computed_pair": {"convention": "%d flops per listed pair (the paper's pairs-per-cycle count)"
                                                      % FLOPS_PER_PAIR,
                                        "flops_per_call": FLOPS_PER_PAIR * listed, "achieved": paper_conv / 1e12,
                                        "frac": paper_conv / PEAK_FP32},
                      "non_packed_peak": PEAK_FP32 / 2e12, "frac_of_non_packed_peak": 2.0 * achieved / PEAK_FP32}
                     if args.coulomb == "ewald" else None),
        "effective_pairs_per_s": eff,
        "pct_fp32_valu_peak": 100.0 * achieved / PEAK_FP32,
        "pairs_per_force_call": {"listed": listed, "real": real, "within_rc": inr, "excluded_within_rc": exc,
                                 "effective_ratio": inr / listed},
        "force_kernel_us": fk_avg * 1e6,
        "force_kernel_timed_launches": fk_n,
        "force_kernel_pairs_per_s": listed / fk_avg,
        "force_kernel_paper_convention_tflops": paper_conv / 1e12,
        "force_call_us": float(np.median(call_blocks)),
        "force_call_us_every_launch_timed": fc_ms / max(fc_n, 1) * 1e3,
        "grid_sort_us": gs_ms / max(gs_n, 1) * 1e3,
        "pairlist_us": pl_ms / max(pl_n, 1) * 1e3,
        "list_build": {"bytes": lb_bytes, "us": lb_us, "GB_per_s": lb_bytes / (lb_us * 1e-6) / 1e9,
                       "entries": n_entries, "bound": "hbm", "frac_of_hbm_peak": lb_bytes / (lb_us * 1e-6) / 8e12,
                       "us_every_stage_timed": lb_us_timed},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(box, w)
    mxn.nb_list_free(state["lst"])
    mxn.nb_grid_free(state["grid"])
    mxn.nb_destroy(ctx)
    print(json.dumps(result), flush=True)


def bench_twostage(args):
    """Two-stage list on the production box (Sec. 2.3's box-only search plus GPU prune): time per force step of
    (one-stage) the production cycle, (two-stage) a box-only search pruned at rlist once per build, and
    (rolling) a box-only outer list of its own radius and lifetime pruned every few steps at an inner radius.
    Every variant runs the same ballistic trajectory; the pairs within rc that each one finds per step are
    counted (nb_list_stats), so a variant that loses pairs shows it."""
    import numpy as np
    import torch
    import synth
    import paper_1306_1737_amd as mxn

    w = synth.PRODUCTION
    m, n = (int(v) for v in args.shape.split("x"))
    r_out = args.outer_rlist or w.rlist
    n_out = args.outer_nstlist or w.nstlist
    P = max(1, args.prune_every)
    print("[bench] generating %d waters" % w.n_mol, file=sys.stderr, flush=True)
    box = synth.water_box(w.n_mol, w.L, seed=1306)
    vel = synth.velocities(box.mass, w.T, seed=1306)
    xs = synth.free_flight(box.xyz, vel, w.dt, max(w.nstlist, n_out))
    dev = torch.device("cuda:0")
    xq = [torch.from_numpy(box.xyzq(x)).to(dev) for x in xs]
    typ = torch.from_numpy(box.type).to(dev)
    eo = torch.from_numpy(box.excl_off).to(dev)
    ei = torch.from_numpy(box.excl_idx).to(dev)
    lj = torch.from_numpy(synth.lj_table_spce().astype(np.float32)).to(dev)
    f = torch.zeros((box.n, 3), dtype=torch.float32, device=dev)
    e = torch.zeros(2, dtype=torch.float64, device=dev)
    ctx = mxn.nb_create(0)
    params = mxn.make_params(w.rc, w.beta, synth.COULOMB_F, lj)
    st = {"grid": None, "lst": None, "inner": None}

    def cycle(kind, list_flags, stats=None):
        st["grid"] = mxn.nb_grid_sort(ctx, box.box, xq[0], typ, (m, n), st["grid"])
        if kind == "one-stage":
            st["lst"] = mxn.nb_pairlist_build(ctx, st["grid"], w.rlist, -1.0, eo, ei, list_flags, st["lst"])
            steps, use = w.nstlist, (lambda k: st["lst"])
        elif kind == "two-stage":
            st["lst"] = mxn.nb_pairlist_build(ctx, st["grid"], w.rlist, w.rlist, eo, ei, list_flags, st["lst"])
            st["inner"] = mxn.nb_pairlist_prune(ctx, st["lst"], xq[0], w.rlist, st["inner"])
            steps, use = w.nstlist, (lambda k: st["inner"])
        else:
            st["lst"] = mxn.nb_pairlist_build(ctx, st["grid"], r_out, r_out, eo, ei, list_flags, st["lst"])
            steps, use = n_out, (lambda k: st["inner"])
        for k in range(steps):
            if kind == "rolling" and k % P == 0:
                st["inner"] = mxn.nb_pairlist_prune(ctx, st["lst"], xq[k], args.r_inner, st["inner"])
            mxn.nb_forces(ctx, st["grid"], use(k), xq[k], params, mxn.NB_ENERGY, f, e)
            if stats is not None:
                c = mxn.nb_list_stats(ctx, st["grid"], use(k), xq[k], w.rc)
                stats.append((c[0], c[2] + c[3]))
        return steps

    out = {}
    for kind in ("one-stage", "two-stage", "rolling"):
        print("[bench] %s" % kind, file=sys.stderr, flush=True)
        cycle(kind, 0)                      # sizes the list storage (one synchronisation)
        mxn.nb_sync(ctx)
        stats = []
        cycle(kind, mxn.NB_LIST_ASYNC, stats)
        for _ in range(max(0, args.warmup - 1)):
            cycle(kind, mxn.NB_LIST_ASYNC)
        mxn.nb_sync(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        calls = 0
        for _ in range(args.steps):
            calls += cycle(kind, mxn.NB_LIST_ASYNC)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mxn.nb_sync(ctx)
        out[kind] = {"ms_per_force_step": (t1 - t0) * 1e3 / calls, "force_steps": calls,
                     "listed_pairs_per_step": float(np.mean([s[0] for s in stats])),
                     "pairs_within_rc": [int(s[1]) for s in stats]}
        for h in ("inner", "lst"):
            if st[h] is not None:
                mxn.nb_list_free(st[h])
                st[h] = None
        mxn.nb_grid_free(st["grid"])
        st["grid"] = None
    base = out["one-stage"]
    for kind, r in out.items():   # pairs within rc each variant finds, against the one-stage list, per step
        k = min(len(r["pairs_within_rc"]), len(base["pairs_within_rc"]))
        r["pairs_within_rc_minus_one_stage"] = [a - b for a, b in zip(r["pairs_within_rc"][:k],
                                                                        base["pairs_within_rc"][:k])]
    ms = out["rolling"]["ms_per_force_step"]
    inr = float(np.mean(out["rolling"]["pairs_within_rc"]))
    result = {
        "metric": "atom-pair interactions/s within rc, two-stage list", "value": inr / (ms * 1e-3),
        "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name + "-twostage", "shape": "%dx%d" % (m, n), "rc": w.rc, "rlist": w.rlist,
                   "outer_rlist": r_out, "outer_nstlist": n_out, "prune_every": P, "r_inner": args.r_inner},
        "variants": out,
    }
    mxn.nb_destroy(ctx)
    print(json.dumps(result), flush=True)


def bench_rdf(args):
    """Pair correlation function on the production box (Sec. 1 and 2.3): each frame of the ballistic trajectory
    is grid-sorted, gets a box-only list (no particle prune) at rc + 0.01 nm, and the pair distance histogram
    of its pairs below rc (per type pair, exact counts).  Times whole frames and the histogram kernel alone."""
    import numpy as np
    import torch
    import synth
    import paper_1306_1737_amd as mxn

    w = synth.PRODUCTION
    m, n = (int(v) for v in args.shape.split("x"))
    r_max, nbins, rl = w.rc, args.rdf_bins, w.rc + 0.01
    print("[bench] generating %d waters" % w.n_mol, file=sys.stderr, flush=True)
    box = synth.water_box(w.n_mol, w.L, seed=1306)
    vel = synth.velocities(box.mass, w.T, seed=1306)
    xs = synth.free_flight(box.xyz, vel, w.dt, w.nstlist)
    dev = torch.device("cuda:0")
    xq = [torch.from_numpy(box.xyzq(x)).to(dev) for x in xs]
    typ = torch.from_numpy(box.type).to(dev)
    eo = torch.from_numpy(box.excl_off).to(dev)
    ei = torch.from_numpy(box.excl_idx).to(dev)
    nt = int(box.type.max()) + 1
    hist = torch.zeros(nt * nt * nbins, dtype=torch.int64, device=dev)
    ctx = mxn.nb_create(0)
    st = {"grid": None, "lst": None}

    def frame(k, flags):
        st["grid"] = mxn.nb_grid_sort(ctx, box.box, xq[k], typ, (m, n), st["grid"])
        st["lst"] = mxn.nb_pairlist_build(ctx, st["grid"], rl, rl, eo, ei, flags, st["lst"])
        mxn.nb_rdf(ctx, st["grid"], st["lst"], xq[k], r_max, nbins, nt, hist)

    frame(0, 0)                       # sizes the list storage
    mxn.nb_sync(ctx)
    for k in range(args.warmup):
        frame(k % len(xq), mxn.NB_LIST_ASYNC)
    mxn.nb_sync(ctx)
    hist.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        frame(s % len(xq), mxn.NB_LIST_ASYNC)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mxn.nb_sync(ctx)
    counted = int(hist.sum().item()) / args.steps
    listed = mxn.nb_list_stats(ctx, st["grid"], st["lst"], xq[(args.steps - 1) % len(xq)], r_max)[0]
    reps = 20
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(reps):
        mxn.nb_rdf(ctx, st["grid"], st["lst"], xq[(args.steps - 1) % len(xq)], r_max, nbins, nt, hist)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ms_frame = (t1 - t0) * 1e3 / args.steps
    us_rdf = (t3 - t2) * 1e6 / reps
    result = {
        "metric": "pair distances binned/s (pair correlation function)", "value": counted / (ms_frame * 1e-3),
        "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_frame,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name + "-rdf", "shape": "%dx%d" % (m, n), "r_max": r_max, "nbins": nbins,
                   "list": "box-only, rlist = r_max + 0.01 nm, rebuilt every frame"},
        "pairs_counted_per_frame": counted, "listed_pairs_per_frame": listed,
        "histogram_call_us": us_rdf, "listed_pairs_per_s_histogram": listed / (us_rdf * 1e-6),
    }
    mxn.nb_list_free(st["lst"])
    mxn.nb_grid_free(st["grid"])
    mxn.nb_destroy(ctx)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
