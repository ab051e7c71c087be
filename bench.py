"""Benchmark of the cell-list neighbour operators on one MI355X.

A step is one pass of the whole hot path over the 2^20-particle periodic cube
(spring force, ~30 neighbours within r = 1, float32): rebuild the cell list
from the original-order positions (cell ids, radix sort, offsets, gather), the
neighbour-sum forward and its adjoint for a seeded upstream gradient.  The step
is captured once as a HIP graph and replayed; the headline value is ordered
pair interactions per second of the step.  Three forms of the step are timed
on three grids (cells about r wide, and r/2 or r/3 wide along x): both sums
searching the box, a recorded neighbour list replayed by both, and a forward
that records each row's accepted candidates for the adjoint to replay.  The
headline takes the fastest form on the --reach grid.

The JSON line's roofline is the step's longest single kernel, the forward (one
kernel per call), timed with HIP events on its own stream: algorithmic lane-ops
per launch (7 per candidate tested, 12 per accepted pair; candidates counted from
the built offsets) over the launch time, against the plain VALU issue rate, with
its HBM fraction on the method's own bytes beside it and the counted traffic from
the committed rocprofv3 summary.  The CPU baseline is the C oracle without
tolerance scales, on every core the process may use and on one core (a row
sample), median of three runs each.  The line also carries the per-phase
breakdown, the per-variant table and the other workloads: candidate reduction at
reach 2, the dense Gaussian and multiquadric sums and adjoint, the soft-sphere
energy gradient, 512 uneven systems in one graph against the single cube run
with the same step form, the molecular dynamics example and the small-N
workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-extra] [--reach 3,1,1] [--no-reach-trials]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X peaks used as roofline denominators
HBM_PEAK_GBS = 8000.0
# plain VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one lane-op per
# lane per clock; packed fp32 is not used), in 10^12 lane-operations per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic VALU lane-operations (transcendental instructions -- exp2, sqrt, rsqrt -- issue
# to their own unit and are counted only inside the per-pair figures below).  Per candidate of the box search: 3 sub, 1 mul, 2 fma, 1 compare.  Per
# accepted pair of the spring forward: about 12 (the reciprocal square root and the force).
# Per replayed pair: its displacement and squared distance again (3 sub, 1 mul, 2 fma).  Per
# pair of the spring adjoint: 3 sub for w, 3 for w.dx, 1 for g, 3 mul for w_par's factor and
# gpar, 3 fma for w_perp, 6 fma into the sums = 19.
OPS_PER_CANDIDATE = 7
OPS_PER_PAIR_FWD = 12
OPS_PER_REPLAYED_PAIR = 6
OPS_PER_PAIR_BWD = 19
# Algorithmic HBM bytes per particle (float32, d = 3): the build reads x (12) and writes a key
# (4), makes one sort pass over the high key bits (16), gathers into cell order (28) and writes
# the offsets (4.5); the forward reads xs (16), the offsets and perm (about 8.5) and writes y
# (12 less the shared offset reads: 28.5 in all); the spring adjoint reads xs (16), gy (12) and
# perm (4) and writes gx (12).  Implementation overheads, reported apart: the recorded masks
# (two 32-bit words per stencil row and a status word, 76 B written and read) and the gather of
# gy into cell order (perm 4 + 12 in + 12 out).
BYTES_BUILD = 16 + 16 + 28 + 4.5
BYTES_FWD = 28.5
BYTES_BWD_SPRING = 44
MASK_RECORD_BYTES = 76
GY_GATHER_BYTES = 28

METRIC = "pair interactions/s (fwd and fwd+bwd) at stated tol; % HBM roofline"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def hip_download(ptr: int, count: int, dtype) -> np.ndarray:
    out = np.zeros(max(count, 1), dtype=dtype)
    if count:
        hip = C.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        assert hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(ptr), count * out.itemsize, 2) == 0
    return out[:count]


COUNTERS = os.path.join(ROOT, "profiles", "spring_cube_n1048576_hbm_counters.txt")


def counted_traffic(names):
    """HBM bytes per launch of the named kernels (summed) from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary (calibrated by a plain device
    copy); None when the summary is missing or does not list one of them."""
    if not names or not os.path.exists(COUNTERS):
        return None
    mb = {}
    with open(COUNTERS) as f:
        for line in f:
            parts = line.rsplit(None, 4)
            if len(parts) == 5:
                try:
                    mb[parts[0].strip()] = float(parts[4])
                except ValueError:
                    pass
    if not all(k in mb for k in names):
        return None
    return sum(mb[k] for k in names) * 1e6


def profile_names(variant_name, direction):
    """Kernel names as rocprofv3 reports them for the spring cube (float32, d = 3, no batch,
    32-bit row offsets)."""
    if "recorded" in variant_name:
        k = ["k_nbr_fwd<float, 3, 1, false>"] if direction == "fwd" else ["k_nbr_bwd<float, 3, 1, false>"]
    elif "accepted-pair bit masks" in variant_name:
        k = ["k_lane_mask<float, 3, 1, false, true, %d>" % (0 if direction == "fwd" else 1)]
    elif "flattened" in variant_name:
        k = ["k_flat<float, 3, 1, false, true, %d>" % (0 if direction == "fwd" else 1)]
    elif direction == "fwd":
        k = ["k_lane_fwd<float, 3, 1, false, true>"]
    else:
        k = ["k_lane_bwd<float, 3, 1, false, true>"]
    return k if direction == "fwd" else ["k_gather_rows<float, 3, 4>"] + k


def candidate_count(cells, reach) -> int:
    """Candidates the box search of a periodic 3-d grid tests: sum over cells of
    count(c) * count(the cells up to reach[k] away in each dimension k around c)."""
    v = cells.view()
    off = hip_download(v.cell_offsets, int(v.ncells) + 1, np.uint32).astype(np.int64)
    n = [v.ncell_host[k] for k in range(3)]
    cnt = np.diff(off).reshape(n[2], n[1], n[0])
    s = np.zeros_like(cnt)
    mx, my, mz = reach
    for dz in range(-mz, mz + 1):
        for dy in range(-my, my + 1):
            for dx in range(-mx, mx + 1):
                s += np.roll(cnt, (dz, dy, dx), axis=(0, 1, 2))
    return int((cnt * s).sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--reach", default="3,1,1",
                    help="search reach per dimension of the headline cell grid (x,y,z)")
    ap.add_argument("--no-reach-trials", action="store_true",
                    help="set up only the --reach grid (no trials at other reaches, no per-variant table)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (known bytes) to calibrate HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1704_08907_amd as A
    from paper_1704_08907_amd import synthetic as syn

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)
    ctx = A.Context(0, stream)

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)  # reads and writes 256 MiB each
        torch.cuda.synchronize()
        del src, dst

    # ---------------- headline workload: spring cube, build + fwd + bwd ----------------
    w = syn.spring_cube()
    s = w.systems[0]
    x = torch.from_numpy(s.x).to(dev)
    gy = torch.from_numpy(w.extra["gy"]).to(dev)
    n = s.n
    y = torch.empty((n, 3), device=dev)
    gx = torch.empty((n, 3), device=dev)
    # box search whose forward records each stencil row's accepted candidates, which the
    # adjoint replays instead of testing every candidate again
    mask_variant = next(v for v in range(A.variant_count()) if "accepted-pair bit masks" in A.variant_name(v))

    def capture(fn):
        fn()
        stream.synchronize()
        A.graph_capture_begin(ctx)
        fn()
        return A.graph_capture_end(ctx)

    def run_graph(g, warmup, steps):
        for _ in range(warmup):
            A.graph_launch(ctx, g)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            A.graph_launch(ctx, g)
        e1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.sync()
        return (t1 - t0) * 1e3 / steps, e0.elapsed_time(e1) / steps

    def setup(reach):
        """Cells of the cube at a search reach per dimension, the tuned variants and the step forms."""
        st = {"reach": reach}
        box = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, None, reach)
        # the radix build's shape (sort tile, bucket bits) for this grid, then its cells
        st["build_shape"] = list(A.autotune_build(ctx, x, [box]))
        cells = A.build_cells(ctx, x, [box])
        st["box"], st["cells"] = box, cells
        # box-search baseline: the autotuner's fastest mapping without a neighbour list
        st["search_fwd"] = A.autotune(ctx, cells, "spring", (1.0,))
        st["search_bwd"] = A.autotune(ctx, cells, "spring", (1.0,), gy=gy)
        # record the neighbour lists; the tuner then also times their replay
        st["cap"] = A.build_neighbours(ctx, cells)
        st["variant_fwd"] = A.autotune(ctx, cells, "spring", (1.0,))
        st["variant_bwd"] = A.autotune(ctx, cells, "spring", (1.0,), gy=gy)

        def step():
            A.build_cells(ctx, x, [box], cells=cells)
            A.build_neighbours(ctx, cells)
            A.pair_sum(ctx, cells, "spring", (1.0,), y=y)
            A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy, gx=gx)

        def step_search():
            A.build_cells(ctx, x, [box], cells=cells)
            ctx.set_variant(st["search_fwd"])
            A.pair_sum(ctx, cells, "spring", (1.0,), y=y)
            ctx.set_variant(st["search_bwd"])
            A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy, gx=gx)
            ctx.set_variant(-1)

        def step_masks():
            A.build_cells(ctx, x, [box], cells=cells)
            ctx.set_variant(mask_variant)
            A.pair_sum(ctx, cells, "spring", (1.0,), y=y)
            A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy, gx=gx)
            ctx.set_variant(-1)

        def step_fused():
            A.build_cells(ctx, x, [box], cells=cells)
            A.pair_sum_and_backward(ctx, cells, "spring", (1.0,), gy, y=y, gx=gx)

        st["forms"] = {"neighbour_list": step, "box_search": step_search, "recorded_masks": step_masks,
                       "fused_gy_known": step_fused}
        return st

    # The step forms are timed briefly on the paper's lattice (reach 1: cells about r wide,
    # searched one cell deep) and on grids with cells r/2 and r/3 wide along x only (the same
    # nine rows, each shorter).  The headline grid is --reach (cells r/3 wide along x, the
    # fastest of the three when measured), its fastest form the headline step.  The fused
    # form (forward and adjoint from one box search) needs gy before the forward, which a
    # training step does not have, so it is reported beside the headline, not as it.
    head_reach = [int(v) for v in args.reach.split(",")]
    head_tag = "".join(map(str, head_reach))
    reaches = [head_reach] if args.no_reach_trials else \
        [m for m in ([1, 1, 1], [2, 1, 1], [3, 1, 1]) if m != head_reach] + [head_reach]
    trial = {}
    setups = {}
    for reach in reaches:
        st = setup(reach)
        tag = "".join(map(str, reach))
        setups[tag] = st
        for name, fn in st["forms"].items():
            g = capture(fn)
            trial["%s@%s" % (name, tag)] = max(run_graph(g, 2, max(5, args.steps // 5)))
            g.close()
    best = min((k for k in trial if not k.startswith("fused") and k.endswith("@" + head_tag)), key=trial.get)
    mode, tag = best.split("@")
    log("step trials (ms): %s -> headline uses %s" % (json.dumps(trial), best))
    chosen = setups[tag]
    reach, box, cells = chosen["reach"], chosen["box"], chosen["cells"]
    search_fwd, search_bwd = chosen["search_fwd"], chosen["search_bwd"]
    variant_fwd, variant_bwd, cap = chosen["variant_fwd"], chosen["variant_bwd"], chosen["cap"]
    for k, st in setups.items():
        if k not in (tag, "111"):
            st["cells"].close()
    cells1 = setups["111"]["cells"] if "111" in setups else None  # the per-variant table's lattice
    cnt = A.pair_sum(ctx, cells, "count", ())
    ctx.sync()
    pairs = int(cnt.sum().item())
    cand = candidate_count(cells, reach)
    log("spring cube: n=%d pairs=%d candidates=%d (%.1f/particle) at reach %s; variants: forward %d (%s), "
        "adjoint %d (%s); list capacity %d" % (n, pairs, cand, cand / n, reach, variant_fwd,
                                               A.variant_name(variant_fwd), variant_bwd,
                                               A.variant_name(variant_bwd), cap))
    graph = capture(chosen["forms"][mode])
    wall_ms, ev_ms = run_graph(graph, args.warmup, args.steps)
    ms = max(wall_ms, ev_ms)
    value = pairs / (ms * 1e-3)
    log("step: %.3f ms (events %.3f ms, wall %.3f ms) -> %.3e pairs/s" % (ms, ev_ms, wall_ms, value))

    # ---------------- per-phase breakdown: each phase captured as its own graph ------------
    def timed(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def timed_graph(fn, reps=20):
        """GPU time of fn's kernels, replayed from a graph (no host launch gaps)."""
        fn()
        stream.synchronize()
        A.graph_capture_begin(ctx)
        fn()
        g = A.graph_capture_end(ctx)
        t = timed(lambda: A.graph_launch(ctx, g), reps)
        g.close()
        return t

    t_build = timed_graph(lambda: A.build_cells(ctx, x, [box], cells=cells))
    ctx.set_build_strategy("counting")
    t_build_counting = timed_graph(lambda: A.build_cells(ctx, x, [box], cells=cells))
    ctx.set_build_strategy("radix")
    A.build_cells(ctx, x, [box], cells=cells)
    t_nbr = timed_graph(lambda: A.build_neighbours(ctx, cells))
    A.build_neighbours(ctx, cells)
    t_fwd_list = timed_graph(lambda: A.pair_sum(ctx, cells, "spring", (1.0,), y=y))
    t_bwd_list = timed_graph(lambda: A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy, gx=gx))
    ctx.set_variant(search_fwd)
    t_fwd_search = timed_graph(lambda: A.pair_sum(ctx, cells, "spring", (1.0,), y=y))
    ctx.set_variant(search_bwd)
    t_bwd_search = timed_graph(lambda: A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy, gx=gx))
    ctx.set_variant(mask_variant)  # each forward records the masks the adjoints then replay
    t_fwd_mask = timed_graph(lambda: A.pair_sum(ctx, cells, "spring", (1.0,), y=y))
    t_bwd_mask = timed_graph(lambda: A.pair_sum_backward(ctx, cells, "spring", (1.0,), gy, gx=gx))
    # the half stencil (each pair tested once, the partner reads the recorded bit): forward
    # only, timed after the replay because it leaves records that no adjoint replays
    ctx.set_variant(next(v for v in range(A.variant_count()) if "half stencil" in A.variant_name(v)))
    t_fwd_half = timed_graph(lambda: A.pair_sum(ctx, cells, "spring", (1.0,), y=y))
    ctx.set_variant(-1)
    per_variant = {}  # on the paper's lattice (reach 1), where every variant applies
    if cells1 is not None:
        A.build_cells(ctx, x, [setups["111"]["box"]], cells=cells1)
        A.build_neighbours(ctx, cells1)  # for the replayed-list variant
    for v in range(A.variant_count() if cells1 is not None else 0):
        ctx.set_variant(v)
        try:
            per_variant[A.variant_name(v)] = {
                "fwd_ms": timed_graph(lambda: A.pair_sum(ctx, cells1, "spring", (1.0,), y=y), reps=5),
                "bwd_ms": timed_graph(lambda: A.pair_sum_backward(ctx, cells1, "spring", (1.0,), gy, gx=gx),
                                      reps=5)}
        except A.AboriaError as e:  # a variant whose requirements these cells do not meet
            per_variant[A.variant_name(v)] = {"not_applicable": str(e)}
    ctx.set_variant(-1)
    ctx.sync()
    log("variants", json.dumps(per_variant))
    nc = int(cells.view().ncells)

    def kernel_of(v, direction):
        """The call's kernels as rocprofv3 names them (a readable label where no profile row exists)."""
        names = profile_names(A.variant_name(v), direction)
        return " + ".join(names) if names else A.variant_name(v)

    # The calls of the chosen step form: (kernels, time, algorithmic lane-ops, algorithmic bytes).
    # Algorithmic work is the method's own (per-unit figures in the module docstring): a box search
    # tests every candidate and evaluates the summand per accepted pair; a call that replays
    # recorded pairs recomputes each pair's displacement and evaluates its summand.  Bytes are the
    # method's per-particle traffic (forward 28.5, spring adjoint 44); what an implementation adds
    # (a mask record, a neighbour list, gathering gy into cell order) is reported as overhead.
    if mode == "recorded_masks":
        v_f, v_b, t_fwd, t_bwd = mask_variant, mask_variant, t_fwd_mask, t_bwd_mask
        extra_bytes = {"fwd": n * MASK_RECORD_BYTES, "bwd": n * (MASK_RECORD_BYTES + GY_GATHER_BYTES)}
        ops_bwd = pairs * (OPS_PER_REPLAYED_PAIR + OPS_PER_PAIR_BWD)
    elif mode == "box_search":
        v_f, v_b, t_fwd, t_bwd = search_fwd, search_bwd, t_fwd_search, t_bwd_search
        extra_bytes = {"fwd": 0, "bwd": n * GY_GATHER_BYTES}
        ops_bwd = cand * OPS_PER_CANDIDATE + pairs * OPS_PER_PAIR_BWD
    else:
        v_f, v_b, t_fwd, t_bwd = variant_fwd, variant_bwd, t_fwd_list, t_bwd_list
        extra_bytes = {"fwd": 4 * pairs, "bwd": 4 * pairs + n * GY_GATHER_BYTES}
        ops_bwd = pairs * (OPS_PER_REPLAYED_PAIR + OPS_PER_PAIR_BWD)
    ops_fwd = (pairs * (OPS_PER_REPLAYED_PAIR + OPS_PER_PAIR_FWD) if mode == "neighbour_list"
               else cand * OPS_PER_CANDIDATE + pairs * OPS_PER_PAIR_FWD)
    phases = {"fwd": (kernel_of(v_f, "fwd"), t_fwd, ops_fwd, n * BYTES_FWD, profile_names(A.variant_name(v_f), "fwd")),
              "bwd": (kernel_of(v_b, "bwd"), t_bwd, ops_bwd, n * BYTES_BWD_SPRING,
                      profile_names(A.variant_name(v_b), "bwd"))}
    if mode == "neighbour_list":
        phases["neighbours"] = ("k_nbr_build<float, 3, false> (neighbour-list recording)", t_nbr,
                                cand * OPS_PER_CANDIDATE, 0, None)

    def roof(key):
        kname, t, ops, nbytes, pnames = phases[key]
        traffic = counted_traffic(pnames)
        ach_ops = ops / (t * 1e-3) / 1e12
        ach_bytes = nbytes / (t * 1e-3) / 1e9
        # the binding roofline is the one the algorithmic work would reach first
        alu = ops / (VALU_PEAK_TOPS * 1e12) >= nbytes / (HBM_PEAK_GBS * 1e9)
        out = {"bound": "alu" if alu else "hbm", "kernel": kname,
               "achieved": ach_ops if alu else ach_bytes, "peak": VALU_PEAK_TOPS if alu else HBM_PEAK_GBS,
               "unit": "Tops/s" if alu else "GB/s",
               "frac": ach_ops / VALU_PEAK_TOPS if alu else ach_bytes / HBM_PEAK_GBS,
               "traffic": traffic, "algorithmic_ops_per_launch": ops, "algorithmic_bytes_per_launch": nbytes,
               "hbm_frac": ach_bytes / HBM_PEAK_GBS, "valu_frac": ach_ops / VALU_PEAK_TOPS,
               "overhead_bytes_per_launch": extra_bytes.get(key, 0), "avg_launch_ms": t}
        return out

    # the roofline line is the longest single kernel of the step: the forward call is one
    # kernel; the adjoint call is two (gy gather + the adjoint), so its adjoint kernel is
    # shorter than the call
    roofline = roof("fwd")
    build_bytes = n * BYTES_BUILD
    step_bytes = build_bytes + n * (BYTES_FWD + BYTES_BWD_SPRING)
    t_fused = trial["fused_gy_known@" + head_tag]
    breakdown = {"step_form": mode, "search_reach": reach, "ncell": [int(cells.view().ncell_host[k]) for k in range(3)],
                 "step_trials_ms": trial,
                 "fwd_pairs_per_s": pairs / ((t_build + t_fwd) * 1e-3),
                 "fwd_bwd_pairs_per_s": value,
                 "fused_gy_known_pairs_per_s": pairs / (t_fused * 1e-3),
                 "step_algorithmic_bytes": step_bytes,
                 "step_hbm_frac": step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "build_ms": t_build, "build_shape_keys_per_thread_bucket_bits_shuffle": chosen["build_shape"],
                 "build_counting_ms": t_build_counting, "fwd_ms": t_fwd, "bwd_ms": t_bwd,
                 "box_search_fwd_ms": t_fwd_search, "box_search_bwd_ms": t_bwd_search,
                 "recorded_masks_fwd_ms": t_fwd_mask, "recorded_masks_bwd_ms": t_bwd_mask,
                 "half_stencil_fwd_ms": t_fwd_half,
                 "neighbour_list_record_ms": t_nbr, "replay_fwd_ms": t_fwd_list, "replay_bwd_ms": t_bwd_list,
                 "build_hbm_frac": build_bytes / (t_build * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "roofline_per_call": {k: {q: v for q, v in roof(k).items()
                                           if q in ("kernel", "bound", "frac", "hbm_frac", "valu_frac",
                                                    "avg_launch_ms", "traffic", "overhead_bytes_per_launch")}
                                       for k in phases},
                 "candidates_per_step": cand, "list_capacity": cap,
                 "step_variant_fwd": A.variant_name(v_f), "step_variant_bwd": A.variant_name(v_b),
                 "box_search_variant_fwd": A.variant_name(search_fwd),
                 "box_search_variant_bwd": A.variant_name(search_bwd),
                 "per_variant": per_variant}
    log("breakdown", json.dumps(breakdown))

    # ---------------- other workloads ----------------
    extra = {}
    if not args.no_extra:
        # candidate reduction: the same cube on cells about r/2 wide searched two cells deep,
        # by the row search and by the flattened, pruned search
        box_r2 = A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff, None, 2)
        c_r2 = A.build_cells(ctx, x, [box_r2])
        r2 = {"ncell": [int(c_r2.view().ncell_host[k]) for k in range(3)],
              "build_ms": timed_graph(lambda: A.build_cells(ctx, x, [box_r2], cells=c_r2), reps=10)}
        for label, word in (("row_search", "adjoint evaluated on every candidate"), ("flattened", "flattened")):
            ctx.set_variant(next(v for v in range(A.variant_count()) if word in A.variant_name(v)))
            r2[label + "_fwd_ms"] = timed_graph(lambda: A.pair_sum(ctx, c_r2, "spring", (1.0,), y=y), reps=10)
            r2[label + "_bwd_ms"] = timed_graph(
                lambda: A.pair_sum_backward(ctx, c_r2, "spring", (1.0,), gy, gx=gx), reps=10)
        ctx.set_variant(-1)
        r2["step_ms_best"] = r2["build_ms"] + min(r2["row_search_fwd_ms"], r2["flattened_fwd_ms"]) + min(
            r2["row_search_bwd_ms"], r2["flattened_bwd_ms"])
        extra["spring_cube_reach2"] = r2
        c_r2.close()

        # dense Gaussian sum, N = 65536, d = 2
        xd, wd, sigma = syn.gaussian_square()
        xd_t = torch.from_numpy(xd).to(dev)
        wd_t = torch.from_numpy(wd).to(dev)
        yd = torch.empty(xd.shape[0], device=dev)
        npair = float(xd.shape[0]) ** 2
        gyd = torch.from_numpy(syn.SplitMix64(12).normal(xd.shape[0]).astype(np.float32)).to(dev)
        # the launch plans (targets per lane, workgroup target): the untuned default, then the
        # dense tuner's choice for each call
        t_dense0 = timed(lambda: A.dense_sum(ctx, xd_t, xd_t, wd_t, sigma, y=yd), reps=10)
        t_dense_b0 = timed(lambda: A.dense_sum_backward(ctx, xd_t, xd_t, wd_t, sigma, gyd), reps=5)
        t_mq0 = timed(lambda: A.dense_sum(ctx, xd_t, xd_t, wd_t, 0.1, y=yd, kernel="multiquadric"), reps=10)
        plan_g = A.autotune_dense(ctx, xd_t, xd_t, wd_t, sigma)
        plan_gb = A.autotune_dense(ctx, xd_t, xd_t, wd_t, sigma, gy=gyd)
        plan_mq = A.autotune_dense(ctx, xd_t, xd_t, wd_t, 0.1, kernel="multiquadric")
        t_dense = timed(lambda: A.dense_sum(ctx, xd_t, xd_t, wd_t, sigma, y=yd), reps=10)
        # per pair: 2 sub, 1 mul, 1 fma, 1 fma (and the exp2)
        extra["dense_gaussian_n65536"] = {"ms": t_dense, "pairs_per_s": npair / (t_dense * 1e-3),
                                          "valu_frac": npair * 5 / (t_dense * 1e-3) / 1e12 / VALU_PEAK_TOPS,
                                          "plan": A.dense_plan_name(plan_g), "ms_untuned": t_dense0}
        # its adjoint with targets = sources: K^T gy plus the target and source position gradients
        t_dense_b = timed(lambda: A.dense_sum_backward(ctx, xd_t, xd_t, wd_t, sigma, gyd), reps=5)
        # passes over the N^2 pairs: K^T gy with the source gradient, then the target gradient
        extra["dense_gaussian_n65536_adjoint"] = {"ms": t_dense_b, "pair_passes": 2,
                                                  "pairs_per_s": 2 * npair / (t_dense_b * 1e-3),
                                                  "plan": A.dense_plan_name(plan_gb), "ms_untuned": t_dense_b0}
        # the multiquadric basis of the RBF example, c = 0.1 (per pair: 2 sub, mul, fma, add of c^2,
        # fma, and the sqrt)
        t_mq = timed(lambda: A.dense_sum(ctx, xd_t, xd_t, wd_t, 0.1, y=yd, kernel="multiquadric"), reps=10)
        extra["dense_multiquadric_n65536"] = {"ms": t_mq, "pairs_per_s": npair / (t_mq * 1e-3),
                                              "valu_frac": npair * 6 / (t_mq * 1e-3) / 1e12 / VALU_PEAK_TOPS,
                                              "plan": A.dense_plan_name(plan_mq), "ms_untuned": t_mq0}
        del xd_t, wd_t, yd, gyd
        # soft sphere N = 2^18 forward + adjoint (energy gradient)
        w4 = syn.soft_sphere_cube()
        s4 = w4.systems[0]
        box4 = A.BoxSpec(3, s4.lo, s4.hi, s4.periodic, s4.cutoff)
        x4 = torch.from_numpy(s4.x).to(dev)
        g4 = torch.from_numpy(w4.extra["gy"]).to(dev)
        c4 = A.build_cells(ctx, x4, [box4])
        e4 = torch.empty((s4.n, 1), device=dev)
        gx4 = torch.empty((s4.n, 3), device=dev)
        p4 = int(A.pair_sum(ctx, c4, "count", ()).sum().item())
        sv4 = (A.autotune(ctx, c4, "soft_sphere", ()), A.autotune(ctx, c4, "soft_sphere", (), gy=g4))
        A.build_neighbours(ctx, c4)

        def step4(with_list):
            A.build_cells(ctx, x4, [box4], cells=c4)
            if with_list:
                A.build_neighbours(ctx, c4)
            ctx.set_variant(-1 if with_list else sv4[0])
            A.pair_sum(ctx, c4, "soft_sphere", (), y=e4)
            ctx.set_variant(-1 if with_list else sv4[1])
            A.pair_sum_backward(ctx, c4, "soft_sphere", (), g4, gx=gx4)
            ctx.set_variant(-1)

        def step4_fused():
            A.build_cells(ctx, x4, [box4], cells=c4)
            A.pair_sum_and_backward(ctx, c4, "soft_sphere", (), g4, y=e4, gx=gx4)

        def step4_masks(bx, cc):
            A.build_cells(ctx, x4, [bx], cells=cc)
            ctx.set_variant(mask_variant)
            A.pair_sum(ctx, cc, "soft_sphere", (), y=e4)
            A.pair_sum_backward(ctx, cc, "soft_sphere", (), g4, gx=gx4)
            ctx.set_variant(-1)

        # the same on cells r/3 wide along x (nine shorter rows)
        box4x = A.BoxSpec(3, s4.lo, s4.hi, s4.periodic, s4.cutoff, None, [3, 1, 1])
        c4x = A.build_cells(ctx, x4, [box4x])

        def step4_fused_x():
            A.build_cells(ctx, x4, [box4x], cells=c4x)
            A.pair_sum_and_backward(ctx, c4x, "soft_sphere", (), g4, y=e4, gx=gx4)

        # energy and its gradient: gy = 1 is known before the forward, so the fused form applies
        t4 = {"box_search": timed_graph(lambda: step4(False), reps=10),
              "neighbour_list": timed_graph(lambda: step4(True), reps=10),
              "recorded_masks": timed_graph(lambda: step4_masks(box4, c4), reps=10),
              "recorded_masks_reach_311": timed_graph(lambda: step4_masks(box4x, c4x), reps=10),
              "fused_energy_and_gradient": timed_graph(step4_fused, reps=10),
              "fused_energy_and_gradient_reach_311": timed_graph(step4_fused_x, reps=10)}
        c4x.close()
        m4 = min(t4.values())
        extra["soft_sphere_n262144_fwd_bwd"] = {"ms": m4, "pairs": p4, "pairs_per_s": p4 / (m4 * 1e-3),
                                                "step_forms_ms": t4}
        # 512 uneven systems: spring forward + soft-sphere adjoint in one graph
        w5 = syn.batch_cubes()
        xs5 = np.concatenate([q.x for q in w5.systems])
        off5 = np.concatenate([[0], np.cumsum([q.n for q in w5.systems])]).tolist()
        boxes5 = [A.BoxSpec(3, q.lo, q.hi, q.periodic, q.cutoff) for q in w5.systems]
        x5 = torch.from_numpy(xs5).to(dev)
        g5 = torch.from_numpy(w5.extra["gy"]).to(dev)
        # cell size tuned for this batch (rebuild + spring forward)
        boxes5, f5 = A.autotune_cells(ctx, x5, boxes5, off5, "spring", (1.0,))
        shape5 = A.autotune_build(ctx, x5, boxes5, off5)
        c5 = A.build_cells(ctx, x5, boxes5, off5)
        y5 = torch.empty((x5.shape[0], 3), device=dev)
        gx5 = torch.empty((x5.shape[0], 3), device=dev)
        p5 = int(A.pair_sum(ctx, c5, "count", ()).sum().item())
        sv5 = (A.autotune(ctx, c5, "spring", (1.0,)), A.autotune(ctx, c5, "soft_sphere", (), gy=g5))
        A.build_neighbours(ctx, c5)
        A.autotune(ctx, c5, "spring", (1.0,))
        A.autotune(ctx, c5, "soft_sphere", (), gy=g5)

        def step5(with_list):
            A.build_cells(ctx, x5, boxes5, off5, cells=c5)
            if with_list:
                A.build_neighbours(ctx, c5)
            ctx.set_variant(-1 if with_list else sv5[0])
            A.pair_sum(ctx, c5, "spring", (1.0,), y=y5)
            ctx.set_variant(-1 if with_list else sv5[1])
            A.pair_sum_backward(ctx, c5, "soft_sphere", (), g5, gx=gx5)
            ctx.set_variant(-1)

        def step5_masks():
            # the spring forward records the pairs; the soft-sphere adjoint replays them
            # (the pair set depends on positions and cutoffs only)
            A.build_cells(ctx, x5, boxes5, off5, cells=c5)
            ctx.set_variant(mask_variant)
            A.pair_sum(ctx, c5, "spring", (1.0,), y=y5)
            A.pair_sum_backward(ctx, c5, "soft_sphere", (), g5, gx=gx5)
            ctx.set_variant(-1)

        t5 = {"box_search": timed_graph(lambda: step5(False), reps=10),
              "neighbour_list": timed_graph(lambda: step5(True), reps=10)}
        if all(m <= 1 for b in boxes5 for m in b.reach_list()[1:]):  # the record covers 3^(d-1) rows
            t5["recorded_masks"] = timed_graph(step5_masks, reps=10)
        m5 = min(t5.values())
        ctx.sync()
        # the single-system reference for the same step: the 2^20 cube with the same step
        # forms (spring forward, soft-sphere adjoint), the same cell-size tuning and the same
        # variant policy, timed the same way
        boxes_s, f_s = A.autotune_cells(ctx, x, [A.BoxSpec(3, s.lo, s.hi, s.periodic, s.cutoff)], [0, n],
                                        "spring", (1.0,))
        A.autotune_build(ctx, x, boxes_s, [0, n])
        c_s = A.build_cells(ctx, x, boxes_s, [0, n])
        g_s = torch.ones((n, 1), device=dev)
        sv_s = (A.autotune(ctx, c_s, "spring", (1.0,)), A.autotune(ctx, c_s, "soft_sphere", (), gy=g_s))

        def step_single(masks):
            A.build_cells(ctx, x, boxes_s, [0, n], cells=c_s)
            ctx.set_variant(mask_variant if masks else sv_s[0])
            A.pair_sum(ctx, c_s, "spring", (1.0,), y=y)
            if not masks:
                ctx.set_variant(sv_s[1])
            A.pair_sum_backward(ctx, c_s, "soft_sphere", (), g_s, gx=gx)
            ctx.set_variant(-1)

        t_s = {"box_search": timed_graph(lambda: step_single(False), reps=10)}
        if all(m <= 1 for b in boxes_s for m in b.reach_list()[1:]):
            t_s["recorded_masks"] = timed_graph(lambda: step_single(True), reps=10)
        m_s = min(t_s.values())
        c_s.close()
        ctx.sync()
        extra["batch_512_systems"] = {"ms": m5, "particles": int(x5.shape[0]), "pairs": p5,
                                      "cell_scale_factor": f5, "build_shape_keys_per_thread_bucket_bits_shuffle": list(shape5),
                                      "pairs_per_s": p5 / (m5 * 1e-3), "step_forms_ms": t5,
                                      "single_cube_same_step": {"ms": m_s, "pairs": pairs,
                                                                "pairs_per_s": pairs / (m_s * 1e-3),
                                                                "cell_scale_factor": f_s,
                                                                "search_reach": boxes_s[0].reach_list(),
                                                                "step_forms_ms": t_s},
                                      "ratio_to_single_cube": (p5 / m5) / (pairs / m_s)}
        # the Section 3 example: N = 2^20 in the periodic unit square, r = sqrt(3/N), c = 1e-3, dt = 1,
        # float64; a step is a cell rebuild, the exp-force sum and the Euler update; 10 steps per graph
        w6 = syn.md_paper()
        s6 = w6.systems[0]
        box6 = A.BoxSpec(2, s6.lo, s6.hi, s6.periodic, s6.cutoff)
        x6 = torch.from_numpy(s6.x).to(dev)
        shape6 = A.autotune_build(ctx, x6, [box6])
        v6 = torch.from_numpy(w6.extra["v"]).to(dev)
        f6 = torch.empty_like(x6)
        c6 = A.build_cells(ctx, x6, [box6])
        p6 = int(A.pair_sum(ctx, c6, "count", ()).sum().item())
        A.autotune(ctx, c6, "exp_force", w6.params)

        def md_steps(k=10):
            for _ in range(k):
                A.build_cells(ctx, x6, [box6], cells=c6)
                A.pair_sum(ctx, c6, "exp_force", w6.params, y=f6)
                A.integrate(ctx, c6, w6.extra["dt"], f6, x6, v6)

        def md_steps_fused(k=10):
            for _ in range(k):
                A.build_cells(ctx, x6, [box6], cells=c6)
                A.md_step(ctx, c6, "exp_force", w6.params, w6.extra["dt"], x6, v6)

        x6b, v6b = torch.empty_like(x6), torch.empty_like(v6)

        def md_steps_cell_ordered(k=10):
            # the reordering container: each step writes the new positions and velocities
            # in the new cell order (ping-pong buffers; k is even, so they end where they began)
            bufs = [(x6, v6), (x6b, v6b)]
            for i in range(k):
                (xa, va), (xb, vb) = bufs[i % 2], bufs[(i + 1) % 2]
                A.build_cells(ctx, xa, [box6], cells=c6)
                A.md_step(ctx, c6, "exp_force", w6.params, w6.extra["dt"], None, va, xb, vb)

        x6_0, v6_0 = x6.clone(), v6.clone()
        forms6 = {}
        for name6, fn6 in (("force_sum_then_integrate", md_steps), ("fused_step", md_steps_fused),
                           ("cell_ordered_fused_step", md_steps_cell_ordered)):
            x6.copy_(x6_0)
            v6.copy_(v6_0)
            forms6[name6] = timed_graph(fn6, reps=5) / 10
        x6.copy_(x6_0)
        v6.copy_(v6_0)
        t_build6 = timed_graph(lambda: A.build_cells(ctx, x6, [box6], cells=c6), reps=10)
        A.cells_reorder(ctx, c6, x6, v6)  # the same positions in cell order
        t_build6_sorted = timed_graph(lambda: A.build_cells(ctx, x6, [box6], cells=c6), reps=10)
        t6 = min(forms6.values())
        ctx.sync()
        extra["md_paper_n1048576_d2_f64"] = {"ms_per_step": t6, "steps_per_s": 1e3 / t6, "pairs": p6,
                                             "pairs_per_s": p6 / (t6 * 1e-3),
                                             "particle_updates_per_s": s6.n / (t6 * 1e-3),
                                             "step_forms_ms": forms6,
                                             "build_ms_random_order": t_build6,
                                             "build_shape_keys_per_thread_bucket_bits_shuffle": list(shape6),
                                             "build_ms_cell_order": t_build6_sorted}
        # the small correctness workload (N = 1000, d = 2, periodic unit square, r = 0.1, spring, float64):
        # build + forward + adjoint as a graph, with the tuned box search and with the single-cell
        # build and all-pairs sums (the small-N switch)
        w1 = syn.md_square()
        s1 = w1.systems[0]
        x1 = torch.from_numpy(s1.x).to(dev)
        gy1 = torch.from_numpy(syn.SplitMix64(3).normal(s1.n * 2).reshape(s1.n, 2)).to(dev)
        y1 = torch.empty((s1.n, 2), dtype=torch.float64, device=dev)
        gx1 = torch.empty_like(y1)
        forms1 = {}
        for form, ncell in (("box_search", None), ("all_pairs", [1, 1])):
            box1 = A.BoxSpec(2, s1.lo, s1.hi, s1.periodic, s1.cutoff, ncell)
            c1 = A.build_cells(ctx, x1, [box1])
            v1 = (A.autotune(ctx, c1, "spring", (1.0,)), A.autotune(ctx, c1, "spring", (1.0,), gy=gy1))

            def step1():
                A.build_cells(ctx, x1, [box1], cells=c1)
                ctx.set_variant(v1[0])
                A.pair_sum(ctx, c1, "spring", (1.0,), y=y1)
                ctx.set_variant(v1[1])
                A.pair_sum_backward(ctx, c1, "spring", (1.0,), gy1, gx=gx1)
                ctx.set_variant(-1)

            forms1[form] = {"ms": timed_graph(step1, reps=20), "variants": [A.variant_name(v) for v in v1]}
        p1 = int(A.pair_sum(ctx, c1, "count", ()).sum().item())
        m1 = min(f["ms"] for f in forms1.values())
        extra["md_square_n1000_d2_f64"] = {"ms": m1, "pairs": p1, "pairs_per_s": p1 / (m1 * 1e-3),
                                           "step_forms": forms1}
        log("extra", json.dumps(extra))

    # ---------------- CPU baseline: the oracle on the host ----------------
    # The oracle as it is (cell ids, counting sort, then the linked-list cell search of the
    # spring forward and its adjoint in float64, no tolerance scales), median of three runs:
    # on every core this process may use over the full cube, and on one core over every
    # sixteenth row (the cell ids, sort and linked lists still cover all particles).  The
    # value is the all-core rate; the pairs of the sampled rows come from the oracle itself.
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        g = oracle.grid_of(s)
        gy_h = w.extra["gy"].astype(np.float64)
        x64 = s.x.astype(np.float64)
        ncores = len(os.sched_getaffinity(0))

        def oracle_rate(nthreads, rows, runs=3):
            npairs = int(oracle.pair_sum(g, "count", (), x64, rows=rows, scales=False, nthreads="all").sum())
            times = []
            for _ in range(runs):
                c0 = time.perf_counter()
                ids, _ = oracle.cell_ids(g, x64)
                oracle.sort_cells(g, ids)
                oracle.pair_sum(g, "spring", (1.0,), x64, rows=rows, scales=False, nthreads=nthreads)
                oracle.pair_sum_backward(g, "spring", (1.0,), x64, gy_h, rows=rows, scales=False,
                                         nthreads=nthreads)
                times.append(time.perf_counter() - c0)
            tc = float(np.median(times))
            return npairs / tc, tc, npairs

        v_all, t_all, p_all = oracle_rate(ncores, None)
        rows1 = np.arange(0, n, 16, dtype=np.int64)
        v_one, t_one, p_one = oracle_rate(1, rows1)
        cpu = {"value": v_all, "unit": "pair interactions/s", "cores": ncores, "kind": "oracle",
               "sample": "full spring cube (N=2^20, %d pairs): cell ids + counting sort + linked-list spring "
                         "forward + adjoint in float64, rows split over %d threads, median of 3 runs (%.2f s "
                         "each)" % (p_all, ncores, t_all),
               "single_core": {"value": v_one, "unit": "pair interactions/s", "cores": 1,
                               "sample": "every 16th row of the cube (%d rows, %d pairs), the cell ids, sort and "
                                         "linked lists over all particles, one thread, median of 3 runs (%.2f s "
                                         "each)" % (rows1.size, p_one, t_one)}}
        log("cpu baseline", json.dumps(cpu))

    out = {"metric": METRIC, "value": value, "unit": "pair interactions/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": w.name, "n": n, "box_side": float(s.hi[0]), "cutoff": 1.0,
                      "pairs_per_step": pairs,
                      "search_reach": reach,
                      "step": {"neighbour_list": "cell rebuild + neighbour-list recording + spring forward + "
                                                 "adjoint (replayed), one hipGraph",
                               "recorded_masks": "cell rebuild + spring forward (box search, recording each "
                                                 "row's accepted candidates) + adjoint (replaying them), "
                                                 "one hipGraph",
                               "box_search": "cell rebuild + spring forward + adjoint (box search), "
                                             "one hipGraph"}[mode],
                      "parallelism": "single GPU"},
           "roofline": roofline, "cpu_baseline": cpu, "breakdown": breakdown, "other_workloads": extra}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
