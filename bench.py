"""Benchmark: points/sec of the full FMM data-structure build on one MI355X.

One step = one fmmds_build (keys, sort, permutation, tables of every level,
E2 and E4 lists of levels 2..depth, for both point sets) from inputs already
resident in HBM, followed by fmmds_free. Default workload: two independent
uniform sets of 2^24 points, max level 8, 64-bit keys.

Prints ONE JSON line on stdout; progress and the per-kernel breakdown go to
stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points/sec full FMM data-structure build at N=M=2^24; batched builds/sec vs plain"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    from paper_1301_1704_amd import inputs as I
    if name == "uniform":
        return I.config_plain_uniform()
    if name == "nonuniform":
        return I.config_plain_nonuniform()
    if name == "small":
        return I.config_plain_small()
    raise SystemExit(f"unknown workload {name}")


TRAFFIC_FILES = {"uniform": "hbm_traffic_uniform_2x2p24_L8.md",
                 "nonuniform": "hbm_traffic_nonuniform_2x2p24_L10_s64.md"}


def counter_traffic(workload_name: str, kernel_class: str):
    """HBM bytes per launch of one kernel class from the committed counter
    summary (rocprofv3 FETCH_SIZE + WRITE_SIZE, already scaled by a copy of
    known size), or None when there is none or the kernel's source file has
    changed since the counters were taken."""
    name = TRAFFIC_FILES.get(workload_name)
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    for ln in open(path):
        parts = ln.split()
        if len(parts) < 2 or parts[0] != "traffic" or parts[1] != kernel_class:
            continue
        kv = dict(p.split("=", 1) for p in parts[2:])
        src = os.path.join(ROOT, kv["source"])
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv["sha"]:
            return None
        return {"read": float(kv["read_bytes_avg"]), "write": float(kv["write_bytes_avg"]),
                "source": name}
    return None


KERNEL_CLASS = [  # rocprofv3 kernel name (namespace and arguments stripped) -> class
    ("k_list_fill", "list_fill"), ("k_list_count", "list_count"),
    ("k_scan_counts2", "scan_counts"), ("k_sort_pass", "sort_pass"), ("k_keygen", "keygen"),
    ("k_digit_offsets", "digit_offsets"), ("k_zero", "zero"), ("k_leaf", "leaf"),
    ("k_level", "level"), ("k_max_occupancy", "max_occupancy"), ("k_tab_count", "tab_count"),
    ("k_tab_scan", "tab_scan"), ("k_tab_write", "leaf"), ("k_tab_masks", "level"),
    ("k_pack_sources", "near_pack"), ("k_near_field", "near_sparse"),
    ("k_near_dense", "near_dense")]
KERNEL_SOURCE = {"list_fill": "lists.hip", "list_count": "lists.hip", "scan_counts": "lists.hip",
                 "sort_pass": "sort.hip", "keygen": "sort.hip", "digit_offsets": "sort.hip",
                 "zero": "sort.hip", "leaf": "tables.hip", "level": "tables.hip",
                 "max_occupancy": "tables.hip", "tab_count": "tables.hip", "tab_scan": "tables.hip",
                 "near_pack": "nearfield.hip", "near_sparse": "nearfield.hip",
                 "near_dense": "nearfield.hip"}
COUNTER_ARGS = ("--steps 2 --warmup 1 --no-cpu-baseline --no-batch --no-serving --no-rebuild "
                "--no-dense --no-nonuniform --no-profile --copy-calibration")


def _short_name(name: str):
    """Kernel name without its argument list (and without an anonymous
    namespace, whose parentheses would cut it short)."""
    return name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").strip()


def _kernel_class(name: str):
    base = _short_name(name).replace("fmmds::", "")
    for pat, cls in KERNEL_CLASS:
        if base == pat or base.split("<")[0] == pat:
            return cls
    return None


def counter_summary(fetch_csv: str, write_csv: str, out: str, workload_name: str):
    """Writes the per-kernel HBM traffic summary (profiles/) from two rocprofv3
    --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch),
    each scaled by what the counter reads for the 1 GiB copy that
    --copy-calibration runs first."""
    import csv
    from collections import defaultdict

    def load(path, counter):
        per, copy = defaultdict(list), []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if r["Kernel_Name"].startswith("__amd_rocclr_copyBuffer"):
                copy.append(v)
            cls = _kernel_class(r["Kernel_Name"])
            if cls:
                per[cls].append(v)
        return per, max(copy)

    f, fcopy = load(fetch_csv, "FETCH_SIZE")
    w, wcopy = load(write_csv, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    fs, ws = gib_kib / fcopy, gib_kib / wcopy
    cmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc {c} --output-format csv -d <dir> -o run"
           " -- python3 <repo>/bench.py --workload " + workload_name + " " + COUNTER_ARGS)
    lines = [f"# HBM traffic per dispatch, workload `{workload_name}` (rocprofv3 FETCH_SIZE / WRITE_SIZE)",
             "", "Counters were collected in two runs of their own:", "", "```",
             cmd.format(c="FETCH_SIZE"), cmd.format(c="WRITE_SIZE"),
             f"python3 bench.py --counter-summary <fetch dir>/run_counter_collection.csv "
             f"<write dir>/run_counter_collection.csv {os.path.relpath(out, ROOT)} "
             f"--workload {workload_name}", "```", "",
             f"Calibration: the 1 GiB device-to-device copy run first reads as FETCH_SIZE "
             f"{fcopy:.0f} KiB and WRITE_SIZE {wcopy:.0f} KiB, so reads are scaled by {fs:.3f} "
             f"and writes by {ws:.3f}.", "",
             "| kernel class | dispatches | read MB / dispatch | write MB / dispatch | source |",
             "|---|---:|---:|---:|---|"]
    data = []
    for cls in sorted(f):
        fv = [x * fs * 1024 for x in f[cls]]
        wv = [x * ws * 1024 for x in w.get(cls, [0.0])]
        src = "paper_1301_1704_amd/csrc/" + KERNEL_SOURCE[cls]
        sha = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()[:16]
        rb, wb = sum(fv) / len(fv), sum(wv) / len(wv)
        lines.append(f"| {cls} | {len(fv)} | {rb / 1e6:.1f} | {wb / 1e6:.1f} | {src} |")
        data.append(f"traffic {cls} read_bytes_avg={rb:.0f} write_bytes_avg={wb:.0f} "
                    f"dispatches={len(fv)} source={src} sha={sha}")
    lines += ["", "Averages over every dispatch of the runs (all builds have the same shape). "
              "Lines read by bench.py (`sha` = the kernel source the counters were taken "
              "with; bench.py reports no traffic once it differs):", "", "```"] + data + ["```"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


BUILD_ONLY_FLAGS = "--no-cpu-baseline --no-batch --no-serving --no-rebuild --no-dense --no-nonuniform"


def kernel_stats_summary(stats_csv: str, out: str, workload_name: str, flags=None):
    """Writes the per-kernel timing summary (profiles/) from the
    run_kernel_stats.csv of a rocprofv3 --kernel-trace --stats run of this
    script. `flags`: the options of the profiled run when it was not the
    plain build alone."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    cmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
           "-d <dir> -o run -- python3 <repo>/bench.py --workload " + workload_name + " " +
           (flags or BUILD_ONLY_FLAGS))
    again = (f"python3 bench.py --kernel-stats-summary <dir>/run_kernel_stats.csv "
             f"{os.path.relpath(out, ROOT)} --workload {workload_name}")
    if flags:
        again += f" --profiled-flags '{flags}'"
        note = ("Every dispatch of the run: the plain builds (warm-up and timed, and those "
                "other measurements compare against) and every measurement the options above "
                "leave on. Averages are per dispatch.")
    else:
        note = ("Every dispatch of the run (calibration, warm-up and timed builds alike; all have "
                "the same shape). Averages are per dispatch, over every level of both point sets. "
                "The source and receiver chains of a build run on two streams until the lists, so "
                "the front kernels' durations include time shared with the other chain.")
    lines = [f"# Kernel times (rocprofv3 --kernel-trace --stats), workload `{workload_name}`", "",
             "```", cmd, again, "```", "", note, "",
             "| kernel | calls | avg (us) | min (us) | max (us) | share |",
             "|---|---:|---:|---:|---:|---:|"]
    by_class = {}
    for r in rows:
        short = _short_name(r["Name"])
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f}% |")
        cls = None if flags else _kernel_class(r["Name"])
        if cls:
            c = by_class.setdefault(cls, [0, 0.0])
            c[0] += int(r["Calls"])
            c[1] += float(r["TotalDurationNs"]) / 1e3
    if by_class:
        lines += ["", "Per kernel class (the classes `bench.py` times with HIP events; template "
                  "instances of one kernel together):", "",
                  "| class | calls | avg (us) |", "|---|---:|---:|"]
    for cls, (calls, tot) in sorted(by_class.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| `{cls}` | {calls} | {tot / calls:.1f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cpu_model() -> str:
    """CPU model name of this host (/proc/cpuinfo)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def host_cores() -> int:
    """Cores this process may use (the GPU machine gives one GPU 16 of them)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class _Pinned:
    """Runs the enclosed work on one core (sched_setaffinity), then restores
    the previous affinity."""

    def __enter__(self):
        self.prev = os.sched_getaffinity(0)
        self.core = min(self.prev)
        os.sched_setaffinity(0, {self.core})
        return self

    def __exit__(self, *a):
        os.sched_setaffinity(0, self.prev)


def cpu_baseline(c, list_share: int = 16):
    """The oracle, single-threaded and pinned to one core, on the benchmark's
    own inputs: its tables of both sets whole (keys, sort, bookmarks, parents
    and children of every level), and its E2 / E4 lists for one receiver box
    in `list_share` of every level (evenly spaced ranges), scaled to all boxes.
    Runs before the process first touches the GPU. The points/s figure is
    (N + M) over the estimated whole-build time."""
    import oracle
    oracle.lib()
    src, recv = c["src"], c["recv"]
    n_pts = src.shape[0] + (0 if recv is None else recv.shape[0])
    with _Pinned() as pin:
        t0 = time.perf_counter()
        o = oracle.OracleTree(src, recv, key_bits=c["key_bits"], cluster_s=c["cluster_s"],
                              max_level=c["max_level"], with_lists=False)
        t_tables = time.perf_counter() - t0
        t_lists, boxes, sampled = 0.0, 0, 0
        for l in range(2, o.depth + 1):
            nr = o.n_boxes(1, l)
            t1 = time.perf_counter()
            lk = o.lookup(l)
            if nr < 64 * list_share:
                ranges = [(0, nr)]
            else:  # 64 ranges, together one box in list_share
                step, width = nr // 64, max(1, nr // (64 * list_share))
                ranges = [(k * step, k * step + width) for k in range(64)]
            for r0, r1 in ranges:
                for kind in (2, 4):
                    lk.range(kind, r0, r1)
            lk.close()
            dt = time.perf_counter() - t1
            part = sum(r1 - r0 for r0, r1 in ranges)
            t_lists += dt * nr / part
            boxes += nr
            sampled += part
        o.close()
    est = t_tables + t_lists
    return {"value": n_pts / est, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": (f"the benchmark's own inputs ({c['name']}): oracle tables of both sets "
                       f"whole ({t_tables:.1f} s), E2/E4 lists of {sampled} of {boxes} receiver "
                       f"boxes (levels 2..{o.depth}, 64 evenly spaced ranges per level) scaled "
                       f"to all boxes ({t_lists:.1f} s estimated)"),
            "seconds_estimated_build": round(est, 3), "seconds_run": round(time.perf_counter() - t0, 3),
            "pinned_core": pin.core, "cpu": cpu_model(), "host_nproc": os.cpu_count()}


def _oracle_sets(job):
    """Oracle builds (tables and lists) of a share of the batch's sets; runs in
    a worker process."""
    import oracle
    xyz, off, lev, idx = job
    t0 = time.perf_counter()
    for i in idx:
        oracle.OracleTree(xyz[int(off[i]):int(off[i + 1])], None, key_bits=64,
                          max_level=int(lev[i]), with_lists=True).close()
    return time.perf_counter() - t0


def cpu_baseline_batched(xyz, off, lev):
    """The oracle over the batched workload's 512 sets, one worker process
    per host core (forked before the process touches the GPU), sets dealt
    largest first to the least loaded worker."""
    import multiprocessing as mp
    import oracle
    oracle.lib()
    cores = host_cores()
    sizes = np.diff(off.astype(np.int64))
    shares = [[] for _ in range(cores)]
    load = [0] * cores
    for i in np.argsort(-sizes):
        k = int(np.argmin(load))
        shares[k].append(int(i))
        load[k] += int(sizes[i])
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        busy = pool.map(_oracle_sets, [(xyz, off, lev, sh) for sh in shares])
    wall = time.perf_counter() - t0
    return {"value": len(lev) / wall, "unit": "builds/s", "cores": cores, "kind": "oracle",
            "sample": f"all {len(lev)} sets of the batched workload, tables and lists",
            "seconds": round(wall, 3), "core_seconds": round(sum(busy), 3), "cpu": cpu_model()}


def bench_batched(F, torch, args, sets):
    """Builds/sec of the batched form (512 sets of 2^10..2^20 points, one
    graph-replayed launch sequence) against the same 512 sets built one by
    one with fmmds_build on the same GPU and stream."""
    xyz, off, lev = sets
    x = torch.from_numpy(xyz).cuda()
    n_sets = len(lev)
    b = F.Batch(off, lev)
    for _ in range(2):  # capture (with tile autotuning), then a replay
        b.launch(x, capture=True)
        b.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        b.launch(x, capture=True)
        b.wait()
    dt_batch = (time.perf_counter() - t0) / args.batch_steps
    items = b.sort_items
    b.free()
    sets = [x[int(off[i]):int(off[i + 1])] for i in range(n_sets)]
    for i in range(0, n_sets, 16):  # warm the plain path (code, cache)
        F.build(sets[i], None, max_level=int(lev[i]), key_bits=64).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_sets):
        F.build(sets[i], None, max_level=int(lev[i]), key_bits=64).free()
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    res = {"workload": f"{n_sets} shared sets, 2^10..2^20 points (log-uniform), levels "
                       f"{int(lev.min())}..{int(lev.max())}, uniform/clustered alternating",
           "points": int(off[-1]), "sets": n_sets, "ms_per_batch": dt_batch * 1e3,
           "builds_per_s": n_sets / dt_batch, "points_per_s": int(off[-1]) / dt_batch,
           "plain_ms_all_sets": dt_plain * 1e3, "plain_builds_per_s": n_sets / dt_plain,
           "speedup_vs_plain": dt_plain / dt_batch, "graph": True, "sort_items": items}
    log(f"batched: {res['ms_per_batch']:.2f} ms per 512-set batch "
        f"({res['builds_per_s']:.0f} builds/s) vs plain {res['plain_ms_all_sets']:.1f} ms "
        f"({res['plain_builds_per_s']:.0f} builds/s)")
    return res


def bench_box_types(F, torch, src, recv, kw, n_ranks=64, l_par=4):
    """Source box types (Section 3.1) of every rank of a simulated partition
    (Section 3.2) of the benchmark build: fmmds_partition once, then
    fmmds_box_types for each of the ranks; the tree is built beforehand and
    stays resident."""
    t = F.build(src, recv, **kw)
    torch.cuda.synchronize()
    owner = t.partition(l_par, n_ranks)
    out, sizes = t.box_types(l_par, owner, 0)  # warm-up
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    owner = t.partition(l_par, n_ranks)
    e1.record()
    counts = []
    for r in range(n_ranks):
        out, _ = t.box_types(l_par, owner, r)
        if r in (0, n_ranks // 2):
            counts.append(out)
    e2.record()
    torch.cuda.synchronize()
    part_ms, all_ms = e0.elapsed_time(e1), e1.elapsed_time(e2)
    names = ["domestic", "export", "import", "root", "other"]
    c0 = torch.bincount(counts[0][:sum(sizes)].to(torch.int64), minlength=5).tolist()
    boxes = sum(sizes)
    t.free()
    res = {"workload": f"partition level {l_par}, {n_ranks} ranks, source boxes of levels "
                       f"2..{len(sizes) + 1} of the benchmark build",
           "ranks": n_ranks, "l_par": l_par, "source_boxes": boxes,
           "partition_ms": part_ms, "ms_all_ranks": all_ms, "ms_per_rank": all_ms / n_ranks,
           "box_types_per_s": boxes * n_ranks / (all_ms * 1e-3),
           "rank0_counts": dict(zip(names, c0))}
    log(f"box types: {all_ms / n_ranks:.3f} ms per rank ({n_ranks} ranks, l_par {l_par}), "
        f"partition {part_ms:.3f} ms; rank 0: {res['rank0_counts']}")
    return res


def bench_second_workload(F, torch, args):
    """The sphere + clusters workload (2 x 2^24 points, max level 10, cluster
    size 64) measured beside the default one: build rate over the same
    number of timed steps, and its near-field sum."""
    c = workload("nonuniform")
    src = torch.from_numpy(c["src"]).cuda()
    recv = torch.from_numpy(c["recv"]).cuda()
    kw = dict(max_level=c["max_level"], key_bits=c["key_bits"], cluster_s=c["cluster_s"])
    for _ in range(args.warmup):
        F.build(src, recv, **kw).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        F.build(src, recv, **kw).free()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    t = F.build(src, recv, **kw)
    torch.cuda.synchronize()
    depth = t.depth
    t.free()
    res = {"workload": c["name"], "value": (src.shape[0] + recv.shape[0]) / dt,
           "unit": "points/s", "ms_per_step": dt * 1e3, "steps": args.steps, "depth": depth}
    log(f"{c['name']}: {dt * 1e3:.3f} ms per build, {res['value']:.3g} points/s")
    if not args.no_near_field:
        res["near_field"] = bench_near_field(F, torch, src, recv, kw)
    return res


def bench_near_field(F, torch, src, recv, kw, reps=5):
    """Near-field Laplace sum over the E2 lists of the benchmark build (one
    charge per source point): pairs per second and FP32 rate, 9 flops per
    pair (3 differences, 3 multiply-adds for r^2, rsqrt, the product, the
    sum), against the FP32 vector peak."""
    t = F.build(src, recv, **kw)
    q = torch.rand(src.shape[0], dtype=torch.float32, device="cuda") - 0.5
    torch.cuda.synchronize()
    phi, cnt = t.near_field(q, count_pairs=True)  # warm-up, and the pair count
    torch.cuda.synchronize()
    pairs = int(cnt.item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        t.near_field(q)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    t.free()
    tflops = 9.0 * pairs / (ms * 1e-3) / 1e12
    res = {"workload": "unit-cube charges in [-0.5, 0.5), receivers of the benchmark build, "
                       "finest-level E2 lists", "pairs": pairs, "ms": ms,
           "pairs_per_s": pairs / (ms * 1e-3), "tflops_fp32": tflops,
           "peak_tflops_fp32": FP32_PEAK_TFLOPS, "frac": tflops / FP32_PEAK_TFLOPS}
    log(f"near field: {ms:.3f} ms, {pairs} pairs, {res['pairs_per_s']:.3g} pairs/s, "
        f"{tflops:.2f} TFLOP/s FP32")
    return res


def bench_rebuild(F, torch, c, kw, reps=5, sigma=1e-4):
    """Rebuild after one time step: the benchmark's points moved by
    sigma * N(0, 1) per coordinate (sigma 1e-4, ~2.6% of the level-8 box
    edge), rebuilt from the previous tree in both input orders, against a
    fresh build of the same moved points."""
    from paper_1301_1704_amd import inputs as I
    src2 = I.moved_points(c["src"], 250, sigma)
    recv2 = None if c["recv"] is None else I.moved_points(c["recv"], 251, sigma)
    L = c["max_level"]
    moved = 0
    for a, b in ((c["src"], src2), (c["recv"], recv2)):
        if a is not None:
            sc = np.float32(1 << L)
            moved += int(np.any(np.floor(a * sc) != np.floor(b * sc), axis=1).sum())
    n_pts = c["src"].shape[0] + (0 if recv2 is None else recv2.shape[0])
    g_src, g_recv = torch.from_numpy(c["src"]).cuda(), None
    if c["recv"] is not None:
        g_recv = torch.from_numpy(c["recv"]).cuda()
    prev = F.build(g_src, g_recv, **kw)
    m_src = torch.from_numpy(src2).cuda()
    m_recv = None if recv2 is None else torch.from_numpy(recv2).cuda()
    perm0 = torch.from_numpy(prev.host_perm(0).astype(np.int64)).cuda()
    p_src = m_src[perm0].contiguous()
    p_recv = None
    if m_recv is not None:
        p_recv = m_recv[torch.from_numpy(prev.host_perm(1).astype(np.int64)).cuda()].contiguous()

    def timed(fn):
        fn().free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn().free()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    rk = dict(key_bits=kw["key_bits"], cluster_s=kw["cluster_s"])
    fresh = timed(lambda: F.build(m_src, m_recv, **kw))
    orig = timed(lambda: F.rebuild(prev, m_src, m_recv, **rk))
    pord = timed(lambda: F.rebuild(prev, p_src, p_recv, in_prev_order=True, **rk))
    F.profile_reset()
    F.profile_enable(True)
    F.rebuild(prev, p_src, p_recv, in_prev_order=True, **rk).free()
    torch.cuda.synchronize()
    F.profile_enable(False)
    br = F.profile_read()
    prev.free()
    res = {"workload": f"the benchmark points after one step, sigma {sigma:g} per coordinate",
           "moved_fraction": moved / n_pts, "fresh_build_ms": fresh,
           "rebuild_ms_original_order": orig, "rebuild_ms_prev_order": pord,
           "points_per_s_prev_order": n_pts / (pord * 1e-3),
           "speedup_prev_order": fresh / pord, "speedup_original_order": fresh / orig,
           "kernels_prev_order": {k: {"launches": v["launches"],
                                      "avg_us": round(1e3 * v["total_ms"] / v["launches"], 2)}
                                  for k, v in br.items()}}
    log(f"rebuild: fresh {fresh:.3f} ms, from prev (original order) {orig:.3f} ms, "
        f"(prev order) {pord:.3f} ms, {moved / n_pts:.2%} of points changed box")
    return res


def bench_dense(F, torch, src, recv, kw, reps=5):
    """The same build through the dense-histogram construction (Algorithms
    1, 3, 4 with 8^L counters per level and direct ScannedRank lookups)."""
    def timed(fn):
        fn().free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn().free()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3
    sort_ms = timed(lambda: F.build(src, recv, **kw))
    dense_ms = timed(lambda: F.build_dense(src, recv, **kw))
    F.profile_reset()
    F.profile_enable(True)
    F.build_dense(src, recv, **kw).free()
    torch.cuda.synchronize()
    F.profile_enable(False)
    br = F.profile_read()
    n_pts = src.shape[0] + (0 if recv is None else recv.shape[0])
    res = {"workload": "the benchmark build", "sort_path_ms": sort_ms, "dense_ms": dense_ms,
           "points_per_s": n_pts / (dense_ms * 1e-3), "dense_vs_sort": sort_ms / dense_ms,
           "kernels": {k: {"launches": v["launches"],
                           "avg_us": round(1e3 * v["total_ms"] / v["launches"], 2)}
                       for k, v in br.items()}}
    log(f"dense variant: {dense_ms:.3f} ms vs sort path {sort_ms:.3f} ms")
    return res


def bench_serving(F, torch, args):
    """Continuous-batching serving of rebuild requests from 64 moving particle
    systems (2^14..2^22 points, 64 Gaussian clusters): Poisson arrivals at
    0.3, 0.5, 0.7 and 0.9x the saturated one-at-a-time build rate of the same
    mix, and every request at once (saturation), each against the
    one-at-a-time loop replaying the identical arrival trace."""
    from paper_1301_1704_amd import inputs as I
    from paper_1301_1704_amd import serving as S
    log("serving: generating 64 systems")
    systems, levels = I.serving_systems()
    xs = [torch.from_numpy(p).cuda() for p in systems]
    for i in range(0, 64, 8):
        F.build(xs[i], None, max_level=levels[i], key_bits=64).free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for x, lv in zip(xs, levels):
        F.build(x, None, max_level=lv, key_bits=64).free()
    torch.cuda.synchronize()
    sat = len(xs) / (time.perf_counter() - t0)
    del xs
    n_req = args.serving_warmup + args.serving_requests
    srv = S.Server(systems, levels, n_slots=4)
    # plans and graphs of the mix made once, outside every measurement
    warm_arr, warm_pick = I.poisson_trace(4 * len(systems), 0.7 * sat, len(systems), seed=81)
    srv.run(warm_arr, warm_pick)
    sweep = []
    for frac in (0.3, 0.5, 0.7, 0.9, None):
        rate = float("inf") if frac is None else frac * sat
        arr, pick = I.poisson_trace(n_req, sat if frac is None else rate, len(systems))
        if frac is None:
            arr = np.zeros_like(arr)  # every request waiting at once
        srv.reset(keep_plans=True)
        reused0 = srv.reused
        reqs = srv.run(arr, pick)
        ours = S.latency_stats(reqs, skip=args.serving_warmup)
        batch_sizes = {}
        for r in reqs[args.serving_warmup:]:
            batch_sizes[r.launched] = batch_sizes.get(r.launched, 0) + 1
        seq = S.latency_stats(S.run_sequential(systems, levels, arr, pick),
                              skip=args.serving_warmup)
        point = {"load": "saturated" if frac is None else frac,
                 "arrival_rate_per_s": None if frac is None else rate, **ours,
                 "mean_requests_per_batch": float(np.mean(list(batch_sizes.values()))),
                 "plans_reused": srv.reused - reused0, "plans": len(srv.entries),
                 "evictions": srv.evictions, "plain_sequential": seq,
                 "p99_vs_plain": seq["p99_ms"] / ours["p99_ms"] if ours["p99_ms"] > 0 else None,
                 "builds_per_s_vs_plain": ours["builds_per_s"] / seq["builds_per_s"]}
        sweep.append(point)
        log(f"serving {point['load']}: p50 {ours['p50_ms']:.2f} ms p99 {ours['p99_ms']:.2f} ms "
            f"{ours['builds_per_s']:.0f} builds/s ({point['mean_requests_per_batch']:.2f} per "
            f"batch); one-at-a-time p50 {seq['p50_ms']:.2f} ms p99 {seq['p99_ms']:.2f} ms "
            f"{seq['builds_per_s']:.0f} builds/s")
    srv.close()
    head = next(p for p in sweep if p["load"] == 0.7)
    return {"workload": "64 systems, 2^14..2^22 points (log-uniform), 64-cluster Gaussian, "
                        "levels 3..6, N(0, 1e-3) displacement per step",
            "saturated_plain_rate_per_s": sat, "warmup_requests": args.serving_warmup,
            "slots": 4, **{k: v for k, v in head.items() if k != "load"}, "sweep": sweep}


PASSES = ("keygen", "sort_pass", "tab_count", "tab_scan", "leaf", "level", "scan_counts")


def roofline_passes(breakdown: dict, workload_name: str) -> dict:
    """The sort and compaction passes against the HBM peak: per kernel class,
    algorithmic bytes of all its launches over their summed event-measured
    durations (each kernel timed alone), and the counter traffic per launch
    when the committed counter summary matches the kernel's source."""
    out = {}
    for k in PASSES:
        b = breakdown.get(k)
        if not b or b["total_ms"] <= 0:
            continue
        achieved = b["bytes"] / (b["total_ms"] * 1e6)
        per_launch = b["bytes"] / b["launches"]
        tr = counter_traffic(workload_name, k)
        out[k] = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(achieved / HBM_PEAK_GBS, 4), "launches": b["launches"],
                  "avg_launch_us": round(1e3 * b["total_ms"] / b["launches"], 2),
                  "bytes_per_launch": round(per_launch),
                  "traffic": None if tr is None else tr["read"] + tr["write"],
                  "traffic_over_algorithmic":
                      None if tr is None else round((tr["read"] + tr["write"]) / per_launch, 3)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform", choices=["uniform", "nonuniform", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-near-field", action="store_true",
                    help="skip the near-field sum measurement")
    ap.add_argument("--no-box-types", action="store_true",
                    help="skip the partition / source box type measurement")
    ap.add_argument("--no-rebuild", action="store_true",
                    help="skip the incremental rebuild measurement")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense-histogram variant measurement")
    ap.add_argument("--no-nonuniform", action="store_true",
                    help="skip the sphere + clusters workload measured beside the uniform one")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-warmup", type=int, default=200)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device-to-device copy first (scales HBM counters)")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-kernel event timing (no roofline object)")
    ap.add_argument("--counter-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "OUT"),
                    help="write the HBM traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--kernel-stats-summary", nargs=2, metavar=("STATS_CSV", "OUT"),
                    help="write the kernel timing summary from a rocprofv3 --stats run and exit")
    ap.add_argument("--profiled-flags", default=None,
                    help="with --kernel-stats-summary: the options of the profiled run, when it "
                         "measured more than the plain build")
    args = ap.parse_args()
    if args.kernel_stats_summary:
        kernel_stats_summary(*args.kernel_stats_summary, args.workload, args.profiled_flags)
        return
    if args.counter_summary:
        counter_summary(*args.counter_summary, args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent point sets shard trivially, one set spans one GPU)", file=sys.stderr)
        sys.exit(2)

    # Host-only work first: inputs, and the oracle legs, which run before the
    # process first touches the GPU (the batched leg forks worker processes).
    c = workload(args.workload)
    log(f"workload {c['name']}: inputs generated")
    batch_sets = None
    if not args.no_batch:
        from paper_1301_1704_amd import inputs as I
        log("batched: generating 512 sets")
        batch_sets = I.batch_sets()
    cpu_line = cpu_batch = None
    if not args.no_cpu_baseline:
        log("cpu baseline: the oracle on the benchmark inputs, one pinned core")
        cpu_line = cpu_baseline(c)
        log(f"cpu baseline: {cpu_line['value']:.3g} points/s ({cpu_line['sample']})")
        if batch_sets is not None:
            log("cpu baseline: the oracle over the 512 batched sets, one process per core")
            cpu_batch = cpu_baseline_batched(*batch_sets)
            log(f"cpu baseline (batched): {cpu_batch['value']:.1f} builds/s on "
                f"{cpu_batch['cores']} cores")

    import torch
    import paper_1301_1704_amd as F

    if not os.path.exists(F.LIB_PATH):
        from paper_1301_1704_amd import _compile as hb
        hb.build()
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    src = torch.from_numpy(c["src"]).cuda()
    recv = None if c["recv"] is None else torch.from_numpy(c["recv"]).cuda()
    n_pts = src.shape[0] + (0 if recv is None else recv.shape[0])
    kw = dict(max_level=c["max_level"], key_bits=c["key_bits"], cluster_s=c["cluster_s"])

    t = F.build(src, recv, **kw)
    torch.cuda.synchronize()
    info = {"depth": t.depth,
            "src_boxes_finest": t.n_boxes(0, t.depth),
            "recv_boxes_finest": t.n_boxes(1, t.depth),
            "e2_entries": int(sum(t.neighbors(l)[3] for l in range(2, t.depth + 1))),
            "e4_entries": int(sum(t.interactions(l)[3] for l in range(2, t.depth + 1)))}
    t.free()
    for _ in range(args.warmup):
        F.build(src, recv, **kw).free()
    torch.cuda.synchronize()

    profile = not args.no_profile
    breakdown, dominant = {}, None
    if profile:
        # Untimed calibration: every kernel timed, alone (the receivers' chain
        # on the build stream too), to find the dominant kernel and the
        # sort / compaction passes' own rates.
        F.profile_reset()
        F.profile_enable(True, serial=True)
        for _ in range(2):
            F.build(src, recv, **kw).free()
        torch.cuda.synchronize()
        F.profile_enable(False)
        breakdown = F.profile_read()
        dominant = max(breakdown.items(), key=lambda kv: kv[1]["total_ms"])[0]
        total = sum(v["total_ms"] for v in breakdown.values())
        log(f"{'kernel':16s} {'launches':>8s} {'avg_us':>10s} {'share':>6s} {'GB/s':>8s}")
        for k, v in sorted(breakdown.items(), key=lambda kv: -kv[1]["total_ms"]):
            log(f"{k:16s} {v['launches']:8d} {1e3 * v['total_ms'] / v['launches']:10.1f} "
                f"{v['total_ms'] / total:6.1%} {v['bytes'] / (v['total_ms'] * 1e6):8.1f}")
        # The timed region carries events around the dominant kernel only.
        F.profile_reset()
        F.profile_enable(True, dominant)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        F.build(src, recv, **kw).free()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    if profile:
        F.profile_enable(False)
        stats = F.profile_read()
    value = n_pts / dt

    line = {"metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u64", "data": "synthetic",
            "config": {"workload": c["name"], "n_src": int(src.shape[0]),
                       "n_recv": int(src.shape[0] if recv is None else recv.shape[0]),
                       "max_level": c["max_level"], "key_bits": c["key_bits"],
                       "cluster_s": c["cluster_s"], **info}}
    if profile and stats.get(dominant):
        v = stats[dominant]
        per_launch = v["bytes"] / v["launches"]
        avg_ms = v["total_ms"] / v["launches"]
        achieved = per_launch / (avg_ms * 1e6)
        total = sum(b["total_ms"] for b in breakdown.values())
        tr = counter_traffic(args.workload, dominant)
        line["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                            "traffic": None if tr is None else tr["read"] + tr["write"],
                            "kernel": dominant, "launches": v["launches"],
                            "avg_launch_us": avg_ms * 1e3, "bytes_per_launch": per_launch,
                            "kernel_time_share": breakdown[dominant]["total_ms"] / total}
        if tr is not None:
            line["roofline"]["traffic_detail"] = {
                "read_bytes": tr["read"], "write_bytes": tr["write"],
                "over_algorithmic": (tr["read"] + tr["write"]) / per_launch,
                "counters": "profiles/" + tr["source"]}
        line["roofline_passes"] = roofline_passes(breakdown, args.workload)
        line["kernels"] = {k: {"launches": b["launches"],
                               "avg_us": round(1e3 * b["total_ms"] / b["launches"], 2),
                               "GBps": round(b["bytes"] / (b["total_ms"] * 1e6), 1)}
                           for k, b in breakdown.items()}
    if not args.no_near_field:
        line["near_field"] = bench_near_field(F, torch, src, recv, kw)
    if not args.no_box_types and args.workload != "small":
        line["box_types"] = bench_box_types(F, torch, src, recv, kw)
    if not args.no_rebuild:
        line["rebuild"] = bench_rebuild(F, torch, c, kw)
    if not args.no_dense and c["max_level"] <= 8:
        line["dense"] = bench_dense(F, torch, src, recv, kw)
    if not args.no_nonuniform and args.workload == "uniform":
        line["nonuniform"] = bench_second_workload(F, torch, args)
    if not args.no_batch:
        line["batched"] = bench_batched(F, torch, args, batch_sets)
        if cpu_batch is not None:
            line["batched"]["cpu_baseline"] = cpu_batch
    if not args.no_serving:
        line["serving"] = bench_serving(F, torch, args)
    if cpu_line is not None:
        line["cpu_baseline"] = cpu_line
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
