"""Benchmark of the directed triad census on one MI355X.

One step = one full census of the workload through the C ABI (validation and
packing, task enumeration and scheduling, the merge/classify kernel, the null
count), with the graph already resident in HBM. Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat24]
                    [--schedule plain|heuristic|learned] [--no-cpu-baseline]
                    [--copy-calibration]   # plain copy kernel for counter scaling

Metric: edge-pairs merged per second (an edge-pair is one task (u,v), u < v,
over a symmetric edge).

Roofline of the census kernel: it is bound by vector-instruction issue, not by
HBM (its DRAM traffic is about a third of the HBM peak). `roofline` therefore
reports the vector unit: achieved = SQ_INSTS_VALU per launch (rocprofv3 counter,
profiles/counters_k_census_<workload>.json, valid while the kernel source hash
matches) x 64 lanes / the kernel's live duration, against the issue peak of
256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.32e12 32-bit lane-operations/s (a
wave64 vector instruction occupies a 16-lane SIMD for 4 cycles).
Beside it, `roofline.hbm` gives the algorithmic-byte figures: the metric's own
B_full = sum over tasks of 4.25*(d(u)+d(v)) + 32 (whole lists; 4-byte id and a
quarter byte of direction flags per entry, plus the two offset pairs), the
bytes of the merge as the kernel runs it, B_trim = 4.25 * (sum_x d+(x)^2 +
sum_x (d(x) d-(x) - d-(x)(d-(x)-1)/2)) + 32 * m_sym (N(u) above u, d+(u) ids,
and N(v) from u on, d(v) - i ids when u is the i-th lowest neighbour of v;
d-(x) = d(x) - d+(x) the neighbours below x), each over the kernel time and
the 8 TB/s peak, and the measured DRAM bytes (FETCH_SIZE + WRITE_SIZE scaled
by a plain copy) over the same peak.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
# vector issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (32-bit lane-ops/s, in T)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOAD_TEXT = {
    "rmat24": "R-MAT scale 24 (16,777,216 vertices), edge factor 16, a/b/c/d = .57/.19/.19/.05, seed 1, "
              "self-loops and duplicate arcs removed",
    "rmat20": "R-MAT scale 20 (1,048,576 vertices), edge factor 16, a/b/c/d = .57/.19/.19/.05, seed 1, "
              "10% of asymmetric pairs reciprocated (seed 2)",
    "cl22": "Chung-Lu directed, n = 2^22, exponent 2.1, mean degree 24, max expected degree 2^18, seed 1",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(g, budget_entries=6.0e10, single_budget=4.0e9, seed=7):
    """The oracle (test infrastructure) on a bounded sample of the same
    workload's tasks, on all host cores, and on one core with a smaller
    sample; rates in edge-pairs/s."""
    import numpy as np

    import oracle
    d = np.diff(g.offsets).astype(np.int64)
    rows = np.repeat(np.arange(g.n, dtype=np.int32), d)
    tasks = np.flatnonzero(g.nbrs > rows).astype(np.int64)
    del rows
    ntasks = tasks.size
    total_entries = int(np.dot(d, d))  # sum over tasks of d(u) + d(v)

    def timed(budget, threads, salt):
        frac = min(1.0, budget / max(1, total_entries))
        stride = max(1, int(round(1.0 / frac)))
        off = int(np.random.default_rng(seed + salt).integers(0, stride))
        sample = tasks[off::stride].copy()
        t0 = time.perf_counter()
        oracle.census_tasks(g, sample, nthreads=threads)
        dt = time.perf_counter() - t0
        return sample.size / dt, (f"every {stride}th task of the {g.name} task list in CSR order (offset {off}): "
                                  f"{sample.size} of {ntasks} tasks, {dt:.1f} s wall")

    threads = max(1, len(os.sched_getaffinity(0)))
    v, text = timed(budget_entries, threads, 0)
    v1, text1 = timed(single_budget, 1, 1)
    return {"value": v, "unit": "edge-pairs/s", "cores": threads, "kind": "oracle", "sample": text,
            "single_core": {"value": v1, "unit": "edge-pairs/s", "cores": 1, "sample": text1}}


def list_byte_sums(d_off, d_nbr, n):
    """(sum_x d+(x)^2, sum_x (d(x) d-(x) - d-(x)(d-(x)-1)/2)) with d-(x) /
    d+(x) the neighbours of x below / above x: the merged list entries of all
    tasks, N(u) above u (d+(u) entries, in d+(u) tasks) and N(v) from u on (for
    the i-th lowest neighbour u of v, d(v) - i entries). Device-side
    bookkeeping, outside the timed region."""
    import torch
    counts = d_off[1:] - d_off[:-1]
    rows = torch.repeat_interleave(torch.arange(n, device=d_off.device, dtype=torch.int32), counts)
    below = torch.bincount(rows[d_nbr < rows].to(torch.int64), minlength=n).to(torch.int64)
    del rows
    above = counts - below
    return int((above * above).sum().item()), int((counts * below - below * (below - 1) // 2).sum().item())


def copy_calibration(nbytes=4 << 30, reps=3):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--schedule", default="plain", choices=["plain", "heuristic", "learned"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-schedules", action="store_true", help="skip the heuristic / learned comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched null-model ensemble comparison")
    ap.add_argument("--no-cl22", action="store_true", help="skip the schedule comparison on the Chung-Lu graph")
    ap.add_argument("--no-adjacent", action="store_true",
                    help="skip the CSR construction, incremental, labelled and significance-profile legs")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the census of one graph runs on a single MI355X; "
              "multi-GPU sharding is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration()
        return

    from paper_1209_6308_amd import graphs, triad
    t0 = time.time()
    g = graphs.workload(args.workload)
    st = g.stats()
    log(f"generated {args.workload} in {time.time() - t0:.1f}s: {st}")
    d_off, d_nbr, d_flg = triad.to_device(g, "cuda")
    stream = torch.cuda.current_stream()
    models = {}
    run = make_runner(torch, triad, g, (d_off, d_nbr, d_flg), stream, models)

    main = run(args.schedule, args.steps, args.warmup, spans=not args.no_schedules)
    counts = main["counts"]
    wall = main["wall_s"]
    ms_per_step = wall * 1e3 / args.steps
    value = st["m_sym"] * args.steps / wall
    kern_s = sum(main["census_ms"]) / len(main["census_ms"]) / 1e3
    # algorithmic bytes of one census: per task (u, v) the ids of N(u) above u
    # and of N(v) from u on, 4.25 B each (id + flag), plus 32 B of offsets
    roof = census_roofline(args.workload, kern_s, d_off, d_nbr, g.n, st)
    b_alg = roof["hbm"]["alg_bytes_trimmed"]
    rec = {
        "metric": "edge-pairs merged/s (R-MAT s24); census kernel roofline (vector issue; HBM figures beside it)",
        "value": round(value, 1),
        "unit": "edge-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "schedule": args.schedule, "n": st["n"],
                   "m_sym": st["m_sym"], "nnz": st["nnz"], "sum_d2": st["sum_d2"], "d_max": st["d_max"],
                   "content_hash": g.content_hash(), "accumulators": "u64",
                   "census": [str(x) for x in counts]},
        "roofline": roof,
    }

    if not args.no_schedules:
        sched = {args.schedule: schedule_summary(main, st["m_sym"], b_alg)}
        for other in ("plain", "heuristic", "learned"):
            if other == args.schedule:
                continue
            r = run(other, args.steps, 1, spans=True)
            if r["counts"] != counts:
                raise SystemExit(f"schedule {other} changed the census")
            sched[other] = schedule_summary(r, st["m_sym"], b_alg)
        sched["identical_counts"] = True
        if "report" in models:
            sched["cost_model"] = models["report"]
        rec["schedules"] = sched
        if args.workload != "cl22" and not args.no_cl22:
            rec["schedules_cl22"] = compare_schedules(torch, graphs, triad, "cl22", min(args.steps, 5), stream,
                                                      models)
    if not args.no_adjacent:
        rec["csr_build"] = csr_build_bench(torch, graphs, triad, args.workload, (d_off, d_nbr, d_flg))
        rec["incremental"] = incremental_bench(torch, triad, g, (d_off, d_nbr, d_flg), counts, stream)
        rec["labelled"] = labelled_bench(torch, triad, g, (d_off, d_nbr, d_flg), counts, stream,
                                         sum(main["census_ms"]) / len(main["census_ms"]))
    if not args.no_batched:
        rec["batched"] = batched_bench(torch)
    if not args.no_adjacent:
        rec["significance"] = significance_bench(torch, graphs, triad)
    if not args.no_cpu_baseline:
        log("timing the oracle on a task sample (host cores)")
        rec["cpu_baseline"] = cpu_baseline(g)
    print(json.dumps(rec), flush=True)


def make_runner(torch, triad, g, dev, stream, models):
    """run(schedule, steps, warmup, spans) -> timings and counts of repeated
    census calls on the device-resident graph `dev` = (offsets, ids, flags)."""
    d_off, d_nbr, d_flg = dev
    d_out = torch.empty(17, dtype=torch.int64, device="cuda")

    def run(schedule, steps, warmup, spans=False):
        kw = {"schedule": schedule}
        if schedule == "learned":
            if "learned" not in models:
                from paper_1209_6308_amd import costmodel
                t0 = time.time()
                models["learned"] = costmodel.load_or_train(stream=stream)
                models["report"] = costmodel.last_training_report()
                models["report"]["train_seconds"] = round(time.time() - t0, 1)
                log(f"cost model trained: {models['report']}")
            kw["model"] = models["learned"]
        for i in range(warmup):
            triad.triad_census_device(g.n, g.nnz, d_off, d_nbr, d_flg, stream=stream, d_out=d_out, **kw)
            log(f"{g.name} {schedule}: warmup {i + 1}/{warmup} done")
        torch.cuda.synchronize()
        census_ms, counts, tasks_ms = [], None, []
        t0 = time.perf_counter()
        for i in range(steps):
            counts, status, tm = triad.triad_census_device(g.n, g.nnz, d_off, d_nbr, d_flg, stream=stream,
                                                           d_out=d_out, **kw)
            census_ms.append(tm["census_ms"])
            tasks_ms.append(tm["tasks_ms"])
            log(f"{g.name} {schedule}: step {i + 1}/{steps}: census kernel {tm['census_ms']:.1f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out = {"wall_s": wall, "census_ms": census_ms, "tasks_ms": tasks_ms, "counts": counts, "waves": tm["waves"]}
        if spans:
            span = torch.zeros((tm["waves"], 2), dtype=torch.int64, device="cuda")
            triad.triad_census_device(g.n, g.nnz, d_off, d_nbr, d_flg, stream=stream, d_out=d_out, wave_span=span,
                                      **kw)
            sp = span.cpu().numpy().astype("float64")
            busy = sp[:, 1] - sp[:, 0]
            out["makespan_imbalance"] = float((sp[:, 1].max() - sp[:, 0].min()) / busy.mean() - 1.0)
            out["wave_end_spread_ms"] = float((sp[:, 1].max() - sp[:, 1].min()) / 1e5)
        return out

    return run


def schedule_summary(r, m_sym, b_alg):
    k = sum(r["census_ms"]) / len(r["census_ms"])
    d = {"edge_pairs_per_s": round(m_sym * len(r["census_ms"]) / r["wall_s"], 1),
         "census_kernel_ms": round(k, 2), "schedule_ms": round(sum(r["tasks_ms"]) / len(r["tasks_ms"]), 2),
         "hbm_frac_alg_trimmed": round(b_alg / (k / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    if "makespan_imbalance" in r:
        d["makespan_imbalance"] = round(r["makespan_imbalance"], 4)
        d["wave_end_spread_ms"] = round(r["wave_end_spread_ms"], 3)
    return d


def compare_schedules(torch, graphs, triad, name, steps, stream, models):
    """Plain / heuristic / learned census of another workload (identical counts
    required): the learned-schedule comparison on the Chung-Lu graph."""
    t0 = time.time()
    g = graphs.workload(name)
    st = g.stats()
    log(f"generated {name} in {time.time() - t0:.1f}s: {st}")
    dev = triad.to_device(g, "cuda")
    run = make_runner(torch, triad, g, dev, stream, models)
    s_above2, s_d_below = list_byte_sums(dev[0], dev[1], g.n)
    b_alg = 4.25 * (s_above2 + s_d_below) + 32.0 * st["m_sym"]
    out, counts = {"workload": WORKLOAD_TEXT[name], "m_sym": st["m_sym"], "steps": steps}, None
    for sched in ("plain", "heuristic", "learned"):
        r = run(sched, steps, 1, spans=True)
        if counts is not None and r["counts"] != counts:
            raise SystemExit(f"schedule {sched} changed the {name} census")
        counts = r["counts"]
        out[sched] = schedule_summary(r, st["m_sym"], b_alg)
    out["identical_counts"] = True
    out["census"] = [str(x) for x in counts]
    if "learned" in models:
        # the network trained on R-MAT scale 10 and 20 cycles, evaluated on this graph's
        from paper_1209_6308_amd import costmodel
        out["cost_model_held_out"] = costmodel.held_out_report(models["learned"], g, stream=stream)
        log(f"cost model on {name} (held out): {out['cost_model_held_out']}")
    return out


def csr_build_bench(torch, graphs, triad, name, dev, reps=3):
    """The CSR with direction flags built on the device from the workload's raw
    arc list (duplicates and self-loops included), against the host build the
    generator does; the result must equal the resident CSR."""
    w = graphs.WORKLOADS[name]
    if w["kind"] != "rmat" or w.get("recip_p"):
        return None
    n = 1 << w["scale"]
    t0 = time.perf_counter()
    src, dst = graphs.rmat_arcs(w["scale"], w["edge_factor"] * n, seed=w["seed"])
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    host = graphs.build_csr(n, src, dst)
    host_s = time.perf_counter() - t0
    del host
    ds, dd = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
    narcs = src.size
    del src, dst
    ms = []
    for i in range(reps):
        off, nbr, flg, t = triad.csr_from_arcs(n, ds, dd, timed=True)
        ms.append(t)
        log(f"csr build {i + 1}/{reps}: {t:.1f} ms")
    same = bool(torch.equal(off, dev[0]) and torch.equal(nbr, dev[1]) and torch.equal(flg, dev[2]))
    if not same:
        raise SystemExit("device CSR construction differs from the host build")
    del off, nbr, flg, ds, dd
    torch.cuda.empty_cache()
    best = min(ms)
    return {"workload": f"{name} raw arcs ({narcs} drawn, duplicates and self-loops included)",
            "device_ms": round(best, 2), "device_ms_all": [round(x, 2) for x in ms],
            "arcs_per_s": round(narcs / (best / 1e3), 1), "host_build_s": round(host_s, 2),
            "host_threads": graphs.nthreads(), "arc_generation_s": round(gen_s, 2),
            "speedup_vs_host": round(host_s / (best / 1e3), 1), "identical_csr": same}


def incremental_bench(torch, triad, g, dev, census, stream, batches=8, k=100000, seed=5):
    """Census of the workload under batches of arc updates (half deletions of
    present arcs, half insertions between random vertices, in order), each
    batch's census from the previous one; the last is checked against a full
    census of the final graph."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    off, nbr, flg = dev
    n, nnz = g.n, g.nnz
    ms, changed, c = [], [], census
    for b in range(batches):
        # deletions: arcs present in the CSR (an entry whose bit0 is set is the arc row -> id)
        j = torch.randint(0, nnz, (k // 2,), device="cuda", generator=gen)
        f = (flg[j >> 2].to(torch.int64) >> (2 * (j & 3))) & 3
        rows = torch.searchsorted(off, j, right=True) - 1
        cols = nbr[j].to(torch.int64)
        out_arc = (f & 1) != 0
        dsrc = torch.where(out_arc, rows, cols)
        ddst = torch.where(out_arc, cols, rows)
        isrc = torch.randint(0, n, (k - k // 2,), device="cuda", generator=gen)
        idst = (isrc + torch.randint(1, n, (k - k // 2,), device="cuda", generator=gen)) % n
        usrc = torch.cat([dsrc, isrc]).to(torch.int32)
        udst = torch.cat([ddst, idst]).to(torch.int32)
        perm = torch.randperm(k, device="cuda", generator=gen)
        usrc, udst = usrc[perm].contiguous(), udst[perm].contiguous()
        uins = torch.cat([torch.zeros(k // 2, dtype=torch.uint8, device="cuda"),
                          torch.ones(k - k // 2, dtype=torch.uint8, device="cuda")])[perm].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c, new, chg = triad.census_update(n, nnz, off, nbr, flg, c, usrc, udst, uins, stream=stream)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
        changed.append(chg)
        off, nbr, flg = new
        nnz = int(nbr.numel())
        log(f"incremental batch {b + 1}/{batches}: {ms[-1]:.1f} ms, {chg} changed pairs")
    full, _, tm = triad.triad_census_device(n, nnz, off, nbr, flg, stream=stream)
    if full != c:
        raise SystemExit("incremental census differs from the full census of the final graph")
    mean = sum(ms[1:]) / max(1, len(ms) - 1)
    return {"workload": f"{g.name}: {batches} batches of {k} arc updates (half deletions of present arcs, half "
                        f"insertions between random vertices, shuffled)",
            "batch_ms": [round(x, 2) for x in ms], "mean_batch_ms": round(mean, 2),
            "updates_per_s": round(k / (mean / 1e3), 1), "changed_pairs": changed,
            "full_census_ms_final_graph": round(tm["census_ms"] + tm["tasks_ms"] + tm["prep_ms"], 2),
            "identical_to_full_census": True}


def labelled_bench(torch, triad, g, dev, counts, stream, census16_ms, reps=2):
    """The 64-state labelled census of the workload (its states must add up to
    C(n,3); the GPU tests check that they condense to the 16-class census)."""
    ms, lab = [], None
    for i in range(reps):
        lab, st, tm = triad.labelled_census_device(g.n, g.nnz, *dev, stream=stream)
        ms.append(tm["census_ms"])
        log(f"labelled census {i + 1}/{reps}: kernel {tm['census_ms']:.1f} ms")
    return {"workload": g.name, "census_kernel_ms": round(min(ms), 2),
            "edge_pairs_per_s_kernel": round(g.nnz // 2 / (min(ms) / 1e3), 1),
            "census16_kernel_ms": round(census16_ms, 2),
            "state_sum_equals_C(n,3)": sum(lab) == g.n * (g.n - 1) * (g.n - 2) // 6,
            "states": [str(x) for x in lab]}


def significance_bench(torch, graphs, triad, scale=12, K=1024):
    """Triad significance profile of an R-MAT graph against K degree-preserving
    randomisations: one batched census of the ensemble plus the z-score kernel."""
    g = graphs.rmat(scale, 8, seed=3, recip_p=0.1)
    t0 = time.perf_counter()
    B = graphs.randomised_ensemble(g, K, seed=1)
    gen_s = time.perf_counter() - t0
    d = triad.batch_to_device(B)
    real_d = triad.to_device(g)
    real = triad.triad_census_device(g.n, g.nnz, *real_d)[0]
    out = torch.empty((B.G, 16), dtype=torch.int64, device="cuda")
    plan = triad.BatchPlan(B.G, int(B.vbase[-1]), B.nnz, *d, d_out=out)
    plan.launch()
    plan.status()
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.launch()
        z, sp = triad.significance_profile(out, real)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    plan.close()
    best = min(ts)
    m_sym = B.nnz // 2
    return {"workload": f"R-MAT scale {scale}, edge factor 8, 10% reciprocated, seed 3; {K} randomisations "
                        "(10 x arcs double-edge swap attempts each)",
            "ms": round(best * 1e3, 2), "ensemble_edge_pairs_per_s": round(m_sym / best, 1),
            "ensemble_generation_s_host": round(gen_s, 1), "z": [round(x, 4) for x in z],
            "profile": [round(x, 4) for x in sp]}


def census_roofline(workload, kern_s, d_off, d_nbr, n, st):
    """Roofline record of the census kernel (see the module docstring)."""
    s_above2, s_d_below = list_byte_sums(d_off, d_nbr, n)
    b_trim = 4.25 * (s_above2 + s_d_below) + 32.0 * st["m_sym"]
    b_full = 4.25 * st["sum_d2"] + 32.0 * st["m_sym"]
    hbm = {"peak_gbs": HBM_PEAK_GBS,
           "alg_bytes_full": b_full, "frac_alg_full": round(b_full / kern_s / 1e9 / HBM_PEAK_GBS, 4),
           "alg_bytes_trimmed": b_trim, "frac_alg_trimmed": round(b_trim / kern_s / 1e9 / HBM_PEAK_GBS, 4),
           "sum_dplus2": s_above2, "sum_d_dminus": s_d_below, "dram_bytes": None, "frac_dram": None}
    roof = {"bound": "alu", "achieved": None, "peak": round(VALU_PEAK_TOPS, 2), "unit": "Tops/s", "frac": None,
            "traffic": None, "kernel": "k_census", "kernel_ms": round(kern_s * 1e3, 2),
            "peak_basis": "vector issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, 32-bit lane-ops",
            "counters": None, "hbm": hbm}
    cfile = os.path.join(ROOT, "profiles", f"counters_k_census_{workload}.json")
    if os.path.exists(cfile):
        with open(cfile) as f:
            c = json.load(f)
        roof["counters"] = os.path.relpath(cfile, ROOT)
        if c.get("kernel_source_hash") == kernel_source_hash():
            valu = float(c["SQ_INSTS_VALU"])
            ach = valu * 64 / kern_s / 1e12
            roof["achieved"] = round(ach, 3)
            roof["frac"] = round(ach / VALU_PEAK_TOPS, 4)
            roof["valu_insts_per_launch"] = valu
            roof["salu_insts_per_launch"] = float(c["SQ_INSTS_SALU"])
            roof["lds_insts_per_launch"] = float(c["SQ_INSTS_LDS"])
            roof["traffic"] = c["hbm_bytes_per_launch"]
            hbm["dram_bytes"] = c["hbm_bytes_per_launch"]
            hbm["frac_dram"] = round(c["hbm_bytes_per_launch"] / kern_s / 1e9 / HBM_PEAK_GBS, 4)
        else:
            roof["note"] = "kernel source changed since the counters were taken"
    return roof


def batched_bench(torch, reps=3):
    """4,096 null-model graphs: one captured batched census (autotuned launch
    shape) against 4,096 single-graph census calls, same graphs, same counts."""
    from paper_1209_6308_amd import graphs, triad
    t0 = time.time()
    B = graphs.null_ensemble(4096, 1)
    nv = int(B.vbase[-1])
    m_sym = B.nnz // 2
    log(f"generated the ensemble in {time.time() - t0:.1f}s: {B.G} graphs, {nv} vertices, {m_sym} edges")
    d = triad.batch_to_device(B)
    cache = os.environ.get("TRIAD_TUNE_CACHE") or None  # a JSON-lines file of tuned launch shapes, if given
    t0 = time.time()
    best = triad.batch_autotune(B.G, nv, B.nnz, *d, cache_path=cache)
    tune_s = time.time() - t0
    log(f"autotuned batch launch shape in {tune_s:.1f}s: {best}")
    plan = triad.BatchPlan(B.G, nv, B.nnz, *d, **best)
    plan.launch()
    plan.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.launch()
    plan.status()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    batched = plan.result()
    plan.close()
    # the same graphs, one census call each (device-resident, rebased offsets)
    members = []
    for g in range(B.G):
        m = B.graph(g)
        members.append((m.n, m.nnz) + triad.to_device(m))
    out = torch.empty(17, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    for (n, nnz, a, b, c) in members:
        per.append(triad.triad_census_device(n, nnz, a, b, c, d_out=out)[0])
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    same = all([x & ((1 << 64) - 1) for x in p] == q for p, q in zip(per, batched))
    if not same:
        raise SystemExit("batched census differs from per-graph census")
    return {"workload": "4,096 degree-preserving randomisations of Erdos-Renyi / Chung-Lu digraphs, "
                        "n ~ U[64, 8192], mean out-degree ~ U[4, 32], reciprocity ~ U[0, 0.3], seed 1",
            "graphs": B.G, "vertices": nv, "m_sym": m_sym, "sum_d2": B.sum_d2(),
            "batched_edge_pairs_per_s": round(m_sym / t_batch, 1), "batched_ms": round(t_batch * 1e3, 2),
            "per_graph_edge_pairs_per_s": round(m_sym / t_single, 1), "per_graph_ms": round(t_single * 1e3, 2),
            "speedup": round(t_single / t_batch, 2), "tuned": best, "autotune_s": round(tune_s, 1),
            "identical_counts": True}


def kernel_source_hash():
    """Hash of the sources the census kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for fn in ("census.hip", "triad_internal.h"):
        with open(os.path.join(ROOT, "paper_1209_6308_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
