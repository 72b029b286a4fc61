"""Benchmark: spectra searched per second on one MI355X (plain batch,
persistent graph-captured batch, and continuous-batching serving).

Workload (default): the large open search -- 20k proteins, Met oxidation and
STY phosphorylation with at most three modified sites (40.9M peptides, 6.8G
postings in lists merging three neighbouring fragment bins, index built on the
GPU), a seeded batch of 100k spectra of the 1M-spectrum recipe (20-200 peaks,
precursor masses lognormal around 1800 Da so windows are very uneven, charges
2-3), +-500 Da windows.

One step = the whole search path (prep and precursor window, fragment-bin
posting scan, shared-peak counting, hyperscore, top-k, score histogram,
expect value, results back to the host) over the batch, with the inputs
already resident in HBM.  `value` is the faster graph-replayed form (plain or
persistent scan schedule); the other forms, the serving loop (Poisson arrivals
of 1-4096-spectrum requests with charges 2-4, p50/p99 latency, and a
saturating load) and small batches are reported beside it.

Prints ONE JSON line with the roofline figure of the dominant kernel (the
posting scan, timed with HIP events on its stream) and the CPU oracle's rate
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# LDS atomic peak of the chip: each CU's LDS serves 128 bytes per clock, i.e.
# 32 four-byte atomic lanes per clock without bank conflicts; 256 CUs at 2.4 GHz.
LDS_ATOMIC_PEAK_GOPS = 256 * 2.4 * 32


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class _DevArray:
    def __init__(self, p, n, typestr):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (p, False), "version": 2}


def device_spectra(sp, torch):
    dev = "cuda:0"
    return [torch.from_numpy(np.ascontiguousarray(sp.peak_off.astype(np.uint64).view(np.int64))).to(dev),
            torch.from_numpy(np.ascontiguousarray(sp.mz)).to(dev),
            torch.from_numpy(np.ascontiguousarray(sp.intensity)).to(dev),
            torch.from_numpy(np.ascontiguousarray(sp.precursor_mz)).to(dev),
            torch.from_numpy(np.ascontiguousarray(sp.charge)).to(dev)]


def fill_plan_inputs(plan, tens, torch):
    d = plan.inputs()
    for p, t, ts in [(d.peak_off, tens[0], "<i8"), (d.mz, tens[1], "<f4"), (d.intensity, tens[2], "<f4"),
                     (d.precursor_mz, tens[3], "<f8"), (d.charge, tens[4], "|i1")]:
        torch.as_tensor(_DevArray(p, t.numel(), ts), device="cuda").copy_(t)
    torch.cuda.synchronize()


def eager_steps(capi, engine, ix, dsp, n, nnz, prm, ws_dev, steps):
    scan_ms, res = [], None
    for _ in range(steps):
        b = C.c_void_p()
        capi.check(capi.ps_search_device(ix.handle, C.byref(ws_dev), C.byref(dsp), nnz, C.byref(prm), C.byref(b)))
        res = engine.collect(b, n, prm)
        capi.ps_batch_free(b)
        scan_ms.append(res.scan_ms)
    return scan_ms, res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads():
    """Host threads this process may use: the affinity mask, capped by
    OMP_NUM_THREADS where the environment sets the process's CPU share."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS", "")
    return min(n, int(share)) if share.isdigit() and int(share) > 0 else n


def cpu_baseline(w, prot, sp, seconds_target=20.0):
    """The oracle (unchanged) on all host threads over a seeded sample of the
    same batch, sized to about `seconds_target` of work."""
    import oracle
    threads = cpu_threads()
    t0 = time.perf_counter()
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                         oracle.mods_from_synth(w.mods), w.max_mods)
    db_s = time.perf_counter() - t0
    rng = np.random.default_rng(99)
    probe = sp.subset(np.sort(rng.choice(sp.n, min(sp.n, threads), replace=False)))
    t0 = time.perf_counter()
    db.search(probe, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared, threads=threads)
    per = (time.perf_counter() - t0) / max(probe.n, 1)
    m = int(max(threads, min(sp.n, seconds_target / max(per, 1e-6))))
    idx = np.sort(rng.choice(sp.n, m, replace=False))
    sub = sp.subset(idx)
    t0 = time.perf_counter()
    db.search(sub, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "spectra/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{m} of the {sp.n} spectra (seed 99), the whole database ({len(db)} peptides, digested and "
                      f"sorted by the oracle in {db_s:.1f} s, not timed), all {threads} host threads, {dt:.1f} s"}


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """HBM bandwidth a plain device-to-device copy reaches (bytes read + bytes
    written per second, best of `reps`): the practical ceiling beside the
    8 TB/s specification."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return 2.0 * nbytes / best / 1e9


KERNEL_SOURCE = {"k_scan_plain": "kernels.hip", "k_scan_persistent": "kernels.hip", "k_assemble": "stats.hip"}


def measured_traffic(workload_name, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload, valid only while the kernel's source file is the
    one the counters were taken on."""
    path = os.path.join(ROOT, "profiles", f"scan_{workload_name}_hbm_counters.md")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCE:
        return None
    vals = {}
    for line in open(path):
        if line.startswith("    ") and ":" in line:
            k, v = line.strip().split(":", 1)
            vals[k.strip()] = v.strip()
    src = KERNEL_SOURCE[kernel]
    now = hashlib.sha256(open(os.path.join(ROOT, "paper_2102_02286_amd", "csrc", src), "rb").read()).hexdigest()
    key = f"traffic_bytes_per_launch {kernel}"
    if vals.get(f"source_sha256 {src}") != now or key not in vals:
        return None
    return float(vals[key])


def build_index(engine, w, prot, merge, **kw):
    return engine.HostIndex.build_on_device(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                                            engine.mods_from_synth(w.mods), w.max_mods, merge_tol=merge, **kw)


def assembly_leg(capi, engine, torch, w, prot, merge, G, dsp, n, nnz, prm, ref, steps, warmup):
    """The same batch searched over G round-robin database partitions (each
    built on the GPU), one after another on this GPU, then assembled on the
    device (ps_assemble).  Times the whole partitioned step and the assembly
    kernel (HIP events on the stream it runs on) and checks that the assembled
    hits and stats equal the whole-database search bit for bit."""
    t0 = time.perf_counter()
    parts = [build_index(engine, w, prot, merge, n_shards=G, shard=g) for g in range(G)]
    torch.cuda.synchronize()
    log(f"partitions: {G} indexes of ~{len(parts[0])} peptides built on the GPU in {time.perf_counter() - t0:.1f}s")
    devs, spaces = [], []
    for p in parts:
        need = C.c_uint64()
        capi.check(capi.ps_workspace_bytes(p.handle, n, nnz, C.byref(prm), C.byref(need)))
        ws = engine.Workspace()
        devs.append(ws.get(need.value))
        spaces.append(ws)
    out = engine.AssembleOut(n, prm.top_k)
    stream = torch.cuda.current_stream()

    def searches():
        batches = []
        for p, d in zip(parts, devs):
            b = C.c_void_p()
            capi.check(capi.ps_search_device(p.handle, C.byref(d), C.byref(dsp), nnz, C.byref(prm), C.byref(b)))
            batches.append(b)
        return batches

    def step():
        batches = searches()
        pp = [engine._device_results(b) for b in batches]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        engine.assemble(pp, n, prm.top_k, out, stream, fit=prm.fit)
        e1.record(stream)
        for b in batches:
            capi.ps_batch_free(b)
        e1.synchronize()
        return e0.elapsed_time(e1)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    asm_ms = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hits, stats, _ = out.to_host()
    same = hits.tobytes() == ref.hits.tobytes() and stats.tobytes() == ref.stats.tobytes()
    assert same, "assembled partition results differ from the whole-database search"
    per_spec = (capi.PS_HIST_BINS * 4 + prm.top_k * capi.HIT_DTYPE.itemsize + capi.STAT_DTYPE.itemsize)
    alg_bytes = float(n) * (G + 1) * per_spec
    ms = float(np.mean(asm_ms))
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    res = {"shards": G, "spectra_per_s": n * steps / dt, "ms_per_step": dt * 1e3 / steps,
           "assemble_ms": ms, "identical_to_whole": bool(same),
           "roofline": {"bound": "hbm", "kernel": "k_assemble", "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": measured_traffic(w.name, "k_assemble") if G == 4 else None,
                        "bytes_per_launch": alg_bytes}}
    log(f"partitions: {res['spectra_per_s']:.0f} spectra/s over {G} partitions ({res['ms_per_step']:.1f} ms/step); "
        f"assembly {ms:.3f} ms = {achieved:.0f} GB/s of {alg_bytes / 1e9:.2f} GB")

    # the same partition results exchanged as 256-byte samples (ps_sample, then
    # ps_assemble shifting each sample into place), under both expect-value fits
    recs = [torch.empty(n * capi.SAMPLED_DTYPE.itemsize, dtype=torch.uint8, device="cuda") for _ in range(G)]
    res["sampled"] = {}
    for fit_name, fit in (("tail", capi.PS_FIT_TAIL), ("gumbel", capi.PS_FIT_GUMBEL)):
        prm_f = capi.ps_search_params.from_buffer_copy(prm)
        prm_f.fit = fit
        out_full, out_s = engine.AssembleOut(n, prm.top_k), engine.AssembleOut(n, prm.top_k)
        samp_ms, asm_s_ms = [], []
        for _ in range(2):                              # the first pass warms the kernels
            batches = []
            for p, d in zip(parts, devs):
                b = C.c_void_p()
                capi.check(capi.ps_search_device(p.handle, C.byref(d), C.byref(dsp), nnz, C.byref(prm_f),
                                                 C.byref(b)))
                batches.append(b)
            pp = [engine._device_results(b) for b in batches]
            engine.assemble(pp, n, prm.top_k, out_full, stream, fit=fit)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record(stream)
            spp = [engine.sample(part, n, stream, rec=r)[0] for part, r in zip(pp, recs)]
            ev[1].record(stream)
            engine.assemble(spp, n, prm.top_k, out_s, stream, fit=fit)
            ev[2].record(stream)
            ev[2].synchronize()
            for b in batches:
                capi.ps_batch_free(b)
            samp_ms.append(ev[0].elapsed_time(ev[1]))
            asm_s_ms.append(ev[1].elapsed_time(ev[2]))
        hf, sf, _ = out_full.to_host()
        hs, ss, _ = out_s.to_host()
        flags = np.stack([engine.sampled_to_host(r, n)["flags"] for r in recs])
        lossless = np.all(flags == 0, axis=0)
        same_l = (hs[lossless].tobytes() == hf[lossless].tobytes()
                  and ss[lossless].tobytes() == sf[lossless].tobytes())
        assert same_l, "sampled assembly differs from the full one where no sample was lost"
        assert hs.tobytes() == hf.tobytes(), "hits never depend on the histograms"
        both = (~lossless) & (ss["status"] == 0) & (sf["status"] == 0)
        rel = np.abs(ss["evalue"][both] - sf["evalue"][both]) / np.abs(sf["evalue"][both])
        res["sampled"][fit_name] = {
            "record_bytes": capi.SAMPLED_DTYPE.itemsize, "histogram_bytes": capi.PS_HIST_BINS * 4,
            "sample_ms": samp_ms[-1], "assemble_ms": asm_s_ms[-1], "lossless_fraction": float(lossless.mean()),
            "identical_where_lossless": bool(same_l),
            "lossy_evalue_rel_change_median": float(np.median(rel)) if rel.size else None,
            "lossy_evalue_rel_change_p90": float(np.quantile(rel, 0.9)) if rel.size else None}
        log(f"partitions, sampled ({fit_name} fit): {G} x ps_sample {samp_ms[-1]:.3f} ms, assembly "
            f"{asm_s_ms[-1]:.3f} ms, {100 * lossless.mean():.2f}% of spectra lost no sample, lossy e-values moved "
            f"by a median {res['sampled'][fit_name]['lossy_evalue_rel_change_median']}")
    return res


def small_batch_leg(capi, engine, torch, ix, sp, params, use, sizes=(256, 1024, 4096, 16384), reps=10):
    """Graph-replayed searches of small batches (the serving regime): one
    workgroup per spectrum leaves most of the GPU idle when a batch holds fewer
    spectra than the GPU holds workgroups, while the persistent work queue
    splits every window into items.  Spectra/s of both schedules, same results;
    the persistent schedule is autotuned for each batch size."""
    out = []
    for n in sizes:
        sub = sp.slice(0, n)
        tens = device_spectra(sub, torch)
        nnz = int(sub.peak_off[-1])
        row = {"spectra": n}
        ref = None
        for name, prm in params:
            use(name)
            if name == "persistent":
                best, _ = engine.autotune(ix, sub, prm)      # sets the index's schedule
                row["persistent_schedule"] = {"tile": best.tile, "tiles_per_item": best.tiles_per_item,
                                              "groups_per_cu": best.groups_per_cu}
            plan = engine.Plan(ix, prm, n_cap=n, nnz_cap=nnz)
            fill_plan_inputs(plan, tens, torch)
            plan.run_device(n, nnz)
            r = plan.results()
            torch.cuda.synchronize()
            dt = float("inf")
            for _ in range(3):                      # best of three groups: the batches are short
                t0 = time.perf_counter()
                for _ in range(reps):
                    plan.run_device(n, nnz)
                    r = plan.results()
                dt = min(dt, (time.perf_counter() - t0) / reps)
            if ref is None:
                ref = r.hits.tobytes()
            assert r.hits.tobytes() == ref, "schedules disagree on a small batch"
            row[name] = {"spectra_per_s": n / dt, "ms_per_batch": dt * 1e3}
            del plan
        log(f"small batch {n}: " + ", ".join(f"{k} {v['spectra_per_s']:.0f} spectra/s" for k, v in row.items()
                                               if isinstance(v, dict) and "spectra_per_s" in v))
        out.append(row)
    return out


def _requests(pool_sp, sizes, starts):
    """Requests as contiguous slices of the pool of spectra (wrapping around)."""
    out = []
    n = pool_sp.n
    for s, k in zip(starts, sizes):
        s, k = int(s), int(k)
        if s + k <= n:
            out.append(pool_sp.slice(s, s + k))
        else:
            out.append(type(pool_sp).concat([pool_sp.slice(s, n), pool_sp.slice(0, s + k - n)]))
    return out


def serve(engine, capi, synth, ix, prm, pool_sp, load, capacity, n_requests, seed, pool_bytes, streams,
          run_spectra):
    """Requests of 1..4096 spectra through the continuous-batching server.
    load = None: all requests offered at once (saturating; the memory guard
    refuses and the client retries); else Poisson arrivals at load x capacity
    spectra/s.  Latency is measured by the server from submit to completion."""
    mean_size = (1 + 4096) / 2
    if load is None:
        rng = np.random.default_rng(seed)
        t_arr = np.zeros(n_requests)
        sizes = rng.integers(1, 4097, size=n_requests)
        rate = None
    else:
        rate = load * capacity / mean_size
        t_arr, sizes = synth.poisson_arrivals(n_requests, rate, 1, 4096, seed=seed)
    starts = np.random.default_rng(seed + 1000).integers(0, pool_sp.n, size=n_requests)
    reqs = _requests(pool_sp, sizes, starts)
    srv = engine.Server(ix, prm, pool_bytes=pool_bytes, run_spectra=run_spectra, max_runs=streams)
    # one full-size request per stream first, so that no timed request pays a first run
    warm = [srv.submit(pool_sp.slice(0, 4096)) for _ in range(streams)]
    for t in warm:
        srv.wait(t, 4096)
    srv.reset_stats()
    tickets = [None] * n_requests

    def waiter():
        for i in range(n_requests):
            while tickets[i] is None:
                time.sleep(0.0002)
            srv.wait(tickets[i], reqs[i].n)

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    retries = 0
    for i in range(n_requests):
        dt = t_arr[i] - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        while True:
            try:
                tickets[i] = srv.submit(reqs[i])
                break
            except capi.PsError as e:
                if e.code != capi.PS_EAGAIN:
                    raise
                retries += 1
                time.sleep(0.0005)
    th.join()
    st = srv.stats()
    srv.close()
    return {"load": load if load is not None else "saturating", "arrival_rate_per_s": rate,
            "requests": n_requests, "latency_samples": int(st.samples), "spectra": int(st.spectra),
            "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "max_ms": st.max_ms, "mean_ms": st.mean_ms,
            "spectra_per_s": st.spectra / st.elapsed_s if st.elapsed_s > 0 else None,
            "runs": int(st.runs), "refused_then_retried": int(st.refused), "streams": int(st.streams),
            "pool_bytes": int(st.pool_bytes), "peak_bytes": int(st.peak_bytes), "max_queue": int(st.max_queue)}


def serving_leg(capi, engine, torch, synth, w, prot, ix, args, plain_schedule):
    """Serving (continuous batching, admission by device memory) on the
    resident index with the serving recipe's spectra (charges 2-4).  Capacity
    is first measured with a saturating load; the Poisson loads are fractions
    of it.  The plain graph over one batch of the same spectra is timed beside
    it, at equal results (the served results equal the batch's bit for bit)."""
    pool_sp = w.spectra(prot, n=args.serving_pool, seed=2, charges=(2, 3, 4))
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=4, schedule=capi.PS_SCHED_PERSISTENT, want_hist=False)
    prm_plain = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k,
                                     w.min_shared, max_charge=4, schedule=capi.PS_SCHED_PLAIN, want_hist=False)
    default = ix.schedule()
    capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(default)))
    best, _ = engine.autotune(ix, pool_sp.slice(0, 4096), prm)
    log(f"serving: persistent schedule tuned on 4096-spectrum requests: tile {best.tile}, "
        f"{best.group_threads or 256} threads per workgroup, {best.tiles_per_item} tiles per item, "
        f"{best.groups_per_cu} groups per CU")
    # the plain batch on the same spectra, as one graph plan
    tens = device_spectra(pool_sp, torch)
    nnz = int(pool_sp.peak_off[-1])
    saved = capi.ps_schedule.from_buffer_copy(ix.schedule())
    capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(plain_schedule)))
    plan = engine.Plan(ix, prm_plain, n_cap=pool_sp.n, nnz_cap=nnz)
    fill_plan_inputs(plan, tens, torch)
    plan.run_device(pool_sp.n, nnz)
    batch_res = plan.results()
    t0 = time.perf_counter()
    for _ in range(3):
        plan.run_device(pool_sp.n, nnz)
        plan.results()
    plain_rate = 3 * pool_sp.n / (time.perf_counter() - t0)
    del plan, tens
    capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(saved)))
    log(f"serving recipe, plain graph over {pool_sp.n} spectra (the plain schedule of the headline): "
        f"{plain_rate:.0f} spectra/s")
    out = {"recipe": f"{pool_sp.n} spectra of the large recipe with charges 2-4 (seed 2); requests are "
                     f"contiguous slices of 1-4096 spectra", "plain_batch_spectra_per_s": plain_rate,
           "persistent_schedule": {"tile": best.tile, "group_threads": best.group_threads,
                                   "tiles_per_item": best.tiles_per_item, "groups_per_cu": best.groups_per_cu},
           "loads": []}
    sat = serve(engine, capi, synth, ix, prm, pool_sp, None, None, args.serving_sat_requests, 5,
                args.serving_pool_gb << 30, args.serving_streams, args.serving_run)
    log(f"serving saturated: {sat['spectra_per_s']:.0f} spectra/s over {sat['requests']} requests "
        f"({sat['runs']} runs), p50 {sat['p50_ms']:.1f} ms p99 {sat['p99_ms']:.1f} ms")
    out["loads"].append(sat)
    cap = sat["spectra_per_s"]
    for load, seed in ((0.5, 2), (0.8, 3), (0.95, 4)):
        r = serve(engine, capi, synth, ix, prm, pool_sp, load, cap, args.serving_requests, seed,
                  args.serving_pool_gb << 30, args.serving_streams, args.serving_run)
        log(f"serving load {load}: p50 {r['p50_ms']:.1f} ms, p99 {r['p99_ms']:.1f} ms, "
            f"{r['spectra_per_s']:.0f} spectra/s over {r['requests']} requests ({r['runs']} runs)")
        out["loads"].append(r)
    # served results equal the batch's (checked on one request of the pool's head)
    srv = engine.Server(ix, prm, pool_bytes=1 << 30, run_spectra=4096, max_runs=2)
    head = pool_sp.slice(0, 777)
    hits, stats, _, _ = srv.wait(srv.submit(head), head.n)
    srv.close()
    assert hits.tobytes() == batch_res.hits[:777].tobytes(), "served results differ from the batch"
    assert stats.tobytes() == batch_res.stats[:777].tobytes(), "served stats differ from the batch"
    out["saturated_vs_plain"] = cap / plain_rate
    capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(saved)))
    return out


def node_share_leg(capi, engine, torch, synth, args):
    """One node's share of the largest database (200k proteins, four
    modification types, <= 3 per peptide: 1.12G peptides): partition 0 of 16
    built on the GPU, searched with spectra of the serving recipe (charges 2-4).
    The sustained rate is measured over a seeded slice of the 5M-spectrum
    recipe (the slice is named), each schedule autotuned on 4096 of them."""
    w = synth.workload("node")
    prot = w.proteome()
    G = 16
    t0 = time.perf_counter()
    ix = build_index(engine, w, prot, w.frag_tol_bins, n_shards=G, shard=0)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    n_pep, n_post, n_bins = ix.shape()
    grain, dir_bytes = ix.directory()
    log(f"node share: partition 0 of {G}: {n_pep} peptides, {n_post} postings, directory {dir_bytes / 1e9:.1f} GB "
        f"(grain {1 << grain}), built on the GPU in {build_s:.1f}s")
    sp = w.spectra(prot, n=args.node_spectra, seed=1)
    nnz = int(sp.peak_off[-1])
    tens = device_spectra(sp, torch)
    dsp = capi.ps_spectra(sp.n, *[x.data_ptr() for x in tens])
    out = {"database": f"{prot.n} proteins, Met-ox, STY phospho, protein N-term acetyl, N/Q deamidation, "
                       f"<= {w.max_mods} mods per peptide; partition 0 of {G} round-robin partitions",
           "partition_peptides": n_pep, "partition_postings": n_post, "directory_bytes": dir_bytes,
           "device_bytes": ix.arena.numel(), "build_s": build_s,
           "slice": f"{sp.n} spectra of the 5M-spectrum recipe (seed 1; 20-200 peaks, lognormal precursor "
                    f"masses around 1800 Da, charges 2-4)", "forms": {}}
    default = capi.ps_schedule.from_buffer_copy(ix.schedule())
    ref = None
    for name, schedule in (("plain", capi.PS_SCHED_PLAIN), ("persistent", capi.PS_SCHED_PERSISTENT)):
        prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                                   max_charge=4, schedule=schedule, want_hist=False)
        capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(default)))
        best, _ = engine.autotune(ix, sp.slice(0, min(sp.n, 4096)), prm)
        need = C.c_uint64()
        capi.check(capi.ps_workspace_bytes(ix.handle, sp.n, nnz, C.byref(prm), C.byref(need)))
        ws = engine.Workspace()
        d = ws.get(need.value)
        eager_steps(capi, engine, ix, dsp, sp.n, nnz, prm, d, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        scan_ms, res = eager_steps(capi, engine, ix, dsp, sp.n, nnz, prm, d, 3)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 3
        if ref is None:
            ref = res
        assert res.hits.tobytes() == ref.hits.tobytes(), "schedules disagree on the node share"
        alg = 4.0 * res.postings + 16.0 * res.lookups
        scan = float(np.mean(scan_ms))
        out["forms"][name] = {"spectra_per_s": sp.n / dt, "ms_per_step": dt * 1e3, "scan_ms": scan,
                              "achieved_GBs": alg / (scan * 1e-3) / 1e9,
                              "frac": alg / (scan * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "postings": res.postings, "dense_postings": res.dense_postings,
                              "layout_GBs": (4.0 * (res.postings - res.dense_postings) + 16.0 * res.lookups
                                             + res.dense_reads) / (scan * 1e-3) / 1e9,
                              "wide_counter_spectra": res.wide_spectra,
                              "schedule": {"tile": best.tile, "group_threads": best.group_threads,
                                           "tiles_per_item": best.tiles_per_item,
                                           "groups_per_cu": best.groups_per_cu}}
        log(f"node share {name}: {sp.n / dt:.0f} spectra/s sustained over {sp.n} spectra, scan {scan:.1f} ms = "
            f"{out['forms'][name]['achieved_GBs']:.0f} GB/s, schedule {out['forms'][name]['schedule']}")
    del ix, tens
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--n-spectra", type=int, default=100000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000, help="requests per Poisson load")
    ap.add_argument("--serving-sat-requests", type=int, default=1000, help="requests of the saturating load")
    ap.add_argument("--serving-pool", type=int, default=40000, help="spectra the requests are sliced from")
    ap.add_argument("--serving-pool-gb", type=int, default=16, help="device memory the server admits into")
    ap.add_argument("--serving-streams", type=int, default=4)
    ap.add_argument("--serving-run", type=int, default=8192, help="packing target of a server run (spectra)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tune-cache", default=None, help="file caching autotuned schedules")
    ap.add_argument("--classic-index", action="store_true",
                    help="one posting list per fragment bin (default: lists merge the 2T+1 neighbouring bins)")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB device copy (counter scale)")
    ap.add_argument("--no-small-batches", action="store_true", help="skip the small-batch plain/persistent leg")
    ap.add_argument("--shards", type=int, default=4,
                    help="also search G round-robin database partitions and assemble them (0: skip)")
    ap.add_argument("--no-node-share", action="store_true", help="skip the node-share partition leg")
    ap.add_argument("--no-dense-compare", action="store_true",
                    help="skip the eager run with every list streamed (dense maps off)")
    ap.add_argument("--node-spectra", type=int, default=20000, help="spectra of the node-share slice")
    ap.add_argument("--only", choices=["plain", "persistent"], default=None,
                    help="time one form only (for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the search runs on one GPU: the index scan and its results are "
                                   "measured on one MI355X, so --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2102_02286_amd import capi, engine, synth

    w = synth.workload(args.workload)
    t0 = time.perf_counter()
    prot = w.proteome()
    sp = w.spectra(prot, n=args.n_spectra)
    log(f"workload {w.name}: {prot.n} proteins, {sp.n} spectra generated in {time.perf_counter() - t0:.1f}s")
    merge = 0 if args.classic_index else w.frag_tol_bins
    t0 = time.perf_counter()
    ix = build_index(engine, w, prot, merge)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    n_pep, n_post, n_bins = ix.shape()
    grain, dir_bytes = ix.directory()
    log(f"index: {n_pep} peptides, {n_post} postings (lists of {2 * merge + 1} bin(s) each), {n_bins} bins, "
        f"directory {dir_bytes / 1e9:.2f} GB, {ix.arena.numel() / 1e9:.1f} GB on the device, built on the GPU in "
        f"{build_s:.2f}s")
    max_charge = int(sp.charge.max()) if sp.n else 1
    nnz = int(sp.peak_off[-1])
    tens = device_spectra(sp, torch)
    dsp = capi.ps_spectra(sp.n, *[x.data_ptr() for x in tens])

    def params(schedule):
        return engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k,
                                    w.min_shared, max_charge=max_charge, schedule=schedule, want_hist=False)

    prm_plain, prm_pers = params(capi.PS_SCHED_PLAIN), params(capi.PS_SCHED_PERSISTENT)
    out = {}

    # ---- schedules: each form autotuned on a sample (identical results are checked inside)
    def as_dict(sc):
        return {f: getattr(sc, f) for f, _ in capi.ps_schedule._fields_ if f != "reserved"}

    default = ix.schedule()
    tuned = {}
    for name, prm in (("plain", prm_plain), ("persistent", prm_pers)):
        capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(default)))
        if not args.no_tune:
            t0 = time.perf_counter()
            best, trials = engine.autotune(ix, sp.slice(0, min(sp.n, 20000)), prm, cache_path=args.tune_cache)
            log(f"autotune {name}: {len(trials)} trials in {time.perf_counter() - t0:.1f}s -> {as_dict(best)}")
        tuned[name] = capi.ps_schedule.from_buffer_copy(ix.schedule())

    def use(name):
        capi.check(capi.ps_index_set_schedule(ix.handle, C.byref(tuned[name])))

    ws = engine.Workspace()
    need = C.c_uint64()
    capi.check(capi.ps_workspace_bytes(ix.handle, sp.n, nnz, C.byref(prm_pers), C.byref(need)))
    ws_dev = ws.get(need.value)

    # ---- eager forms: the scan kernels timed with HIP events on their stream
    eager = {}
    for name, prm in (("plain", prm_plain), ("persistent", prm_pers)):
        if args.only not in (None, name):
            continue
        use(name)
        eager_steps(capi, engine, ix, dsp, sp.n, nnz, prm, ws_dev, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        scan_ms, res = eager_steps(capi, engine, ix, dsp, sp.n, nnz, prm, ws_dev, args.steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        eager[name] = {"spectra_per_s": sp.n * args.steps / dt, "ms_per_step": dt * 1e3 / args.steps,
                       "scan_ms": float(np.mean(scan_ms)), "scan_ms_min": float(np.min(scan_ms)), "res": res}
        log(f"{name} eager: {eager[name]['spectra_per_s']:.0f} spectra/s, {eager[name]['ms_per_step']:.1f} ms/step, "
            f"scan {eager[name]['scan_ms']:.1f} ms (HIP events), {res.wide_spectra} spectra on 64-bit counters")
    if len(eager) == 2:
        assert eager["plain"]["res"].hits.tobytes() == eager["persistent"]["res"].hits.tobytes(), \
            "plain and persistent results differ"
        assert eager["plain"]["res"].stats.tobytes() == eager["persistent"]["res"].stats.tobytes()

    # ---- the same eager search with every list streamed as postings (dense maps
    # off): what the maps of the y1 lists save, at identical results
    streamed = None
    if not args.no_dense_compare and eager:
        name = "persistent" if "persistent" in eager else "plain"
        prm = prm_pers if name == "persistent" else prm_plain
        use(name)
        ix.set_dense(False)
        try:
            eager_steps(capi, engine, ix, dsp, sp.n, nnz, prm, ws_dev, 1)
            scan_ms, res = eager_steps(capi, engine, ix, dsp, sp.n, nnz, prm, ws_dev, args.steps)
        finally:
            ix.set_dense(True)
        assert res.hits.tobytes() == eager[name]["res"].hits.tobytes(), "dense maps changed the results"
        assert res.stats.tobytes() == eager[name]["res"].stats.tobytes(), "dense maps changed the results"
        streamed = {"schedule": name, "scan_ms": float(np.mean(scan_ms)), "dense_scan_ms": eager[name]["scan_ms"],
                    "speedup": float(np.mean(scan_ms)) / eager[name]["scan_ms"]}
        log(f"{name} eager with every list streamed (no dense maps): scan {streamed['scan_ms']:.1f} ms vs "
            f"{eager[name]['scan_ms']:.1f} ms with them ({streamed['speedup']:.2f}x), identical results")

    # ---- graph plans over the resident batch (both schedules); the faster is the headline
    def graph_steps(name, prm, eager_ref):
        use(name)
        plan = engine.Plan(ix, prm, n_cap=sp.n, nnz_cap=nnz)
        fill_plan_inputs(plan, tens, torch)
        for _ in range(args.warmup):
            plan.run_device(sp.n, nnz)
            plan.results()
        torch.cuda.synchronize()
        log(f"timing {args.steps} {name} graph steps")
        t0 = time.perf_counter()
        graph_ms = []
        for _ in range(args.steps):
            plan.run_device(sp.n, nnz)
            r = plan.results()
            graph_ms.append(r.graph_ms)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert r.hits.tobytes() == eager_ref.hits.tobytes(), f"{name} graph replay and eager results differ"
        g = {"spectra_per_s": sp.n * args.steps / dt, "ms_per_step": dt * 1e3 / args.steps,
             "graph_ms": float(np.mean(graph_ms)), "work_items": int(r.items)}
        log(f"{name} graph: {g['spectra_per_s']:.0f} spectra/s, {g['ms_per_step']:.1f} ms/step, "
            f"graph {g['graph_ms']:.1f} ms")
        del plan
        return g

    forms = {}
    for name, prm in (("plain", prm_plain), ("persistent", prm_pers)):
        if name in eager:
            forms[name] = graph_steps(name, prm, eager[name]["res"])
    ref = eager.get("plain", eager.get("persistent"))["res"]
    st = np.bincount(ref.stats["status"], minlength=6)
    log(f"status counts {st.tolist()}")

    # headline: the faster graph form; its scan kernel's HIP-event time gives the roofline
    form = max(forms, key=lambda k: forms[k]["spectra_per_s"])

    # the same form with the spectra handed over in host memory (ps_plan_run copies
    # them in, then replays the graph): the rate with the PCIe transfer, never `value`
    def host_input_steps(prm, eager_ref):
        use(form)
        plan = engine.Plan(ix, prm, n_cap=sp.n, nnz_cap=nnz)
        plan.search(sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = plan.search(sp)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert r.hits.tobytes() == eager_ref.hits.tobytes(), "host-input plan and eager results differ"
        in_bytes = int(sp.peak_off[-1]) * 8 + sp.n * (8 + 8 + 1)
        del plan
        return {"spectra_per_s": sp.n * args.steps / dt, "ms_per_step": dt * 1e3 / args.steps,
                "input_bytes": in_bytes}
    pcie = host_input_steps(prm_plain if form == "plain" else prm_pers, eager[form]["res"])
    log(f"{form} graph with host inputs: {pcie['spectra_per_s']:.0f} spectra/s, {pcie['ms_per_step']:.1f} ms/step "
        f"({pcie['input_bytes'] / 1e6:.0f} MB of spectra copied in per step)")
    kernel = "k_scan_plain" if form == "plain" else "k_scan_persistent"
    head_scan = eager[form]["scan_ms"]
    postings, lookups = ref.postings, ref.lookups
    alg_bytes = 4.0 * postings + 16.0 * lookups
    achieved = alg_bytes / (head_scan * 1e-3) / 1e9
    # what the layout reads: streamed postings, bin lookups, and two bits per id
    # of every dense probe's map
    streamed_post = postings - ref.dense_postings
    layout_bytes = 4.0 * streamed_post + 16.0 * lookups + 1.0 * ref.dense_reads
    layout_gbs = layout_bytes / (head_scan * 1e-3) / 1e9
    copy_gbs = copy_bandwidth(torch)
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
    lds_gops = streamed_post / (head_scan * 1e-3) / 1e9
    out.update({
        "metric": "spectra searched/sec at 1 MI355X (serving vs plain batch), p99 latency, HBM GB/s %",
        "value": forms[form]["spectra_per_s"],
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": forms[form]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {prot.n} proteins, Met-ox + STY phospho <= {w.max_mods} mods, "
                               f"{n_pep} peptides, {n_post} postings (lists merging {2 * merge + 1} neighbouring "
                               f"bin(s)), index built on the GPU; a seeded batch of {sp.n} spectra of the "
                               f"1M-spectrum recipe (20-200 peaks, precursor masses lognormal around 1800 Da, "
                               f"charges 2-3); window +-{w.window / 1e6:g} Da, fragment tol {w.frag_tol_bins} "
                               f"bin(s), top {w.top_peaks} peaks, top {w.top_k} hits; whole search replayed as a "
                               f"hipGraph, {form} scan schedule",
                   "schedule": form},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(w.name, kernel),
                     "kernel": f"{kernel} (posting scan)", "scan_ms": head_scan,
                     "bytes_per_launch": alg_bytes, "postings_per_launch": postings,
                     "bin_lookups_per_launch": lookups, "copy_GBs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs,
                     "layout": {"bytes_per_launch": layout_bytes, "achieved": layout_gbs,
                                "frac": layout_gbs / HBM_PEAK_GBS, "dense_postings": ref.dense_postings,
                                "dense_map_reads": ref.dense_reads,
                                "note": "bytes the index layout reads: 4 B per streamed posting, 16 B per "
                                        "bin lookup, 1 B per dense-map read; the 4-byte figure above "
                                        "counts every posting"},
                     "lds_atomics": {"achieved_Gops": lds_gops, "peak_Gops": LDS_ATOMIC_PEAK_GOPS,
                                     "frac": lds_gops / LDS_ATOMIC_PEAK_GOPS,
                                     "note": "one 4-byte LDS atomic per streamed posting"}},
        "streamed_only": streamed,
        "wide_counter_spectra": int(ref.wide_spectra),
        "overflow_spectra": int(ref.overflow_spectra),
        "forms": {k: {**forms[k], "eager_spectra_per_s": eager[k]["spectra_per_s"],
                      "eager_ms_per_step": eager[k]["ms_per_step"], "scan_ms": eager[k]["scan_ms"]}
                  for k in forms},
        "host_inputs": {"form": form, **pcie, "note": "the headline graph with the spectra copied in from host "
                        "memory every step (PCIe-inclusive; never the value)"},
        "schedule": {k: as_dict(tuned[k]) for k in tuned},
        "index_build": {"device_s": build_s, "entries": n_pep, "postings": n_post,
                        "device_bytes": ix.arena.numel(), "directory_bytes": dir_bytes},
    })
    log(f"headline: {form} graph {forms[form]['spectra_per_s']:.0f} spectra/s; roofline: {alg_bytes / 1e9:.1f} GB "
        f"algorithmic per step in {head_scan:.1f} ms = {achieved:.0f} GB/s ({100 * achieved / HBM_PEAK_GBS:.1f}%); "
        f"the layout reads {layout_bytes / 1e9:.1f} GB = {layout_gbs:.0f} GB/s ({100 * layout_gbs / HBM_PEAK_GBS:.1f}%), "
        f"{100 * ref.dense_postings / max(postings, 1):.1f}% of postings through dense maps")

    # ---- partitioned database: G partition searches + on-device result assembly
    if args.shards > 1 and "plain" in eager:
        use("plain")
        out["assembly"] = assembly_leg(capi, engine, torch, w, prot, merge, args.shards, dsp, sp.n, nnz,
                                       prm_plain, eager["plain"]["res"], args.steps, args.warmup)

    # ---- small batches: where the persistent work queue pays
    if len(forms) == 2 and not args.no_small_batches:
        out["small_batches"] = small_batch_leg(capi, engine, torch, ix, sp,
                                               [("plain", prm_plain), ("persistent", prm_pers)], use)

    # ---- serving: continuous batching with admission by device memory
    if not args.no_serving:
        out["serving"] = serving_leg(capi, engine, torch, synth, w, prot, ix, args, tuned.get("plain", default))

    # ---- one node's share of the largest database
    if not args.no_node_share:
        torch.cuda.empty_cache()
        out["node_share"] = node_share_leg(capi, engine, torch, synth, args)

    if args.copy_probe:
        # a plain device copy of known size: its FETCH_SIZE / WRITE_SIZE under
        # rocprofv3 --pmc scale the scan kernel's counters to bytes
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 1 << 30

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, prot, sp)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.2f} spectra/s ({out['cpu_baseline']['sample']})")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
