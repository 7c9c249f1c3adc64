#!/usr/bin/env python3
"""Benchmark of the dense full-tableau simplex on one MI355X; prints one JSON line.

One step = one pass of the whole solve on the 8000 x 8000 dense LP (seed 3;
tableau 8001 x 16001 binary64, about 1 GB, resident in HBM): rebuild the
tableau of Table I from the device-resident A, b, c (Initialization Step),
pivot with Steps 1-3 until optimal, and extract x, y and the objective.

Reported:
  value           pivots/s over the timed steps (inputs already in HBM);
  roofline        the Step 3 update pass (the HBM-bound kernel): algorithmic
                  bytes per launch / its average duration from HIP events
                  recorded around it on its own stream during the timed
                  steps, against 8 TB/s;
  cpu_baseline    the CPU oracle on the host cores (generation excluded):
                  full solves of the same LP on all cores (value) and its
                  first pivots on one, the 200 x 200 and 2000 x 2000 LPs,
                  the batch of 512 serially and one LP per thread, an
                  estimate for the serving trace from its first 200 LPs,
                  and a STREAM-style triad of the host;
  small           the 200 x 200 and 2000 x 2000 LPs on the GPU;
  batched         the 512-LP batch against one-at-a-time solves;
  serving         the 10,000-LP Poisson trace through the server against
                  one-at-a-time solves of the same trace (arrivals at 1.5x
                  the one-at-a-time rate; all at once; all at once under a
                  tight budget).

    python bench.py [--steps K] [--warmup W] [--workload NAME]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pivots/s + HBM GB/s (m=n=8000 FP64); batched LP solves/s & p99 latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def update_bytes(m: int, n: int, cols: int, pivots: int) -> float:
    """Algorithmic bytes of the update passes that applied `pivots` pivots and
    rewrote `cols` columns in total (a column counts once per pass, however
    many pivots of the pass change it): each rewritten column is read and
    written once (16 (m+1) B); every pivot also brings its pivot column F
    (8 (m+1) B) and, for every column, its pivot-row and row-0 entries
    (16 W B)."""
    W = n + m + 1
    return 16.0 * (m + 1) * cols + pivots * (8.0 * (m + 1) + 16.0 * W)


def first_pass_bytes(m: int, n: int, columns: int, pivots: int) -> float:
    """Algorithmic bytes of the first update pass after a deferred build,
    which wrote `columns` columns (the n structural ones, the RHS and the
    columns appended during its group) with `pivots` pivots applied: A and c
    read and the structural columns written (the build of that part of the
    tableau), the other columns read and written, and per pivot its F column
    and the pivot-row and row-0 entries of every column."""
    W = n + m + 1
    return (8.0 * m * n + 8.0 * n + 8.0 * (m + 1) * n + 16.0 * (m + 1) * (columns - n)
            + pivots * (8.0 * (m + 1) + 16.0 * W))


CSRC = os.path.join(ROOT, "paper_2211_10979_amd", "csrc")


def kernel_source(kernel):
    """The header that defines the update kernel instance `kernel`."""
    name = "fused_kernels.hpp" if kernel.startswith("k_gupdate") else "plain_kernels.hpp"
    return os.path.join(CSRC, name)


def committed_traffic(kernel, workload):
    """HBM bytes per update launch that applied pivots, from the committed
    rocprofv3 counter summary of this kernel on this workload (FETCH_SIZE and
    WRITE_SIZE, each scaled by the copy-kernel calibration). None unless that
    summary was taken on this kernel instance built from the current source."""
    import hashlib

    counters = os.path.join(ROOT, "profiles", f"{kernel.split('<')[0]}_{workload}_counters.md")
    if not os.path.exists(counters):
        return None
    kv = {}
    for line in open(counters):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            v = v.strip()
            if v.startswith("`"):  # a quoted value, taken whole
                v = v[1:].split("`", 1)[0]
            elif v:
                v = v.split()[0]
            kv[k.strip()] = v
    src = hashlib.sha256(open(kernel_source(kernel), "rb").read()).hexdigest()
    if kv.get("kernel") != kernel or kv.get("source_sha256") != src:
        return None
    try:
        return float(kv["traffic_bytes_per_applied_launch"])
    except (KeyError, ValueError):
        return None


def bench_plain(args, lpgpu, lpgen, torch):
    lp = lpgen.workload(args.workload)
    m, n = lp.m, lp.n
    dev = torch.device("cuda", 0)
    dA = torch.from_numpy(lp.A).to(dev)
    db = torch.from_numpy(lp.b).to(dev)
    dc = torch.from_numpy(lp.c).to(dev)
    torch.cuda.synchronize()
    h = lpgpu.lp_create_device(m, n, dA, db, dc, time_kernels=args.time_kernels, chunk_pivots=args.chunk,
                               cols_per_block=args.cols_per_block, rows_per_thread=args.rows_per_thread,
                               fuse_pivots=args.fuse)
    try:
        def step():
            lpgpu.lp_reload_device(h, dA, db, dc)
            lpgpu.lp_solve(h)
            return lpgpu.lp_get_solution(h)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        tot_piv = tot_cols = tot_launch = tot_applied = 0
        first_piv = first_changed = first_launches = 0
        first_ms = first_alg = 0.0
        upd_ms = upd_ms_applied = 0.0
        solve_ms = 0.0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res, x, y = step()
            t = lpgpu.lp_get_timing(h)
            tot_piv += t["pivots"]
            tot_cols += t["updated_columns"]
            tot_launch += t["update_launches"]
            tot_applied += t["applied_launches"]
            upd_ms += t["update_ms"]
            upd_ms_applied += t["update_ms_applied"]
            solve_ms += t["solve_ms"]
            if t["first_pass_columns"]:
                first_launches += 1
                first_piv += t["first_pass_pivots"]
                first_changed += t["first_pass_changed"]
                first_ms += t["first_pass_ms"]
                first_alg += first_pass_bytes(m, n, t["first_pass_columns"], t["first_pass_pivots"])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        rows, cols = lpgpu.lp_get_pivots(h)
        info = lpgpu.lp_get_info(h)
        fuse = info.update_fuse
        readback = info.status_readback
        if fuse > 1:  # the update instance: groups of up to 2, 4, 8, 12, 16, 24, 32 or 48 pivots
            kf = next(k for k in (2, 4, 8, 12, 16, 24, 32, 48) if k >= fuse)
            if info.decide_workgroups > 0 and kf >= 48:  # on the matrix cores
                kernel = f"k_gpure_mf<{kf}>"
            else:
                name = "k_gupdate_pure" if info.decide_workgroups > 0 else "k_gupdate"
                kernel = f"{name}<{info.update_block}, {info.update_cols}, {kf}>"
        else:
            kernel = (f"k_update<{info.update_block}, {info.update_cols}, {info.update_rows}, "
                      f"{info.update_hints & 1}, {info.update_hints >> 1}>")
    finally:
        lpgpu.lp_destroy(h)
    from paper_2211_10979_amd.certify import certify

    ok, resid = certify(lp.A, lp.b, lp.c, x, y, res["objective"])
    W = n + m + 1
    per_piv = tot_piv / args.steps
    # the update passes after the first group; the first pass after a
    # deferred build (which also builds the structural columns) on its own
    upd_cols, upd_piv = tot_cols - first_changed, tot_piv - first_piv
    alg_total = update_bytes(m, n, upd_cols, upd_piv) + first_alg
    out = dict(
        value=tot_piv / elapsed,
        ms_per_step=1000.0 * elapsed / args.steps,
        pivots_per_solve=per_piv,
        solves_per_s=args.steps / elapsed,
        status=lpgpu.STATUS_NAMES[res["status"]],
        objective=res["objective"],
        certificates_ok=bool(ok),
        certificate_max_residual=max(resid.values()),
        fuse_pivots=fuse,
        status_readback=readback,
        end_to_end_alg_gbs=alg_total / elapsed / 1e9,
        end_to_end_alg_frac=alg_total / elapsed / 1e9 / HBM_PEAK_GBS,
        device_solve_ms_per_step=solve_ms / args.steps,
        full_tableau_bytes_per_pivot=16.0 * (m + 1) * W,
        log=(rows, cols),
        lp=lp,
    )
    if tot_launch:
        # every update launch is timed, including the one queued after the
        # optimum (it returns at once and carries no algorithmic bytes), so
        # that the average matches rocprofv3's over all dispatches; the
        # launches that applied pivots are also reported on their own
        alg = update_bytes(m, n, upd_cols, upd_piv)
        per_launch_bytes = alg / tot_launch
        avg_ms = upd_ms / tot_launch
        ach = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        tr = committed_traffic(kernel, args.workload)
        traffic = None if tr is None else round(tr * tot_applied / tot_launch)  # per launch, as achieved
        out["roofline"] = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                               frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic,
                               kernel=kernel, avg_launch_us=round(avg_ms * 1e3, 2),
                               alg_bytes_per_launch=per_launch_bytes, launches=tot_launch,
                               applied_launches=tot_applied,
                               avg_applied_launch_us=round(upd_ms_applied / max(tot_applied, 1) * 1e3, 2),
                               alg_bytes_per_applied_launch=alg / max(tot_applied, 1),
                               achieved_applied=round(alg / max(upd_ms_applied, 1e-9) / 1e6, 1),
                               pivots=upd_piv, alg_bytes_per_pivot=alg / max(upd_piv, 1),
                               columns_per_pivot=upd_cols / max(upd_piv, 1))
    # the library's default path (no per-launch timing events, which each
    # delay the next dispatch by a few microseconds): the same steps, timed
    # on their own
    if args.time_kernels:
        h2 = lpgpu.lp_create_device(m, n, dA, db, dc, time_kernels=0, chunk_pivots=args.chunk,
                                    cols_per_block=args.cols_per_block, rows_per_thread=args.rows_per_thread,
                                    fuse_pivots=args.fuse)
        try:
            def step2():
                lpgpu.lp_reload_device(h2, dA, db, dc)
                lpgpu.lp_solve(h2)
                return lpgpu.lp_get_solution(h2)

            for _ in range(args.warmup):
                step2()
            torch.cuda.synchronize()
            piv2 = 0
            t0 = time.perf_counter()
            for _ in range(args.steps):
                r2, _, _ = step2()
                piv2 += r2["pivots"]
            torch.cuda.synchronize()
            el2 = time.perf_counter() - t0
            assert r2["pivots"] == res["pivots"] and r2["objective"] == res["objective"]
            out["default_path"] = dict(pivots_per_s=round(piv2 / el2, 1), ms_per_step=round(1000.0 * el2 / args.steps, 4),
                                       note="time_kernels 0: no timing events between the kernels")
        finally:
            lpgpu.lp_destroy(h2)
    if first_launches:
        out["first_pass"] = dict(kernel=f"k_gfirst_rl<{kf}>" if kf >= 32 else f"k_gfirst<{kf}>", launches=first_launches,
                                 avg_launch_us=round(first_ms / first_launches * 1e3, 2),
                                 alg_bytes_per_launch=first_alg / first_launches,
                                 achieved_gbs=round(first_alg / max(first_ms, 1e-9) / 1e6, 1),
                                 pivots_per_launch=first_piv / first_launches)
    return out


def bench_batch(args, lpgpu, lpgen, torch):
    """512 LPs (m, n uniform on [32, 512]): the batched form against the same
    LPs solved one at a time by the single-LP solver, both from
    device-resident inputs, both rebuilding every tableau inside the timed
    region."""
    from paper_2211_10979_amd.certify import certify

    sizes = lpgen.batch_sizes(lpgen.BATCH_SEED, args.batch_lps)
    lps = [lpgen.dense_lp(lpgen.BATCH_SEED, m, n, k=k) for k, (m, n) in enumerate(sizes)]
    h = lpgpu.lp_batch_create([(lp.A, lp.b, lp.c) for lp in lps])
    try:
        tune_ms = lpgpu.lp_batch_autotune(h, os.environ.get("LP_AUTOTUNE_CACHE"), trials=2)
        shape = dict(lpgpu.lp_batch_get_shape(h), **lpgpu.lp_batch_get_split(h))
        for _ in range(2):
            lpgpu.lp_batch_reset(h)
            lpgpu.lp_batch_solve(h)
        reps = args.batch_steps
        dev_ms = 0.0
        t0 = time.perf_counter()
        for _ in range(reps):
            lpgpu.lp_batch_reset(h)
            lpgpu.lp_batch_solve(h)
            dev_ms += lpgpu.lp_batch_solve_ms(h)
        batch_s = (time.perf_counter() - t0) / reps
        results = [lpgpu.lp_batch_get_solution(h, k, lp.m, lp.n) for k, lp in enumerate(lps)]
        logs = [lpgpu.lp_batch_get_pivots(h, k) for k in range(len(lps))]
    finally:
        lpgpu.lp_batch_destroy(h)
    pivots = sum(r[0]["pivots"] for r in results)
    alg = sum(r[0]["pivots"] * 16.0 * (lp.m + 1) * (lp.n + 2) for r, lp in zip(results, lps))
    cert_ok = all(certify(lp.A, lp.b, lp.c, x, y, res["objective"])[0] for (res, x, y), lp in zip(results, lps))

    # one at a time: a context per LP, inputs on the device, same rebuild + solve
    dev = torch.device("cuda", 0)
    ctxs, dins = [], []
    for lp in lps:
        d = [torch.from_numpy(a).to(dev) for a in (lp.A, lp.b, lp.c)]
        dins.append(d)
        ctxs.append(lpgpu.lp_create_device(lp.m, lp.n, *d))
    try:
        for h1, d in zip(ctxs[:16], dins[:16]):
            lpgpu.lp_reload_device(h1, *d)
            lpgpu.lp_solve(h1)
        same = True
        t0 = time.perf_counter()
        for k, (h1, d) in enumerate(zip(ctxs, dins)):
            lpgpu.lp_reload_device(h1, *d)
            lpgpu.lp_solve(h1)
            res, x, y = lpgpu.lp_get_solution(h1)
            if k < len(results):
                same &= bool(np.array_equal(x, results[k][1]) and res["pivots"] == results[k][0]["pivots"])
        solo_s = time.perf_counter() - t0
        for k, h1 in enumerate(ctxs):
            r, q = lpgpu.lp_get_pivots(h1)
            same &= r.tolist() == logs[k][0].tolist() and q.tolist() == logs[k][1].tolist()
    finally:
        for h1 in ctxs:
            lpgpu.lp_destroy(h1)
    n = len(lps)
    return dict(workload=f"batch of {n} dense LPs, m and n uniform on [32, 512], seed {lpgen.BATCH_SEED}",
                solves_per_s=round(n / batch_s, 1), ms_per_batch=round(1e3 * batch_s, 3),
                device_ms_per_batch=round(dev_ms / reps, 3), pivots=pivots,
                alg_gbs=round(alg / (dev_ms / reps * 1e-3) / 1e9, 1),
                one_at_a_time_solves_per_s=round(n / solo_s, 1),
                speedup_vs_one_at_a_time=round(solo_s / batch_s, 2),
                kernel_shape=shape, autotune_best_ms=round(tune_ms, 3),
                identical_to_single_lp_solver=bool(same), certificates_ok=bool(cert_ok))


class Prefetch:
    """Trace LPs generated in trace order on a pool of threads, at most
    `ahead` in flight; iterating yields (k, lp). The draws run in C with the
    interpreter lock released, so the pool keeps pace with the GPU."""

    def __init__(self, lpgen, sizes, workers, ahead, start=0, stop=None):
        from concurrent.futures import ThreadPoolExecutor

        self.lpgen, self.sizes = lpgen, sizes
        self.start, self.stop = start, len(sizes) if stop is None else stop
        self.pool = ThreadPoolExecutor(max_workers=workers)
        self.ahead = ahead

    def _gen(self, k):
        m, n = self.sizes[k]
        return self.lpgen.dense_lp(self.lpgen.TRACE_SEED, m, n, k=k)

    def __iter__(self):
        from collections import deque

        futs = deque()
        nxt = self.start
        while nxt < self.stop and len(futs) < self.ahead:
            futs.append((nxt, self.pool.submit(self._gen, nxt)))
            nxt += 1
        while futs:
            k, f = futs.popleft()
            lp = f.result()
            if nxt < self.stop:
                futs.append((nxt, self.pool.submit(self._gen, nxt)))
                nxt += 1
            yield k, lp

    def close(self):
        self.pool.shutdown(wait=True)


def bench_hybrid(args, lpgpu, lpgen):
    """The paper's CPU + GPU column split (Section IV; Tables VI-VII sweep the
    GPU's share theta) on the timed workload: one solve per theta after a
    warm-up, with the one-pivot single-GPU solve (the hybrid's GPU side runs
    the same update kernel) and theta = 1 as references."""
    lp = lpgen.workload(args.workload)
    m, n = lp.m, lp.n
    threads = host_workers()
    thetas = [float(t) for t in args.hybrid_thetas.split(",") if t]
    one = lpgpu.solve(lp.A, lp.b, lp.c, fuse_pivots=1)
    out = dict(workload=args.workload, host_threads=threads, one_pivot_single_gpu=dict(
        pivots_per_s=round(one["pivots"] / (one["solve_ms"] * 1e-3), 1), solve_ms=round(one["solve_ms"], 3)),
        sweep=[])
    for k, theta in enumerate([thetas[0]] + thetas):
        h = lpgpu.lp_hybrid_create(lp.A, lp.b, lp.c, theta, threads)
        try:
            lpgpu.lp_hybrid_solve(h)
            res, _, _ = lpgpu.lp_hybrid_get_solution(h, m, n)
            rows, cols = lpgpu.lp_hybrid_get_pivots(h)
            info = lpgpu.lp_hybrid_info(h)
        finally:
            lpgpu.lp_hybrid_destroy(h)
        if k == 0:
            continue  # warm-up
        same = rows.tolist() == one["rows"].tolist() and cols.tolist() == one["cols"].tolist()
        piv = max(res["pivots"], 1)
        out["sweep"].append(dict(theta=theta, pivots_per_s=round(res["pivots"] / (res["solve_ms"] * 1e-3), 1),
                                 solve_ms=round(res["solve_ms"], 3), host_columns=info["host_columns"],
                                 host_ms_per_pivot=round(info["host_ms"] / piv, 4),
                                 status=lpgpu.STATUS_NAMES[res["status"]], same_pivots=same))
        log(f"hybrid theta {theta}: {out['sweep'][-1]}")
    best = max(out["sweep"], key=lambda r: r["pivots_per_s"])
    out["best_theta"] = best["theta"]
    return out


def host_workers():
    """Worker threads for host-side generation: the CPU share of the box (at
    most 16), whatever the affinity mask shows."""
    return max(1, min(16, len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16") or 16)))


def bench_serve(args, lpgpu, lpgen):
    """The Poisson arrival stream of dense LPs (m, n log-uniform on [64,
    4096]) through the server, against one-at-a-time solves of the same
    trace. Every LP is generated from its index when it is needed and dropped
    after it has been handed over, so the host holds only a window of the
    trace."""
    import queue
    import resource
    import threading

    from paper_2211_10979_amd.certify import certify

    count = args.serve_lps
    sizes, gaps = lpgen.trace_sizes(lpgen.TRACE_SEED, count)
    workers = host_workers()
    tab_gb = sum(lpgpu.lp_tableau_bytes(m, n) for m, n in sizes) / (1 << 30)

    def solo(lp):
        t0 = time.perf_counter()
        h = lpgpu.lp_create(lp.A, lp.b, lp.c)
        lpgpu.lp_solve(h)
        res, x, y = lpgpu.lp_get_solution(h)
        lpgpu.lp_destroy(h)
        return time.perf_counter() - t0, res, x, y

    # one at a time over the whole trace: service times measured back to back
    log(f"serving: one-at-a-time baseline over {count} LPs ({workers} generator threads)")
    warm = Prefetch(lpgen, sizes, workers, 8, stop=min(count, 5))
    for _, lp in warm:
        solo(lp)
    warm.close()
    service = np.empty(count)
    solo_piv = np.empty(count, dtype=np.int64)
    solo_status = np.empty(count, dtype=np.int64)
    solo_x = [None] * count
    cert_ok = True
    pf = Prefetch(lpgen, sizes, workers, 4 * workers)
    for k, lp in pf:
        dt, res, x, y = solo(lp)
        service[k] = dt
        solo_piv[k] = res["pivots"]
        solo_status[k] = res["status"]
        solo_x[k] = x
        if k < 200:
            cert_ok &= bool(certify(lp.A, lp.b, lp.c, x, y, res["objective"])[0])
        if k % 2000 == 1999:
            log(f"serving: one-at-a-time {k + 1}/{count}")
    pf.close()
    c_seq = count / float(service.sum())
    lam = args.serve_load * c_seq
    arrivals = np.cumsum(gaps) / lam
    arrivals -= arrivals[0]
    # the same trace, one at a time: each LP starts at max(its arrival, the
    # previous finish)
    finish = 0.0
    lat = np.empty(count)
    for k in range(count):
        finish = max(arrivals[k], finish) + service[k]
        lat[k] = finish - arrivals[k]
    solo_makespan = finish

    def serve(arr_times, submitters, slots, budget_gb=None):
        """Submits the trace at the given times (submitter threads take LPs
        from one generator in trace order) and collects every result."""
        budget_gb = args.serve_budget_gb if budget_gb is None else budget_gb
        s = lpgpu.lp_server_create(int(budget_gb * (1 << 30)), slots)
        tickets = queue.Queue()
        mismatches = [0]
        failures = []
        try:
            pf = Prefetch(lpgen, sizes, workers, 4 * workers)
            it = iter(pf)
            lock = threading.Lock()
            t0 = time.perf_counter()

            def submitter():
                try:
                    while True:
                        with lock:
                            try:
                                k, lp = next(it)
                            except StopIteration:
                                return
                        wait = arr_times[k] - (time.perf_counter() - t0)
                        if wait > 0:
                            time.sleep(wait)
                        tickets.put((k, lpgpu.lp_server_submit(s, lp.A, lp.b, lp.c)))
                except Exception as e:  # reported after the run
                    failures.append(e)
                    tickets.put((-1, None))

            ths = [threading.Thread(target=submitter) for _ in range(submitters)]
            for th in ths:
                th.start()
            for done in range(count):
                k, t = tickets.get()
                if k < 0:
                    raise failures[0]
                m, n = sizes[k]
                res, x, _ = lpgpu.lp_server_wait(s, t, m, n)
                if res["pivots"] != solo_piv[k] or res["status"] != solo_status[k] or not np.array_equal(x, solo_x[k]):
                    mismatches[0] += 1
                if done % 2000 == 1999:
                    log(f"serving: {done + 1}/{count} results")
            span = time.perf_counter() - t0
            for th in ths:
                th.join()
            pf.close()
            st = lpgpu.lp_server_stats(s)
        finally:
            lpgpu.lp_server_destroy(s)
        return span, st, mismatches[0]

    log(f"serving: server, Poisson arrivals at {lam:.1f}/s")
    makespan, st, bad = serve(arrivals, 1, args.serve_slots)
    log("serving: server, all requests at once")
    burst_span, burst_st, burst_bad = serve(np.zeros(count), workers, max(args.serve_slots, count))
    log(f"serving: server, all requests at once under a {args.serve_tight_gb} GB budget")
    tight_span, tight_st, tight_bad = serve(np.zeros(count), workers, max(args.serve_slots, count),
                                            budget_gb=args.serve_tight_gb)
    peak_rss_gb = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / (1 << 20)
    return dict(workload=f"{count} dense LPs of the Poisson trace (m, n log-uniform on [64, 4096], seed "
                         f"{lpgen.TRACE_SEED}, {tab_gb:.1f} GB of tableaux in all), arrival rate "
                         f"{args.serve_load} x the one-at-a-time rate",
                lps=count, arrival_rate_per_s=round(lam, 1), budget_gb=args.serve_budget_gb,
                max_slots=args.serve_slots, solves_per_s=round(count / makespan, 1),
                p50_ms=round(st["p50_ms"], 3), p99_ms=round(st["p99_ms"], 3),
                peak_resident_gb=round(st["peak_bytes"] / (1 << 30), 3), ticks=st["ticks"],
                one_at_a_time_solves_per_s=round(count / solo_makespan, 1),
                one_at_a_time_service_solves_per_s=round(c_seq, 1),
                one_at_a_time_p50_ms=round(1e3 * float(np.percentile(lat, 50)), 3),
                one_at_a_time_p99_ms=round(1e3 * float(np.percentile(lat, 99)), 3),
                speedup_vs_one_at_a_time=round(solo_makespan / makespan, 3),
                saturated_solves_per_s=round(count / burst_span, 1),
                saturated_speedup_vs_one_at_a_time=round((count / burst_span) / c_seq, 3),
                saturated_p50_ms=round(burst_st["p50_ms"], 3), saturated_p99_ms=round(burst_st["p99_ms"], 3),
                saturated_max_slots=max(args.serve_slots, count),
                saturated_peak_resident_gb=round(burst_st["peak_bytes"] / (1 << 30), 3),
                tight_budget_gb=args.serve_tight_gb, tight_solves_per_s=round(count / tight_span, 1),
                tight_p50_ms=round(tight_st["p50_ms"], 3), tight_p99_ms=round(tight_st["p99_ms"], 3),
                tight_peak_resident_gb=round(tight_st["peak_bytes"] / (1 << 30), 3),
                identical_to_one_at_a_time=bool(bad == 0 and burst_bad == 0 and tight_bad == 0),
                mismatches=bad + burst_bad + tight_bad, certificates_ok_first_200=bool(cert_ok),
                peak_host_rss_gb=round(peak_rss_gb, 2), generator_threads=workers)


# ---------------------------------------------------------------- CPU legs


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def stream_triad(threads, n=1 << 26, reps=5):
    """STREAM-style triad a = b + s * c over three arrays of n doubles, split
    over `threads` threads (numpy releases the interpreter lock). Each chunk
    goes through a small cache-resident temporary, so memory traffic is the
    triad's 24 bytes per element. Best of `reps`, in GB/s."""
    from concurrent.futures import ThreadPoolExecutor

    a = np.zeros(n)
    b = np.ones(n)
    c = np.full(n, 2.0)
    step = 1 << 19
    bounds = np.linspace(0, n, threads + 1).astype(np.int64)

    def part(t):
        tmp = np.empty(step)
        for lo in range(bounds[t], bounds[t + 1], step):
            hi = min(lo + step, bounds[t + 1])
            w = tmp[: hi - lo]
            np.multiply(c[lo:hi], 3.0, out=w)
            np.add(b[lo:hi], w, out=a[lo:hi])

    best = 0.0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for _ in range(reps):
            t0 = time.perf_counter()
            list(ex.map(part, range(threads)))
            best = max(best, 24.0 * n / (time.perf_counter() - t0) / 1e9)
    return round(best, 1)


def cpu_leg_omp(args):
    """The CPU oracle's OpenMP legs, in a child process that never touches
    the GPU, run with OMP_PROC_BIND=close: the benchmark LP with all cores
    and with one, and the two small single LPs; input generation excluded."""
    import oracle
    from paper_2211_10979_amd import lpgen

    threads = host_workers()
    out = dict(cpu_model=cpu_model(), nproc=len(os.sched_getaffinity(0)), threads=threads,
               omp_proc_bind=os.environ.get("OMP_PROC_BIND"))

    def timed_solves(lp, nthreads, budget):
        """Full solves until `budget` seconds have passed (at least one)."""
        t_total, piv, solves, log0 = 0.0, 0, 0, None
        while solves == 0 or t_total < budget:
            o = oracle.OracleLP(lp.A, lp.b, lp.c, threads=nthreads)
            t0 = time.perf_counter()
            o.step(-1)
            t_total += time.perf_counter() - t0
            piv += o.pivots
            solves += 1
            if log0 is None:
                log0 = o.log()
            o.close()
        return t_total, piv, solves, log0

    lp = lpgen.workload(args.workload)
    t_all, piv, solves, olog = timed_solves(lp, threads, args.cpu_seconds)
    gpu = np.load(args.gpu_log)
    match = olog[0].tolist() == gpu["rows"].tolist() and olog[1].tolist() == gpu["cols"].tolist()
    out["value"] = piv / t_all
    out["sample"] = (f"{solves} full solve(s) of {args.workload} ({piv // solves} pivots each) on {threads} threads, "
                     f"{t_all:.1f} s, input generation excluded")
    out["solves_per_s"] = solves / t_all
    out["oracle_log_matches_gpu"] = bool(match)
    # one thread: the first pivots of the same LP, timed pivot by pivot
    o = oracle.OracleLP(lp.A, lp.b, lp.c, threads=1)
    t1 = 0.0
    while t1 < args.cpu_seconds / 3 and o.status == oracle.RUNNING:
        t0 = time.perf_counter()
        o.step(1)
        t1 += time.perf_counter() - t0
    k1 = o.pivots
    o.close()
    out["one_thread"] = dict(value=k1 / t1, unit="pivots/s", sample=f"first {k1} pivots of {args.workload}, 1 thread")
    for name in ("dense_200x200", "dense_2000x2000"):
        small = lpgen.workload(name)
        t, p, sv, _ = timed_solves(small, threads, 1.0)
        out[name] = dict(pivots_per_s=p / t, solves_per_s=sv / t, solves=sv, threads=threads)
    return out


def cpu_leg_lp(args):
    """The CPU oracle one LP per thread (single-threaded oracle, no OpenMP
    binding, so the threads spread over the cores), in a child process that
    never touches the GPU: the batch of 512 serially and in parallel, and a
    sample of the serving trace; plus the host's STREAM-style triad."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_2211_10979_amd import lpgen

    threads = host_workers()
    out = dict(triad_gbs_1_thread=stream_triad(1), triad_gbs_all=stream_triad(threads))
    bsizes = lpgen.batch_sizes(lpgen.BATCH_SEED, 512)
    blps = [lpgen.dense_lp(lpgen.BATCH_SEED, m, n, k=k) for k, (m, n) in enumerate(bsizes)]

    def one(lp1):
        o1 = oracle.OracleLP(lp1.A, lp1.b, lp1.c, threads=1)
        o1.step(-1)
        p1 = o1.pivots
        o1.close()
        return p1

    t0 = time.perf_counter()
    bp = sum(one(x) for x in blps)
    t_serial = time.perf_counter() - t0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        t0 = time.perf_counter()
        bp2 = sum(ex.map(one, blps))
        t_par = time.perf_counter() - t0
    out["batch_512"] = dict(serial_solves_per_s=512 / t_serial, lp_parallel_solves_per_s=512 / t_par,
                            pivots=bp, same_pivots=bool(bp == bp2), threads=threads)
    # the serving trace: its first LPs (the order is random, so the prefix is a
    # random sample) one per thread, until 200 LPs or the time budget
    tsizes, _ = lpgen.trace_sizes(lpgen.TRACE_SEED, 10000)
    done, t_sample = 0, 0.0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        while done < 200 and t_sample < args.cpu_seconds:
            chunk = [lpgen.dense_lp(lpgen.TRACE_SEED, m, n, k=done + i)
                     for i, (m, n) in enumerate(tsizes[done: min(200, done + threads)])]
            t0 = time.perf_counter()
            list(ex.map(one, chunk))
            t_sample += time.perf_counter() - t0
            done += len(chunk)
    rate = done / t_sample
    out["trace_estimate"] = dict(estimate=True, sample_lps=done, sample_seconds=round(t_sample, 2),
                                 solves_per_s=rate, est_seconds_for_10000=10000 / rate, threads=threads,
                                 how="the trace's first LPs, one per thread; 10,000 / their rate")
    return out


def cpu_baseline(args, gpu_log):
    """Runs the CPU legs in child processes (no GPU): the OpenMP legs with
    OMP_PROC_BIND=close, the one-LP-per-thread legs without binding."""
    import subprocess
    import tempfile

    out = {}
    with tempfile.TemporaryDirectory() as d:
        lpath = os.path.join(d, "log.npz")
        np.savez(lpath, rows=gpu_log[0], cols=gpu_log[1])
        for part, bind in (("omp", "close"), ("lp", "false")):
            opath = os.path.join(d, f"{part}.json")
            env = dict(os.environ, OMP_PROC_BIND=bind, OMP_NUM_THREADS=str(host_workers()))
            cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", part, "--cpu-out", opath, "--gpu-log",
                   lpath, "--workload", args.workload, "--cpu-seconds", str(args.cpu_seconds)]
            subprocess.run(cmd, env=env, check=True)
            with open(opath) as f:
                out.update(json.load(f))
    threads = out.pop("threads")
    return dict(value=out.pop("value"), unit="pivots/s", cores=threads, kind="oracle", sample=out.pop("sample"),
                **out)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dense_8000x8000")
    ap.add_argument("--chunk", type=int, default=0, help="pivots per graph replay (0 = library default)")
    ap.add_argument("--fuse", type=int, default=0, help="pivots per update pass (0 = library default)")
    ap.add_argument("--cols-per-block", type=int, default=0)
    ap.add_argument("--rows-per-thread", type=int, default=0)
    ap.add_argument("--time-kernels", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-lps", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--serve-lps", type=int, default=10000,
                    help="LPs of the arrival trace served (the full trace has 10000)")
    ap.add_argument("--serve-load", type=float, default=1.5, help="arrival rate / one-at-a-time solve rate")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=4096)
    ap.add_argument("--serve-tight-gb", type=float, default=0.5,
                    help="budget of a second saturated leg in which the budget binds")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--hybrid-thetas", default="1.0,0.99,0.98,0.97,0.96,0.95,0.9",
                    help="GPU shares of the CPU + GPU split to time")
    ap.add_argument("--no-hybrid", action="store_true")
    ap.add_argument("--small-steps", type=int, default=20, help="timed steps of the 200 x 200 and 2000 x 2000 legs")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--cpu-leg", default=None, choices=("omp", "lp"), help=argparse.SUPPRESS)
    ap.add_argument("--cpu-out", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--gpu-log", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run the plain copy kernel over this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.cpu_leg:  # a child process of cpu_baseline: CPU only
        out = cpu_leg_omp(args) if args.cpu_leg == "omp" else cpu_leg_lp(args)
        with open(args.cpu_out, "w") as f:
            json.dump(out, f)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(f"bench.py runs on one GPU only: the solver keeps each LP on a single device "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2211_10979_amd import lpgen, lpgpu

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lpgpu.library()  # fails loudly when the HIP library is not built

    if args.copy_calibration > 0:
        nbytes = int(args.copy_calibration * (1 << 30))
        ms = lpgpu.lp_diag_copy(nbytes, reps=5)
        print(json.dumps(dict(copy_bytes=nbytes, copy_ms=ms, copy_gbs=2 * nbytes / ms / 1e6)), flush=True)
        return

    log(f"plain solve: {args.workload}, warmup {args.warmup}, steps {args.steps}")
    plain = bench_plain(args, lpgpu, lpgen, torch)
    lp = plain.pop("lp")
    gpu_log = plain.pop("log")
    roof = plain.pop("roofline", None)
    w = lpgen.WORKLOADS[args.workload]
    line = dict(
        metric=METRIC,
        value=round(plain["value"], 2),
        unit="pivots/s",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=round(plain["ms_per_step"], 4),
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="f64",
        data="synthetic",
        config=dict(workload=args.workload, m=w["m"], n=w["n"], seed=w["seed"],
                    tableau=f"{w['m'] + 1}x{w['m'] + w['n'] + 1}", generator="A,b,c integer uniform [1,1000]",
                    pivots_per_update_pass=plain["fuse_pivots"], parallelism="single GPU"),
        roofline=roof,
        plain=plain,
    )
    if not args.no_small:
        line["small"] = {}
        for name in ("dense_200x200", "dense_2000x2000"):
            log(f"plain solve: {name}")
            sargs = argparse.Namespace(**{**vars(args), "workload": name, "steps": args.small_steps})
            r = bench_plain(sargs, lpgpu, lpgen, torch)
            r.pop("lp"), r.pop("log")
            rf = r.pop("roofline", None)
            line["small"][name] = dict(pivots_per_s=round(r["value"], 1), solves_per_s=round(r["solves_per_s"], 1),
                                       ms_per_step=round(r["ms_per_step"], 4), pivots_per_solve=r["pivots_per_solve"],
                                       status=r["status"], certificates_ok=r["certificates_ok"],
                                       update_kernel=None if rf is None else rf["kernel"],
                                       update_avg_launch_us=None if rf is None else rf["avg_launch_us"])
    if not args.no_batch:
        log(f"batched: {args.batch_lps} LPs")
        line["batched"] = bench_batch(args, lpgpu, lpgen, torch)
    if not args.no_serve:
        line["serving"] = bench_serve(args, lpgpu, lpgen)
    if not args.no_hybrid:
        log(f"hybrid: {args.workload}, theta {args.hybrid_thetas}")
        line["hybrid"] = bench_hybrid(args, lpgpu, lpgen)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle")
        line["cpu_baseline"] = cpu_baseline(args, gpu_log)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
