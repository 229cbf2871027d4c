#!/usr/bin/env python3
"""Benchmark: fused-gate HBM throughput on a 33-qubit complex128 state.

Workload: the random layered circuit (40 layers of H, RZ, U3 on every qubit
then CX on a random matching; seed 2402) on 33 qubits, complex128 (128 GiB in
HBM, updated in place), fused to k_max-qubit gates.  One step = fuse the
circuit on the host + apply every fused gate (one HBM sweep each).

value = whole-job algorithmic HBM GB/s = sweeps * 2 * 2^33 * 16 B / step time.
The roofline object reports the dominant kernel family: algorithmic bytes per
launch / its mean launch time from HIP events recorded on the state's stream.
The CPU baseline times the oracle on a bounded sample of the same generator.

The HHL half of the metric is reported in the "hhl" object (skip with
--no-hhl): solves/s of the plain one-circuit-at-a-time path (64-bus system,
10 clock qubits, complex128 and complex64), of the batched persistent path
(8192 instances, 2-6 system and 4-10 clock qubits) and of the serving loop
(Poisson arrivals at 2000 req/s, 8-256 buses, 6-12 clock qubits) with p50 /
p99 latency, each for complex128 and complex64.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--k 4]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fused-gate HBM GB/s (33q SV); HHL solves/s + p99 latency, FP64 vs FP32"
HBM_PEAK_GBS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_2402_08136_amd", "csrc", f)
               for f in ("kernels.hip", "device_common.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fused_sweep_33q.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources the sweep kernels are compiled from."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(label):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    key = "bytes_per_launch " + label
    return float(vals[key]) if key in vals else None


def kernel_label(family, qubits, real="double", n=33):
    """Name of the kernel template instance a launch used (as rocprofv3 shows
    it), from its family and target qubits."""
    k = len(qubits)
    if family == "dense_direct" and real == "float" and 0 in qubits:
        return f"k_dense_pair0<{k}>"    # complex64, bit 0 a target: a pair holds two entries of a group
    if family == "dense_direct" and real == "float" and n >= 7 + k:
        return f"k_dense_pair<{k}>"     # complex64: two amplitudes per lane access
    if family == "dense_bfly" and real == "float":   # amplitude pairs, targets in bits 1..3
        return f"k_dense_bfly_pair<{k}, {sum(q < 4 for q in qubits)}>"
    if family == "dense_mfma" and real == "float" and k == 4 and 0 not in qubits and n >= k + 5:
        return f"k_dense_mfma_pair<{k}>"  # complex64 matrix cores on amplitude pairs
    if family == "dense_mfma":          # matrix cores: 5 qubits, or 4 with targets inside a line
        return f"k_dense_mfma<{real}, {k}>"
    if family == "dense_bfly":          # targets inside a 128-byte line: bits 0..2
        return f"k_dense_bfly<{k}, {sum(q < 3 for q in qubits)}>"
    name = {"dense_direct": "k_dense_direct", "dense_lds": "k_dense_lds",
            "dense_small": "k_dense_generic", "diag": "k_diag", "wide": "k_wide",
            "ucry": "k_ucry"}[family]
    return f"{name}<{real}, {k}>" if family.startswith("dense") else f"{name}<{real}>"


def cpu_baseline(budget_s=10.0, n=26):
    """Oracle (plain C, one thread) on the same layered-circuit generator at
    n qubits, unfused, gate by gate until ~budget_s of CPU time."""
    import numpy as np

    import oracle
    import workloads as W

    gates = W.layered_circuit(n, 2, 2402)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    done = 0
    t0 = time.perf_counter()
    L = oracle.lib()
    import ctypes
    for g in gates:
        q = np.asarray(g.qubits, dtype=np.int32)
        p = np.ascontiguousarray(g.params, dtype=np.float64)
        pp = p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if p.size else None
        rc = L.orc_apply_gate(psi.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              n, oracle.KIND[g.kind],
                              q.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(q), pp, p.size)
        if rc < 0:
            raise RuntimeError("oracle failed")
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    gbs = done * 2 * (1 << n) * 16 / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": 1, "host_cpu_count": os.cpu_count(),
            "kind": "oracle",
            "sample": f"first {done} unfused gates of the layered-circuit generator "
                      f"(seed 2402) at n={n} (1 GiB state), one thread, {dt:.1f} s; "
                      f"GB/s = gates * 2 * 2^n * 16 B / time"}


# ------------------------------------------------------------- HHL legs ---
# Host threads for the oracle pools: the machine's CPU share for one GPU is 16
# cores, whatever os.cpu_count() reports there.
HOST_THREADS = max(1, min(16, os.cpu_count() or 1))
AMP_BAR = {"c128": 1e-12, "c64": 2e-5}


def oracle_pool(jobs, budget_s=None, threads=HOST_THREADS):
    """FP64 oracle HHL solves of jobs [(key, A, b, m)] on a pool of host
    threads (the C oracle runs outside the GIL), one solve per thread at a
    time.  With budget_s no job starts after that much wall time.  Returns
    ({key: (x_hat, info, y, psi)}, wall seconds)."""
    import concurrent.futures as cf

    import oracle

    def solve(A, b, m):
        psi, _, xh, info = oracle.hhl_solve(A, b, m)
        half = 1 << (info["n"] - 1)
        return xh, info, psi[half:half + (1 << info["ns"])].copy(), psi

    out = {}
    t0 = time.perf_counter()
    it = iter(jobs)
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        running = {}

        def start_next():
            if budget_s is not None and time.perf_counter() - t0 > budget_s:
                return False
            job = next(it, None)
            if job is None:
                return False
            key, A, b, m = job
            running[ex.submit(solve, A, b, m)] = key
            return True

        for _ in range(threads):
            if not start_next():
                break
        while running:
            done, _ = cf.wait(list(running), return_when=cf.FIRST_COMPLETED)
            for f in done:
                out[running.pop(f)] = f.result()
                start_next()
    return out, time.perf_counter() - t0


def result_errors(pairs, dtype):
    """Errors of library results against the FP64 oracle: pairs of
    ((y, p1, x_hat), (x_hat_ref, info_ref, y_ref, psi_ref)).  y is the
    postselected block (ancilla 1, clock 0), p1 = P(ancilla = 1)."""
    dy, dp1, fid = 0.0, 0.0, 1.0
    for (y, p1, xh), (xh_ref, info_ref, y_ref, _) in pairs:
        dy = max(dy, float(np.max(np.abs(np.asarray(y) - y_ref))))
        dp1 = max(dp1, abs(p1 - info_ref["p1"]))
        fid = min(fid, float(np.dot(xh, xh_ref)) ** 2)
    return {"checked": len(pairs), "max_abs_dy": dy, "max_abs_dp_anc1": dp1,
            "min_fidelity_vs_oracle": fid, "bar": AMP_BAR[dtype],
            "within_bar": bool(dy <= AMP_BAR[dtype] and dp1 <= AMP_BAR[dtype])}


def cpu_solves(n_done, wall, sample):
    return {"value": round(n_done / wall, 2) if wall > 0 else None, "unit": "solves/s",
            "cores": HOST_THREADS, "host_cpu_count": os.cpu_count(), "kind": "oracle",
            "sample": f"{n_done} FP64 oracle HHL solves ({sample}), one solve per host thread, "
                      f"{wall:.1f} s wall"}


def _y_of(s, c, ns, dtype):
    """Postselected block of a state: psi[2^{n-1} + s] for s < 2^ns."""
    return s.get(1 << (c.n_qubits - 1), 1 << ns).astype(np.complex128)


def hhl_plain_4bus(hs, W, seeds=100):
    """The 4-bus, 4-clock-qubit solve (7 qubits, unfused) on the plain
    one-circuit-at-a-time path, complex128 and complex64, over seeded
    systems; every full state against the oracle's."""
    systems = [W.dc_powerflow(4, sd) for sd in range(seeds)]
    refs, wall = oracle_pool([(i, A, b, 4) for i, (A, b) in enumerate(systems)])
    out = {"systems": seeds, "cpu_baseline": cpu_solves(len(refs), wall, f"4-bus, m=4, seeds 0..{seeds - 1}")}
    for dtype in ("c128", "c64"):
        circs = [hs.circuit_build_hhl(A, b, 4) for A, b in systems]
        dpsi, pairs = 0.0, []
        t0 = time.perf_counter()
        for i, (c, (A, b)) in enumerate(zip(circs, systems)):
            s = hs.sv_create(c.n_qubits, dtype)
            s.apply(c)
            x_hat, info = s.postselect_solution(c, b.size)
            psi = s.get().astype(np.complex128)
            s.close()
            dpsi = max(dpsi, float(np.max(np.abs(psi - refs[i][3]))))
            half = 1 << (c.n_qubits - 1)
            pairs.append(((psi[half:half + 4], info["p_anc1"], x_hat), refs[i]))
        dt = time.perf_counter() - t0
        err = result_errors(pairs, dtype)
        err["max_abs_dpsi_full_state"] = dpsi
        out[dtype] = {"solves_per_s": round(seeds / dt, 1), "error_vs_oracle": err}
    return out


def hhl_single(hs, W, reps=40):
    """Plain one-circuit-at-a-time path on the 64-bus, 10-clock-qubit system
    (17 qubits): reset + apply (cached hipGraph) + postselect per solve, at
    every fusion width k = 1..5, complex128 and complex64; each result's full
    state against the FP64 oracle's.  Seeds 1..9 add error checks at k = 4."""
    seeds = list(range(10))
    systems = {sd: W.dc_powerflow(64, sd) for sd in seeds}
    refs, wall = oracle_pool([(sd, A, b, 10) for sd, (A, b) in systems.items()])
    A, b = systems[0]
    c = hs.circuit_build_hhl(A, b, 10)
    xs = np.linalg.solve(A, b)
    out = {"cpu_baseline": cpu_solves(len(refs), wall, "64-bus, m=10, seeds 0..9")}
    for dtype in ("c128", "c64"):
        by_k, best = {}, None
        for k in (1, 2, 3, 4, 5):
            run = hs.fuse(c, k)
            s = hs.sv_create(c.n_qubits, dtype)
            s.apply(run)
            s.postselect_solution(c, 63)
            t0 = time.perf_counter()
            for _ in range(reps):
                s.reset()
                s.apply(run)
                s.postselect_solution(c, 63)
            dt = (time.perf_counter() - t0) / reps
            x_hat, info = s.postselect_solution(c, 63)
            psi = s.get().astype(np.complex128)
            s.close()
            half = 1 << (c.n_qubits - 1)
            err = result_errors([((psi[half:half + 64], info["p_anc1"], x_hat), refs[0])], dtype)
            err["max_abs_dpsi_full_state"] = float(np.max(np.abs(psi - refs[0][3])))
            by_k[str(k)] = {"solves_per_s": round(1.0 / dt, 1), "ms_per_solve": round(dt * 1e3, 4),
                            "fused_ops": run.n_gates, "error_vs_oracle": err}
            if best is None or dt < best[1]:
                best = (k, dt, x_hat, info)
        k, dt, x_hat, info = best
        x = hs.sv_solution_x(x_hat, info)
        # the other seeds at k = 4
        pairs = []
        for sd in seeds[1:]:
            As, bs = systems[sd]
            cs = hs.circuit_build_hhl(As, bs, 10)
            s = hs.sv_create(cs.n_qubits, dtype)
            s.apply(hs.fuse(cs, 4))
            xh, inf = s.postselect_solution(cs, 63)
            y = _y_of(s, cs, 6, dtype)
            s.close()
            pairs.append(((y, inf["p_anc1"], xh), refs[sd]))
        out[dtype] = {"solves_per_s": round(1.0 / dt, 1), "ms_per_solve": round(dt * 1e3, 4), "k_max": k,
                      "fidelity_vs_Ainv_b": float(np.dot(x_hat, xs / np.linalg.norm(xs)) ** 2),
                      "rel_err_vs_Ainv_b": float(np.linalg.norm(x - xs) / np.linalg.norm(xs)),
                      "by_k": by_k, "seeds_1_9_k4_error_vs_oracle": result_errors(pairs, dtype)}
    return out


def hhl_batch(hs, W, count=8192):
    """Batched persistent path on the 8192-instance mix (seed 8136); one
    autotuned k_max per (ns, m) shape; device time of the replayed graph.
    The first instance of every (ns, m) shape (a stratified sample: shapes
    are drawn uniformly) is checked against the FP64 oracle."""
    specs = W.batch_specs(count, 8136)
    t0 = time.perf_counter()
    circs, systems = [], []
    for ns, m, gseed in specs:
        A, b = W.dc_powerflow(1 << ns, gseed)
        systems.append((A, b, m))
        circs.append(hs.circuit_build_hhl(A, b, m, device_evolutions=True))
    build_s = time.perf_counter() - t0
    first = {}
    for i, (ns, m, _) in enumerate(specs):
        first.setdefault((ns, m), i)
    refs, wall = oracle_pool([(i, *systems[i]) for i in sorted(first.values())])
    out = {"instances": count, "host_build_s": round(build_s, 2),
           "cpu_baseline": cpu_solves(len(refs), wall, "the first instance of each of the "
                                      f"{len(first)} (ns, m) shapes of the mix")}
    flop = sum(m * 2 ** (ns + m + 1 + 3 + ns) for ns, m, _ in specs)
    out["controlled_evolution_flop_per_batch"] = flop
    out["controlled_evolution_flop_note"] = (
        "the circuit's 2m controlled e^{iAt2^j} products as written (8 flop per complex multiply-add, "
        "half the state each); where fusion merges them into MUX gates the device runs 7/12 (three "
        "into a MUX3) or 3/4 (two into a MUX2) of that")
    shapes, counts = {}, {}
    for (ns, m, _), c in zip(specs, circs):
        shapes.setdefault((ns, m), c)
        counts[(ns, m)] = counts.get((ns, m), 0) + 1
    for dtype in ("c128", "c64"):
        # every launch choice per shape, tuned on as many copies of a sample
        # instance as the batch holds of that shape
        t0 = time.perf_counter()
        tuned = {}
        for (ns, m), c in sorted(shapes.items()):
            t, _ = hs.svb_autotune_ex(dtype, c, counts[(ns, m)])
            tuned[f"{ns},{m}"] = {"k": t["k_max"], "group_max": t["group_max"], "wave_target": t["wave_target"],
                                  "resident_kib": t["resident_kib"], "ms": round(t["ms"], 4)}
        tune_s = time.perf_counter() - t0
        bt = hs.Batch(dtype, 0)
        for c in circs:
            bt.add(c)
        t0 = time.perf_counter()
        bt.run()      # upload, device evolution tables, capture, run
        setup_s = time.perf_counter() - t0
        runs = [bt.run() for _ in range(5)]
        ms = float(np.median(runs))
        # where the device time goes: the same launches one work item after
        # another, each timed with HIP events (batched-kernel size classes
        # and groups of same-shape instances run through the sweep kernels)
        items = bt.run_timed()
        breakdown = {}
        for it in items:
            key = f"{it['kind']} n={it['n']}"
            e = breakdown.setdefault(key, {"items": 0, "instances": 0, "ms": 0.0, "ops_per_instance": 0})
            e["items"] += 1
            e["instances"] += it["count"]
            e["ms"] = round(e["ms"] + it["ms"], 3)
            e["ops_per_instance"] = max(e["ops_per_instance"], it["ops"])
        # the grouped sweeps op by op, by kernel family: algorithmic bytes
        # (each amplitude read and written once; a wide gate with c controls
        # only the 1 - 2^-c of the state where they are not all 0) and the
        # gate's complex multiply-adds on those amplitudes
        amp = 16 if dtype == "c128" else 8
        by_family = {}
        for op in bt.run_timed_ops():
            it = items[op["item"]]
            touched = it["count"] * 2 ** it["n"] * (1.0 - 0.5 ** op["controls"] if op["controls"] else 1.0)
            fam = op["family"]
            key = f"{fam} k={op['k']}" + {0: "", 1: " controlled", 2: " two controls (MUX2)",
                                           3: " three controls (MUX3)"}[op["controls"]]
            e = by_family.setdefault(key, {"launches": 0, "ms": 0.0, "bytes": 0.0, "flop": 0.0})
            e["launches"] += 1
            e["ms"] += op["ms"]
            e["bytes"] += 2 * amp * touched
            if fam.startswith("dense") or fam == "wide":
                e["flop"] += 8 * 2 ** op["k"] * touched
        bt.run()
        for e in by_family.values():
            sec = e["ms"] * 1e-3
            e["GBps"] = round(e.pop("bytes") / sec / 1e9, 1) if sec > 0 else None
            op_flop = e.pop("flop")
            e["TFLOPs"] = round(op_flop / sec / 1e12, 2) if op_flop and sec > 0 else None
            e["ms"] = round(e["ms"], 3)
        pairs = []
        for i in sorted(first.values()):
            y, p1 = bt.postselected(i)
            xh, _ = bt.solution(i)
            pairs.append(((y, p1, xh), refs[i]))
        out[dtype] = {"solves_per_s": round(count / (ms * 1e-3), 1), "device_ms": round(ms, 3),
                      "controlled_evolution_TFLOPs": round(flop / (ms * 1e-3) / 1e12, 2),
                      "first_run_s": round(setup_s, 3), "autotune_s": round(tune_s, 2),
                      "tuned_by_shape": tuned, "error_vs_oracle": result_errors(pairs, dtype),
                      "eager_item_breakdown": {"sum_ms": round(sum(it["ms"] for it in items), 3),
                                               "by_kind_and_qubits": breakdown},
                      "swept_ops_by_family": dict(sorted(by_family.items(), key=lambda kv: -kv[1]["ms"]))}
        bt.close()
    return out


def _serve_run(hs, sched, pool, pool_per_size, dtype, budget_bytes=0, sample_every=0):
    """Submit the schedule open loop; drain; stats; the results of every
    sample_every-th request (polled after the drain)."""
    srv = hs.Server(dtype, hbm_budget_bytes=budget_bytes)
    t_start = time.perf_counter()
    rejected = 0
    tickets = [None] * len(sched)
    for i, (ta, ns, m, _) in enumerate(sched):
        delay = t_start + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        A, b = pool[ns][i % pool_per_size]
        try:
            tickets[i] = srv.submit(A, b, m)
        except hs.HHLSVError:
            rejected += 1
    srv.drain()
    st = srv.stats()
    prof = srv.profile()
    res = {}
    if sample_every:
        for i in range(0, len(sched), sample_every):
            if tickets[i] is not None:
                ns = sched[i][1]
                xh, info, y, p1 = srv.poll_ex(tickets[i], 1 << ns)
                res[i] = (y, p1, xh)
    srv.stop()
    return {"p50_ms": round(st["p50_s"] * 1e3, 3), "p99_ms": round(st["p99_s"] * 1e3, 3),
            "solves_per_s": round(st["solves_per_s"], 1), "done": st["done"],
            "failed": st["failed"], "rejected": st["rejected"] + rejected,
            "mean_phase_ms": {k: round(prof[k] * 1e3, 4) for k in
                              ("queue_s", "prep_s", "upload_s", "ready_wait_s", "gpu_s")},
            "grouped_launches": int(prof["groups"]), "requests_in_groups": int(prof["grouped"])}, res


def hhl_serve(hs, W, seconds, rate=2000.0, pool_per_size=48, constrained_seconds=10.0,
              oracle_budget_s=12.0, max_check_qubits=19):
    """Serving loop under open-loop Poisson arrivals (seed 2000 for arrivals,
    2001 for sizes); request systems come from a pool of seeded systems per
    size.  Latency = submit to finish inside the server.  Each precision's
    measured window follows a 2 s warm-up window of other arrivals.  1% of the requests
    (every 100th) are polled for their postselected block; a time-boxed
    subset of those, taken round robin over the system sizes, is checked
    against the FP64 oracle.  A shorter run with a 256 MiB HBM budget forces
    admission waits."""
    sched = W.serve_specs(rate, seconds, 2000, 2001)
    pool = {}
    for ns in range(3, 9):
        pool[ns] = [W.dc_powerflow(1 << ns, 50000 + 100 * ns + i) for i in range(pool_per_size)]
    # a 2 s warm-up window (other seeds, not counted) before each measured
    # run: the first requests of a process load the kernels they use, which
    # moved the measured p50 by up to 2x from run to run
    warm = W.serve_specs(rate, 2.0, 7, 8)
    out = {"offered_rate_per_s": rate, "duration_s": seconds, "requests": len(sched),
           "warmup_requests_per_dtype": len(warm)}
    results = {}
    for dtype in ("c128", "c64"):
        _serve_run(hs, warm, pool, pool_per_size, dtype)
        out[dtype], results[dtype] = _serve_run(hs, sched, pool, pool_per_size, dtype, sample_every=100)
        log(f"[bench] serve {dtype}: {out[dtype]}")
    # oracle check: round robin over ns strata of the 1% sample
    strata = {}
    for i in sorted(results["c128"]):
        ta, ns, m, _ = sched[i]
        if ns + m + 1 <= max_check_qubits and i in results["c64"]:
            strata.setdefault(ns, []).append(i)
    order = []
    while any(strata.values()):
        for ns in sorted(strata):
            if strata[ns]:
                order.append(strata[ns].pop(0))
    jobs = [(i, *pool[sched[i][1]][i % pool_per_size], sched[i][2]) for i in order]
    refs, wall = oracle_pool(jobs, budget_s=oracle_budget_s)
    checked = sorted(refs)
    for dtype in ("c128", "c64"):
        out[dtype]["error_vs_oracle"] = result_errors([(results[dtype][i], refs[i]) for i in checked], dtype)
        out[dtype]["error_vs_oracle"]["sample"] = (
            f"{len(checked)} of the {len(results[dtype])} polled requests (every 100th), round robin over "
            f"ns = {sorted({sched[i][1] for i in checked})}, states of <= {max_check_qubits} qubits")
    out["cpu_baseline"] = cpu_solves(len(refs), wall, f"served requests of <= {max_check_qubits} qubits, "
                                     "round robin over the system sizes")
    # constrained HBM budget: admission waits for memory
    sched_c = W.serve_specs(rate, constrained_seconds, 2000, 2001)
    out["constrained_256MiB"] = {"duration_s": constrained_seconds, "requests": len(sched_c)}
    for dtype in ("c128", "c64"):
        out["constrained_256MiB"][dtype], _ = _serve_run(hs, sched_c, pool, pool_per_size, dtype,
                                                         budget_bytes=256 << 20)
        log(f"[bench] serve {dtype}, 256 MiB budget: {out['constrained_256MiB'][dtype]}")
    # the plain one-circuit-at-a-time FP64 path on a sample of the same requests
    sample = sched[:: max(1, len(sched) // 200)]
    t0 = time.perf_counter()
    for i, (ta, ns, m, _) in enumerate(sample):
        A, b = pool[ns][i % pool_per_size]
        c = hs.circuit_build_hhl(A, b, m, device_evolutions=True)
        st = hs.sv_create(c.n_qubits, "c128")
        st.apply(hs.fuse(c, 3))
        st.postselect_solution(c, A.shape[0])
        st.close()
    out["plain_fp64_path_solves_per_s"] = round(len(sample) / (time.perf_counter() - t0), 1)
    return out


def pf_newton_leg(hs, W):
    """Newton-Raphson AC power flow with HHL inner solves on synthetic 14- and
    30-bus cases (dilated Jacobian systems, 9 clock qubits)."""
    import numpy as np

    out = {}
    for nb, seed in ((14, 0), (30, 3)):
        case = W.ac_powerflow_case(nb, seed)
        t0 = time.perf_counter()
        vm, va, info = hs.pf_newton(case, 9, mode="dilate", k_max=3, max_iter=40, tol=1e-9,
                                    device_evolutions=True)
        wall = time.perf_counter() - t0
        out[f"{nb}_bus"] = {"unknowns": info["n_unknowns"], "iterations": info["iterations"],
                            "converged": info["converged"], "final_mismatch": info["mismatch"],
                            "wall_s": round(wall, 4), "hhl_s": round(info["hhl_seconds"], 4),
                            "min_voltage": round(float(np.min(vm)), 6)}
        log(f"[bench] power flow {nb}-bus: {out[f'{nb}_bus']}")
    return out


def c64_sweep(hs, circ, n, k, warmup, steps, probe_idx, ref_amps):
    """The same circuit on a complex64 state (half the bytes per sweep): one
    warm-up application and `steps` timed ones, then the largest difference
    from the complex128 state after as many applications (ref_amps, None if
    that state was not sampled) over a seeded sample of amplitudes."""
    import numpy as np

    log(f"[bench] complex64: allocating {8 * 2 ** n / 2 ** 30:.0f} GiB state")
    s = hs.sv_create(n, "c64")
    bps = 2 * (1 << n) * 8
    for _ in range(warmup):
        s.apply(hs.fuse(circ, k))
    s.synchronize()
    t0 = time.perf_counter()
    ms_l, fam_l, qsets = [], [], []
    for _ in range(steps):
        fused = hs.fuse(circ, k)
        ms, fam = s.apply_timed(fused)
        ms_l.append(ms)
        fam_l.append(fam)
        qsets += [tuple(g[1]) for g in fused.gates()]
    s.synchronize()
    elapsed = time.perf_counter() - t0
    ms_all, fam_all = np.concatenate(ms_l), np.concatenate(fam_l)
    rate = bps / (ms_all * 1e-3) / 1e9
    labels = np.array([kernel_label(hs.KERNEL_FAMILY[int(f)], q, "float", n) for f, q in zip(fam_all, qsets)])
    fams = {}
    for lab in np.unique(labels):
        sel = labels == lab
        fams[str(lab)] = {"total_ms": round(float(ms_all[sel].sum()), 2), "launches": int(sel.sum()),
                          "mean_ms": round(float(ms_all[sel].mean()), 3),
                          "GBps": round(bps / (float(ms_all[sel].mean()) * 1e-3) / 1e9, 1)}
    dom = max(fams, key=lambda f: fams[f]["total_ms"])
    diff = (float(np.max(np.abs(s.get_at(probe_idx).astype(np.complex128) - ref_amps)))
            if ref_amps is not None else None)
    out = {"value_GBps": round(len(ms_all) * bps / elapsed / 1e9, 2), "bytes_per_sweep": bps,
           "sweeps": len(ms_all),
           "per_sweep_GBps": {"min": round(float(rate.min()), 1), "median": round(float(np.median(rate)), 1),
                              "max": round(float(rate.max()), 1)},
           "kernel_families": fams,
           "dominant": {"kernel": dom, "GBps": fams[dom]["GBps"],
                        "frac_of_hbm_peak": round(fams[dom]["GBps"] / HBM_PEAK_GBS, 4)},
           "max_abs_diff_vs_complex128": diff, "sampled_amplitudes": int(probe_idx.size),
           "max_abs_amplitude_sampled": float(np.max(np.abs(ref_amps))) if ref_amps is not None else None,
           "applications_compared": warmup + steps,
           "final_norm2": s.norm2()}
    s.close()
    log(f"[bench] complex64: {out['value_GBps']:.0f} GB/s, max |c64 - c128| {diff}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--k", type=int, default=4, help="fusion width k_max (1..5)")
    ap.add_argument("--n", type=int, default=33, help="qubits (the workload is 33)")
    ap.add_argument("--layers", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hhl", action="store_true", help="skip the HHL solves/s part")
    ap.add_argument("--no-k-sweep", action="store_true",
                    help="skip the per-sweep rates at the other fusion widths")
    ap.add_argument("--no-c64", action="store_true",
                    help="skip the complex64 run of the same circuit")
    ap.add_argument("--k-sweep-layers", type=int, default=10,
                    help="layers of the circuit used for the per-k sweep rates")
    ap.add_argument("--part", choices=["all", "single", "batch", "serve", "powerflow"], default="all",
                    help="run one HHL leg alone (for profiling); prints that leg's JSON, not the bench line")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson arrival window")
    ap.add_argument("--serve-constrained-seconds", type=float, default=5.0,
                    help="length of the arrival window of the 256 MiB HBM-budget run")
    ap.add_argument("--c64-steps", type=int, default=2,
                    help="timed steps of the complex64 run of the same circuit (after one warm-up step)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import paper_2402_08136_amd as hs
    import workloads as W

    if args.part != "all":
        leg = {"single": lambda: {"plain_4bus_m4": hhl_plain_4bus(hs, W), "single_64bus_m10": hhl_single(hs, W)},
               "batch": lambda: hhl_batch(hs, W),
               "serve": lambda: hhl_serve(hs, W, args.serve_seconds,
                                          constrained_seconds=args.serve_constrained_seconds),
               "powerflow": lambda: pf_newton_leg(hs, W)}[args.part]
        print(json.dumps({"part": args.part, "result": leg()}), flush=True)
        return

    n, k = args.n, args.k
    log(f"[bench] building {args.layers}-layer circuit on {n} qubits")
    circ = hs.circuit_from_gates(n, W.layered_circuit(n, args.layers, 2402))
    log(f"[bench] allocating {16 * 2 ** n / 2 ** 30:.0f} GiB state")
    state = hs.sv_create(n, "c128")
    bytes_per_sweep = 2 * (1 << n) * 16

    # seeded sample of amplitudes, for the complex64 run of the same circuit:
    # taken after as many applications as that run makes (one warm-up plus
    # its timed steps), outside the timed region
    probe_idx = np.random.default_rng(2402).integers(0, 1 << n, size=65536, dtype=np.uint64)
    c64_apps = 1 + args.c64_steps
    ref_amps = None
    for w in range(args.warmup):
        t = time.perf_counter()
        state.apply(hs.fuse(circ, k))
        state.synchronize()
        log(f"[bench] warmup {w}: {time.perf_counter() - t:.2f} s")
        if w + 1 == c64_apps:
            ref_amps = state.get_at(probe_idx)

    state.synchronize()
    t0 = time.perf_counter()
    launch_ms, families = [], []
    n_sweeps = 0
    for st in range(args.steps):
        fused = hs.fuse(circ, k)
        ms, fam = state.apply_timed(fused)
        launch_ms.append(ms)
        families.append(fam)
        n_sweeps += fused.n_gates
        log(f"[bench] step {st}: {fused.n_gates} sweeps, {ms.sum() / 1e3:.2f} s device")
    state.synchronize()
    elapsed = time.perf_counter() - t0
    norm = state.norm2()
    if ref_amps is None and args.warmup + args.steps == c64_apps:
        ref_amps = state.get_at(probe_idx)
    # achievable bandwidth: in-place read and write-back with the sweeps'
    # access shape, on the same state (left unchanged)
    probe_ms = float(np.median(state.stream_probe(5)))
    achievable = bytes_per_sweep / (probe_ms * 1e-3) / 1e9

    ms_all = np.concatenate(launch_ms)
    fam_all = np.concatenate(families)
    qsets = [tuple(g[1]) for g in fused.gates()] * args.steps
    value = n_sweeps * bytes_per_sweep / elapsed / 1e9
    per_sweep = bytes_per_sweep / (ms_all * 1e-3) / 1e9
    by_fam = {}
    labels = np.array([kernel_label(hs.KERNEL_FAMILY[int(f)], q, "double", n) for f, q in zip(fam_all, qsets)])
    for lab in np.unique(labels):
        sel = labels == lab
        by_fam[str(lab)] = (float(ms_all[sel].sum()), int(sel.sum()), float(ms_all[sel].mean()))
    dom = max(by_fam, key=lambda f: by_fam[f][0])
    dom_avg_ms = by_fam[dom][2]
    achieved = bytes_per_sweep / (dom_avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"random layered circuit, {n} qubits, complex128 state "
                        f"({16 * 2 ** n / 2 ** 30:.0f} GiB in place), {args.layers} layers, "
                        f"seed 2402, fused to k_max={k}",
            "n_qubits": n, "layers": args.layers, "k_max": k,
            "sweeps_per_step": n_sweeps // max(1, args.steps),
            "bytes_per_sweep": bytes_per_sweep,
            "per_sweep_GBps": {"min": round(float(per_sweep.min()), 1),
                               "median": round(float(np.median(per_sweep)), 1),
                               "max": round(float(per_sweep.max()), 1)},
            "kernel_families": {f: {"total_ms": round(v[0], 2), "launches": v[1],
                                    "mean_ms": round(v[2], 3),
                                    "GBps": round(bytes_per_sweep / (v[2] * 1e-3) / 1e9, 1)}
                                for f, v in by_fam.items()},
            "final_norm2": norm,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "achievable": round(achievable, 1),
            "frac_of_achievable": round(achieved / achievable, 4),
            "achievable_probe": "median of 5 launches of sv_stream_probe (in-place read and write-back "
                                "of the same state with the dense sweeps' access shape, grid and XCD slices)",
        },
    }
    if not args.no_k_sweep:
        # per-sweep rates at every fusion width on a shorter circuit of the
        # same generator (the rate of a sweep does not depend on the depth)
        by_k = {str(k): {"sweeps": n_sweeps // max(1, args.steps),
                         "median_GBps": round(float(np.median(per_sweep)), 1),
                         "min_GBps": round(float(per_sweep.min()), 1),
                         "max_GBps": round(float(per_sweep.max()), 1), "layers": args.layers}}
        short = hs.circuit_from_gates(n, W.layered_circuit(n, args.k_sweep_layers, 2402))
        for kk in (2, 3, 4, 5):
            if kk == k:
                continue
            fk = hs.fuse(short, kk)
            msk, _ = state.apply_timed(fk)
            rate = bytes_per_sweep / (msk * 1e-3) / 1e9
            by_k[str(kk)] = {"sweeps": fk.n_gates, "median_GBps": round(float(np.median(rate)), 1),
                             "min_GBps": round(float(rate.min()), 1), "max_GBps": round(float(rate.max()), 1),
                             "layers": args.k_sweep_layers}
            log(f"[bench] k={kk}: {fk.n_gates} sweeps, median {np.median(rate):.0f} GB/s")
        out["config"]["per_sweep_GBps_by_k"] = dict(sorted(by_k.items()))
    state.close()
    if not args.no_c64:
        out["complex64_sweep"] = c64_sweep(hs, circ, n, k, 1, args.c64_steps, probe_idx, ref_amps)
    if not args.no_hhl:
        log("[bench] HHL: one-circuit-at-a-time path")
        hhl = {"plain_4bus_m4": hhl_plain_4bus(hs, W), "single_64bus_m10": hhl_single(hs, W)}
        log("[bench] HHL: batched 8192 instances")
        hhl["batch_8192"] = hhl_batch(hs, W)
        log(f"[bench] HHL: serving, {args.serve_seconds:.0f} s of arrivals at 2000/s")
        hhl["serve"] = hhl_serve(hs, W, args.serve_seconds, constrained_seconds=args.serve_constrained_seconds)
        log("[bench] HHL: Newton-Raphson AC power flow")
        hhl["power_flow_newton"] = pf_newton_leg(hs, W)
        out["hhl"] = hhl
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
