"""GPU tests of the serving loop: oracle parity on a mix of request sizes,
results identical alone and in the mix, admission under a small HBM budget,
failure isolation (oversize request, injected allocation failure), queue-limit
rejection and cancellation."""
import sys
import time

import numpy as np
import pytest

import oracle
import workloads as W
from _ref import check_postselected, oracle_postselected

pytestmark = pytest.mark.gpu

# (ns, m): n = 7..19.  By default every request runs alone on the grouped
# sweeps; with LDS batching on, n <= 12 (complex128) runs batched with the
# state in LDS, and with HBM batching up to 17, 14..17 batched in HBM.
MIX = [(2, 4), (3, 6), (6, 10), (4, 8), (2, 6), (5, 8), (3, 10), (6, 7), (4, 5), (5, 10), (3, 3), (6, 6),
       (7, 10), (8, 10)]


def _hs():
    import paper_2402_08136_amd as hs
    return hs


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _systems(shapes, seed0=500):
    out = []
    for i, (ns, m) in enumerate(shapes):
        A, b = W.dc_powerflow(1 << ns, seed0 + i)
        out.append((A, b, m))
    return out


def _wait_all(srv, tickets, timeout=120.0, y_counts=None):
    """Poll until every ticket is done: {ticket: (x_hat, info) or the
    error}; with y_counts ({ticket: 2^ns}) the results are (x_hat, info, y,
    p_anc1) with the raw postselected block."""
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t in res:
                continue
            try:
                r = srv.poll_ex(t, y_counts[t]) if y_counts else srv.poll(t)
            except Exception as e:     # noqa: BLE001 - failures are results here
                res[t] = e
                continue
            if r is not None:
                res[t] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.002)
    return res


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("route", ["sweeps", "lds", "lds+hbm"])
def test_serving_matches_oracle(dtype, route):
    hs = _hs()
    systems = _systems(MIX)
    opts = {"sweeps": {}, "lds": {"lds_max_qubits": -1},
            "lds+hbm": {"lds_max_qubits": -1, "batch_max_qubits": 17}}[route]
    srv = hs.Server(dtype, k_max=3, **opts)
    tickets = [srv.submit(A, b, m) for A, b, m in systems]
    res = _wait_all(srv, tickets, y_counts={t: 1 << ns for t, (ns, _) in zip(tickets, MIX)})
    worst = 0.0
    for t, (A, b, m) in zip(tickets, systems):
        ref = oracle_postselected(A, b, m)
        x_hat, info, y, p1 = res[t]
        assert p1 == info["p_anc1"]
        worst = max(worst, check_postselected(y, p1, x_hat, ref, dtype, (t, route)))
        assert float(np.dot(x_hat, ref[0]) ** 2) >= 0.999
    _say(f"serve {dtype} {route}: max|dy| vs oracle {worst:.3e}")
    st = srv.stats()
    prof = srv.profile()
    _say(f"serve {dtype}: {st} {prof}")
    assert st["done"] == len(systems) and st["failed"] == 0 and st["p50_s"] <= st["p99_s"]
    lds_limit = 12 if dtype == "c128" else 13    # states of up to 64 KiB run in LDS
    limit = {"sweeps": 0, "lds": lds_limit, "lds+hbm": 17}[route]
    n_alone = sum(ns + m + 1 > limit for ns, m in MIX)
    assert prof["alone"] == n_alone and prof["batched"] == len(systems) - n_alone
    srv.stop()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_serving_alone_equals_mix_bitwise(dtype):
    hs = _hs()
    systems = _systems(MIX, seed0=700)
    srv = hs.Server(dtype, k_max=3, streams=4, max_batch=5, lds_max_qubits=-1, batch_max_qubits=15)
    # the mix: everything at once, twice over
    tickets = [srv.submit(A, b, m) for A, b, m in systems + systems]
    mix = _wait_all(srv, tickets)
    for i, (A, b, m) in enumerate(systems):
        t = srv.submit(A, b, m)
        alone = _wait_all(srv, [t])[t]
        for tm in (tickets[i], tickets[i + len(systems)]):
            x_m, info_m = mix[tm]
            assert np.array_equal(alone[0], x_m)
            assert alone[1] == info_m
    srv.stop()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_grouped_launches_equal_single_launches_bitwise(dtype):
    """Same-shape requests that share launches (one launch per fused op for
    the whole group, each member with its own matrices) give the same bits
    as the same requests launched one at a time, and match the oracle."""
    hs = _hs()
    shapes = [(4, 10)] * 6 + [(5, 9)] * 5 + [(3, 11)]    # n = 15 (two op lists) and 15
    systems = _systems(shapes, seed0=900)
    grouped = hs.Server(dtype, k_max=3, launchers=1, group_window_us=300000)
    tickets = [grouped.submit(A, b, m) for A, b, m in systems]
    res_g = _wait_all(grouped, tickets, y_counts={t: 1 << ns for t, (ns, _) in zip(tickets, shapes)})
    prof = grouped.profile()
    grouped.stop()
    _say(f"grouped {dtype}: {prof}")
    assert prof["groups"] >= 2 and prof["grouped"] >= 6
    single = hs.Server(dtype, k_max=3, launchers=1)
    for t, (A, b, m), (ns, _) in zip(tickets, systems, shapes):
        t1 = single.submit(A, b, m)
        x1, info1, y1, _ = _wait_all(single, [t1], y_counts={t1: 1 << ns})[t1]
        xg, info_g, yg, p1g = res_g[t]
        assert np.array_equal(x1, xg) and np.array_equal(y1, yg)
        assert info1 == info_g
        check_postselected(yg, p1g, xg, oracle_postselected(A, b, m), dtype, t)
    assert single.profile()["groups"] == 0
    single.stop()


def test_admission_under_small_budget_and_oversize():
    hs = _hs()
    big = _systems([(6, 10)] * 6, seed0=900)        # 17 qubits: 2 MiB state + tables
    srv = hs.Server("c128", hbm_budget_bytes=8 << 20, k_max=3)
    tickets = [srv.submit(A, b, m) for A, b, m in big]
    res = _wait_all(srv, tickets)
    for t, (A, b, m) in zip(tickets, big):
        _, _, xh, _ = oracle.hhl_solve(A, b, m, want_state=False)
        assert float(np.dot(res[t][0], xh) ** 2) >= 0.999
    # a request that can never fit: 21 qubits = 32 MiB state
    A, b = W.dc_powerflow(256, 3)
    t = srv.submit(A, b, 12)
    r = _wait_all(srv, [t])[t]
    assert isinstance(r, hs.HHLSVError) and "OOM" in str(r)
    srv.stop()


def test_injected_allocation_failure_is_isolated():
    hs = _hs()
    systems = _systems(MIX[:6], seed0=1100)
    srv = hs.Server("c128", k_max=2, prep_threads=1, fail_alloc_at=3)
    tickets = [srv.submit(A, b, m) for A, b, m in systems]
    res = _wait_all(srv, tickets)
    failed = [t for t in tickets if isinstance(res[t], Exception)]
    assert len(failed) == 1 and failed[0] == tickets[2] and "OOM" in str(res[failed[0]])
    for t, (A, b, m) in zip(tickets, systems):
        if t in failed:
            continue
        _, _, xh, _ = oracle.hhl_solve(A, b, m, want_state=False)
        assert float(np.dot(res[t][0], xh) ** 2) >= 0.999
    st = srv.stats()
    assert st["failed"] == 1 and st["done"] == len(systems) - 1
    srv.stop()


def test_queue_limit_and_cancel():
    hs = _hs()
    A, b = W.dc_powerflow(64, 1)
    srv = hs.Server("c128", k_max=3, prep_threads=1, queue_limit=4)
    tickets, rejected = [], 0
    for _ in range(40):
        try:
            tickets.append(srv.submit(A, b, 10))
        except hs.HHLSVError as e:
            assert "BUSY" in str(e)
            rejected += 1
    assert rejected > 0 and srv.stats()["rejected"] == rejected
    cancelled = 0
    for t in tickets[::-1]:
        try:
            srv.cancel(t)
            cancelled += 1
        except hs.HHLSVError:
            pass              # already admitted: runs to completion
    res = _wait_all(srv, tickets)
    n_cancel = sum(isinstance(r, Exception) and "cancelled" in str(r) for r in res.values())
    assert n_cancel == cancelled
    assert all(not isinstance(r, Exception) or "cancelled" in str(r) for r in res.values())
    srv.stop()


_NS9 = {}


def _ns9_system():
    """A 512-bus system (511 reduced + 1 pad = 2^9: 9 system qubits) with 2
    clock qubits: n = 12, which fits in LDS at both precisions, so the
    controlled evolutions (512 columns) run through the batched kernel's
    wide gate for more columns than a workgroup has threads."""
    if not _NS9:
        A, b = W.dc_powerflow(512, 5)
        _NS9["sys"] = (A, b, 2)
        _NS9["ref"] = oracle_postselected(A, b, 2)
    return _NS9["sys"], _NS9["ref"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_nine_system_qubits_batched_and_served(dtype):
    hs = _hs()
    (A, b, m), ref = _ns9_system()
    bt = hs.Batch(dtype, 3)
    c = hs.circuit_build_hhl(A, b, m)
    assert c.n_qubits == 12 and c.info()["n_sys"] == 9
    bt.add(c)
    bt.run()
    x_hat, info = bt.solution(0)
    y, p1 = bt.postselected(0)
    err_b = check_postselected(y, p1, x_hat, ref, dtype, "batch")
    srv = hs.Server(dtype, k_max=3, lds_max_qubits=-1)
    t = srv.submit(A, b, m)
    xs, infos, ys, p1s = _wait_all(srv, [t], y_counts={t: 512})[t]
    assert srv.profile()["batched"] == 1
    srv.stop()
    err_s = check_postselected(ys, p1s, xs, ref, dtype, "served")
    _say(f"ns=9 m=2 {dtype}: max|dy| batch {err_b:.3e}, served {err_s:.3e}")
