"""GPU tests of batched persistent execution: parity with the oracle and with
the one-circuit path on a mix of shapes, LDS- and HBM-resident states,
bitwise equality alone vs in a mix, and hipGraph replay."""
import sys

import numpy as np
import pytest

import workloads as W
from _ref import AMP_TOL, check_postselected, oracle_postselected

pytestmark = pytest.mark.gpu


def _hs():
    import paper_2402_08136_amd as hs
    return hs


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# (ns, m): n = ns + m + 1 from 3 to 17; n >= 14 at c128 (>= 15 at c64) runs
# with the state in HBM.
SHAPES = [(1, 1), (1, 3), (2, 4), (3, 5), (2, 8), (4, 6), (5, 7), (6, 6), (3, 10), (6, 8), (5, 10), (6, 10)]


def _systems():
    out = []
    for i, (ns, m) in enumerate(SHAPES):
        A, b = W.dc_powerflow(max(2, 1 << ns), 300 + i) if ns > 1 else W.dc_powerflow(3, 300 + i)
        out.append((A, b, m))
    return out


TOL = AMP_TOL


def _oracle_refs(systems):
    return [oracle_postselected(A, b, m) for A, b, m in systems]


def check_instance(y, p1, x_hat, ref, dtype, what):
    return check_postselected(y, p1, x_hat, ref, dtype, what)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_batch_matches_oracle_and_single_path(k, dtype):
    hs = _hs()
    systems = _systems()
    refs = _oracle_refs(systems)
    bt = hs.Batch(dtype, k)
    circs = []
    for A, b, m in systems:
        c = hs.circuit_build_hhl(A, b, m)
        circs.append(c)
        bt.add(c)
    ms = bt.run()
    worst = 0.0
    for i, (c, ref) in enumerate(zip(circs, refs)):
        x_hat, info = bt.solution(i)
        y, p1 = bt.postselected(i)
        assert p1 == info["p_anc1"]
        worst = max(worst, check_instance(y, p1, x_hat, ref, dtype, (i, SHAPES[i])))
        # same circuit through the one-state path
        s = hs.sv_create(c.n_qubits, dtype)
        s.apply(hs.fuse(c, k))
        half = 1 << (c.n_qubits - 1)
        y1 = s.get(half, y.size)
        s.close()
        assert np.max(np.abs(y - y1)) <= TOL[dtype]
    _say(f"batch k={k} {dtype}: {len(bt)} instances in {ms:.3f} ms; max|dy| vs oracle {worst:.3e}")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_alone_equals_in_mix_bitwise(dtype):
    hs = _hs()
    systems = _systems()
    circs = [hs.circuit_build_hhl(A, b, m) for A, b, m in systems]
    mix = hs.Batch(dtype, 3)
    for c in circs:
        mix.add(c)
    # a mix with the instances in another order and duplicates
    mix2 = hs.Batch(dtype, 3)
    order = list(range(len(circs)))[::-1]
    for i in order:
        mix2.add(circs[i])
        mix2.add(circs[i])
    mix.run()
    mix2.run()
    for i, c in enumerate(circs):
        alone = hs.Batch(dtype, 3)
        alone.add(c)
        alone.run()
        xa, ia = alone.solution(0)
        xm, im = mix.solution(i)
        j = 2 * order.index(i)
        xm2, im2 = mix2.solution(j)
        assert np.array_equal(xa, xm) and np.array_equal(xa, xm2)
        assert ia == im == im2


def test_batch_graph_replay_and_growth():
    hs = _hs()
    systems = _systems()[:6]
    bt = hs.Batch("c128", 2)
    circs = [hs.circuit_build_hhl(A, b, m) for A, b, m in systems]
    for c in circs:
        bt.add(c)
    bt.run()
    first = [bt.solution(i) for i in range(len(circs))]
    for _ in range(3):
        bt.run()
        again = [bt.solution(i) for i in range(len(circs))]
        for (x0, i0), (x1, i1) in zip(first, again):
            assert np.array_equal(x0, x1) and i0 == i1
    A, b = W.dc_powerflow(16, 999)
    bt.add(hs.circuit_build_hhl(A, b, 6))
    bt.run()
    for i in range(len(circs)):
        x1, i1 = bt.solution(i)
        assert np.array_equal(first[i][0], x1) and first[i][1] == i1
    ref = _oracle_refs([(A, b, 6)])[0]
    x_new, _ = bt.solution(len(circs))
    y, p1 = bt.postselected(len(circs))
    check_instance(y, p1, x_new, ref, "c128", "added after a run")


def test_autotune_picks_a_width():
    hs = _hs()
    A, b = W.dc_powerflow(8, 5)
    c = hs.circuit_build_hhl(A, b, 5)
    k, ms = hs.svb_autotune("c128", c, copies=32)
    _say(f"autotune ns=3 m=5: best k={k}, ms per k={np.round(ms, 4).tolist()}")
    assert 1 <= k <= 5 and np.all(ms > 0)
    bt = hs.Batch("c128", 0)
    bt.add(c)
    bt.run()
    x, info = bt.solution(0)
    y, p1 = bt.postselected(0)
    check_instance(y, p1, x, _oracle_refs([(A, b, 5)])[0], "c128", "autotuned")


def test_autotune_ex_records_every_choice():
    hs = _hs()
    A, b = W.dc_powerflow(32, 6)                 # 5 system + 8 clock qubits: n = 14
    c = hs.circuit_build_hhl(A, b, 8, device_evolutions=True)
    t, ms = hs.svb_autotune_ex("c64", c, copies=24)
    _say(f"autotune_ex ns=5 m=8 c64: {t}, ms per k={np.round(ms, 4).tolist()}")
    assert 1 <= t["k_max"] <= 5 and t["tuned"] == 1 and t["ms"] > 0 and np.all(ms > 0)
    assert t["resident_kib"] in (8, 16, 32, 64, 128) and 1 <= t["group_max"] <= 256 and t["wave_target"] >= 1
    assert hs.svb_get_tune("c64", 5, 8) == dict(t, ms=0.0)


# (ns, m, dtype): a state of 128 KiB (c128 n = 13) or 128 KiB (c64 n = 14)
@pytest.mark.parametrize("ns,m,dtype", [(4, 8, "c128"), (5, 8, "c64")])
@pytest.mark.parametrize("choice", ["resident128", "groups16_wave256", "wave4096"])
def test_tuned_choices_match_oracle(ns, m, dtype, choice):
    """Each launch choice the autotuner can make, set directly, against the
    oracle: LDS residency up to 128 KiB, small groups, both wave targets."""
    hs = _hs()
    kw = {"resident128": dict(resident_kib=128), "groups16_wave256": dict(group_max=16, wave_target=256),
          "wave4096": dict(wave_target=4096)}[choice]
    systems = [W.dc_powerflow(1 << ns, 700 + i) + (m,) for i in range(20)]
    refs = _oracle_refs(systems[:3])
    try:
        hs.svb_set_tune(dtype, ns, m, k_max=4, **kw)
        bt = hs.Batch(dtype, 0)
        for A, b, mm in systems:
            bt.add(hs.circuit_build_hhl(A, b, mm, device_evolutions=True))
        items = bt.run_timed()
        kinds = {it["kind"] for it in items}
        _say(f"tuned choice {choice} ns={ns} m={m} {dtype}: items {items}")
        assert kinds == ({"batched"} if choice == "resident128" else {"swept"})
        if choice == "groups16_wave256":
            assert [it["count"] for it in items] == [16, 4]
        for i, ref in enumerate(refs):
            x_hat, _ = bt.solution(i)
            y, p1 = bt.postselected(i)
            check_instance(y, p1, x_hat, ref, dtype, (choice, i))
        bt.run()
        for i, ref in enumerate(refs):
            x_hat, _ = bt.solution(i)
            y, p1 = bt.postselected(i)
            check_instance(y, p1, x_hat, ref, dtype, (choice, "graph", i))
    finally:
        hs.svb_set_tune(dtype, ns, m)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.svb_set_tune(dtype, ns, m, resident_kib=96)


# (ns, m, dtype): a state of 64 KiB (c128 n = 12, c64 n = 13), in LDS by default
@pytest.mark.parametrize("ns,m,dtype", [(3, 8, "c128"), (4, 8, "c64")])
def test_lds_sized_state_on_sweeps_matches_oracle(ns, m, dtype):
    """The autotuner's other residency choice: a state that fits in LDS run
    through the grouped sweeps instead (residency cut at 32 KiB)."""
    hs = _hs()
    systems = [W.dc_powerflow(1 << ns, 720 + i) + (m,) for i in range(12)]
    refs = _oracle_refs(systems[:2])
    try:
        for kw, kind in ((dict(resident_kib=32), "swept"), ({}, "batched")):
            hs.svb_set_tune(dtype, ns, m, k_max=4, **kw)
            bt = hs.Batch(dtype, 0)
            for A, b, mm in systems:
                bt.add(hs.circuit_build_hhl(A, b, mm, device_evolutions=True))
            items = bt.run_timed()
            assert {it["kind"] for it in items} == {kind}
            bt.run()
            for i, ref in enumerate(refs):
                x_hat, _ = bt.solution(i)
                y, p1 = bt.postselected(i)
                check_instance(y, p1, x_hat, ref, dtype, (kind, i))
            bt.close()
    finally:
        hs.svb_set_tune(dtype, ns, m)


def test_run_timed_ops_covers_every_swept_op():
    """Per-op timing of the grouped sweeps: one entry per fused op of every
    group, in item order, on sweep kernel families; the swept results it
    leaves and the next graph run both match the oracle."""
    hs = _hs()
    systems = [W.dc_powerflow(1 << 4, 900 + i) + (8,) for i in range(6)]   # n = 13 at c128: swept
    systems += [W.dc_powerflow(1 << 2, 910 + i) + (4,) for i in range(3)]  # n = 7: batched kernel
    refs = _oracle_refs([systems[0], systems[-1]])
    bt = hs.Batch("c128", 3)
    for A, b, m in systems:
        bt.add(hs.circuit_build_hhl(A, b, m, device_evolutions=True))
    items = bt.run_timed()
    swept = [i for i, it in enumerate(items) if it["kind"] == "swept"]
    assert len(swept) == 1 and items[swept[0]]["count"] == 6
    ops = bt.run_timed_ops()
    _say(f"run_timed_ops: {len(ops)} ops, {sum(o['ms'] for o in ops):.3f} ms; items {items}")
    assert len(ops) == items[swept[0]]["ops"]
    assert {o["item"] for o in ops} == set(swept)
    assert all(o["ms"] > 0 and o["family"] != "dense_small" for o in ops)
    assert any(o["family"] == "wide" and o["controls"] >= 1 for o in ops)
    for when in ("after per-op timing", "graph"):
        for i, ref in ((0, refs[0]), (len(systems) - 1, refs[1])):
            x_hat, _ = bt.solution(i)
            y, p1 = bt.postselected(i)
            check_instance(y, p1, x_hat, ref, "c128", (when, i))
        bt.run()
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        bt.run_timed_ops(cap=1)


@pytest.mark.parametrize("ns,m,dtype", [(4, 8, "c128"), (5, 8, "c64")])
@pytest.mark.parametrize("k", [4, 5])
def test_batch_dense_gates_on_matrix_cores(ns, m, dtype, k):
    """Batch groups run every 4- and 5-qubit gate on the matrix cores, also
    with three targets inside a cache line (e.g. qubits 0..3, or 1..4 at
    complex64) where a single state takes a vector kernel; against the
    oracle, and bit for bit the same alone (a group of one) as in a group of
    four."""
    hs = _hs()
    systems = [W.dc_powerflow(1 << ns, 940 + i) + (m,) for i in range(4)]
    refs = _oracle_refs(systems[:2])
    circs = [hs.circuit_build_hhl(A, b, mm, device_evolutions=True) for A, b, mm in systems]
    line_bits = 3 if dtype == "c128" else 4   # a 128-byte line holds 8 / 16 amplitudes
    low = [q for kind, q, _ in hs.fuse(circs[0], k).gates() if kind == "dense" and len(q) == k and q[2] < line_bits]
    assert low, "the fused circuit has a gate with three targets inside a line"
    bt = hs.Batch(dtype, k)
    for c in circs:
        bt.add(c)
    bt.run()
    ops = bt.run_timed_ops()
    wide = [o for o in ops if o["family"].startswith("dense") and o["k"] >= 4]
    _say(f"batch ns={ns} m={m} {dtype} k={k}: {len(ops)} ops, dense k>=4 families "
         f"{sorted({o['family'] for o in wide})}")
    assert wide and all(o["family"] == "dense_mfma" for o in wide)
    bt.run()
    for i, ref in enumerate(refs):
        x_hat, _ = bt.solution(i)
        y, p1 = bt.postselected(i)
        check_instance(y, p1, x_hat, ref, dtype, ("mfma", k, i))
    alone = hs.Batch(dtype, k)
    alone.add(circs[0])
    alone.run()
    ya, pa = alone.postselected(0)
    yg, pg = bt.postselected(0)
    assert np.array_equal(ya, yg) and pa == pg
    alone.close()
    bt.close()


def test_batch_errors():
    hs = _hs()
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.Batch("c128", 6)
    bt = hs.Batch("c128", 2)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        bt.run()
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        bt.add(hs.circuit_create(5))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_with_device_evolutions(dtype):
    hs = _hs()
    systems = _systems()
    refs = _oracle_refs(systems)
    bt = hs.Batch(dtype, 3)
    for A, b, m in systems:
        bt.add(hs.circuit_build_hhl(A, b, m, device_evolutions=True))
    bt.run()
    for i, ref in enumerate(refs):
        x_hat, info = bt.solution(i)
        y, p1 = bt.postselected(i)
        check_instance(y, p1, x_hat, ref, dtype, (i, SHAPES[i]))
