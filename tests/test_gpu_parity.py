"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, on the
same seeded inputs, element by element over the full state.

Bars: complex128 max |delta amplitude| <= 1e-12, complex64 <= 2e-5.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 2e-5}


def _hs():
    import paper_2402_08136_amd as hs
    return hs


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(n, gates, psi0, dtype, k=None):
    """Apply through the C-ABI on a fresh state initialised to psi0."""
    hs = _hs()
    c = hs.circuit_from_gates(n, gates)
    run = hs.fuse(c, k) if k else c
    s = hs.sv_create(n, dtype)
    s.set(psi0)
    s.apply(run)
    out = s.get()
    s.close()
    return out


# ------------------------------------------------------ random circuits ---
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,seed", [(1, 0), (3, 1), (5, 2), (7, 3), (11, 4), (13, 5)])
@pytest.mark.parametrize("k", [None, 1, 2, 3, 4, 5])
def test_random_circuit_parity(n, seed, k, dtype):
    _say(f"random circuit n={n} seed={seed} k={k} dtype={dtype}")
    gates = W.random_circuit(n, 40, seed, kmax=min(5, n))
    psi0 = W.random_state(n, seed)
    want = oracle.apply_circuit(psi0, n, gates)
    got = run_gpu(n, gates, psi0, dtype, k if k is None or k <= n else n)
    assert np.max(np.abs(got - want)) <= TOL[dtype]


# ----------------------------------------- tiled kernel target patterns ---
def _targets(pattern, k, n, rng):
    if pattern == "low":
        return sorted(rng.choice(6, size=k, replace=False).tolist())
    if pattern == "high":
        return sorted(rng.choice(np.arange(6, n), size=k, replace=False).tolist())
    if pattern == "adjacent":
        q0 = int(rng.integers(0, n - k + 1))
        return list(range(q0, q0 + k))
    if pattern == "spread":
        return sorted(set(np.linspace(0, n - 1, k).astype(int).tolist()))
    if pattern == "midline":
        # targets in bits 3..5 (inside a lane run, outside a cache line)
        lo = rng.choice(np.arange(3, 6), size=min(3, max(1, k // 2)), replace=False).tolist()
        hi = rng.choice(np.arange(6, n), size=k - len(lo), replace=False).tolist()
        return sorted(lo + hi)
    # mixed: at least one low and one high
    lo = rng.choice(6, size=max(1, k // 2), replace=False).tolist()
    hi = rng.choice(np.arange(6, n), size=k - len(lo), replace=False).tolist()
    return sorted(lo + hi)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("pattern", ["low", "high", "mixed", "adjacent", "spread", "midline"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("n", [12, 15])
def test_dense_gate_target_patterns(n, k, pattern, dtype):
    rng = np.random.default_rng(1000 * n + 10 * k + len(pattern))
    qs = _targets(pattern, k, n, rng)
    if pattern == "mixed" and k == 1:
        qs = [int(rng.integers(0, n))]
    kk = len(qs)
    U = W.random_unitary(1 << kk, rng)
    # shuffle the qubit list so the matrix index order is not the sorted order
    perm = rng.permutation(kk)
    qs_list = [qs[i] for i in perm]
    g = W.Gate("dense", tuple(qs_list), np.ascontiguousarray(U).view(np.float64).ravel())
    _say(f"dense n={n} targets={qs_list} dtype={dtype}")
    psi0 = W.random_state(n, int(rng.integers(1 << 30)))
    want = oracle.apply_circuit(psi0, n, [g])
    got = run_gpu(n, [g], psi0, dtype)
    assert np.max(np.abs(got - want)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("extra", [0, 1, 2])
@pytest.mark.parametrize("in_line", [False, True])
def test_dense_register_path_smallest_states(k, extra, in_line, dtype):
    """The register and butterfly paths at n = 6 + k (one tile row), n = 7 + k
    (the first size where complex64 moves amplitude pairs) and n = 8 + k;
    in_line puts one target in bit 1 or 2 (inside a cache line)."""
    n = 6 + k + extra
    rng = np.random.default_rng(31 * k + extra + (500 if in_line else 0))
    if in_line:
        first = int(rng.integers(1, 3))
        rest = rng.choice(np.arange(4, n), size=k - 1, replace=False).tolist()
        qs = sorted([first] + rest)
    else:
        qs = sorted(rng.choice(np.arange(4, n), size=k, replace=False).tolist())
    U = W.random_unitary(1 << k, rng)
    g = W.Gate("dense", tuple(qs), np.ascontiguousarray(U).view(np.float64).ravel())
    _say(f"register path n={n} targets={qs} dtype={dtype}")
    psi0 = W.random_state(n, 90 + 7 * k + extra)
    want = oracle.apply_circuit(psi0, n, [g])
    got = run_gpu(n, [g], psi0, dtype)
    assert np.max(np.abs(got - want)) <= TOL[dtype]


# (targets, family at complex128, family at complex64): the register path
# takes every gate of k <= 4 with no target inside a 128-byte cache line
# (bits < 3 at complex128, < 4 at complex64); targets inside the line
# (k <= 4) take the cross-lane butterfly: one or two at complex128, one at
# complex64 (on amplitude pairs, so not bit 0); at complex64 bit 0 alone
# inside the line takes the register path on pairs that hold two entries of
# one group; 5-qubit gates, and 4-qubit gates with two targets inside the
# line (at complex64 one or two), take the matrix cores when every target
# inside a line is one of the two lowest; the LDS regroup the rest.
FAMILY_CASES = [((8, 11), "dense_direct", "dense_direct"),
                ((3, 9, 14), "dense_direct", "dense_bfly"),
                ((4, 5, 7, 13), "dense_direct", "dense_direct"),
                ((2, 6), "dense_bfly", "dense_bfly"),
                ((0, 2, 9), "dense_bfly", "dense_lds"),
                ((0, 5, 9), "dense_bfly", "dense_direct"),
                ((0, 6, 8, 12), "dense_bfly", "dense_mfma"),
                ((0, 6, 8), "dense_bfly", "dense_direct"),
                ((0,), "dense_bfly", "dense_direct"),
                ((1, 4, 5, 12), "dense_bfly", "dense_mfma"),
                ((0, 1, 3, 14), "dense_mfma", "dense_lds"),
                ((1, 2, 6, 11), "dense_mfma", "dense_mfma"),
                ((0, 3, 5, 11), "dense_bfly", "dense_mfma"),
                ((1, 2, 9), "dense_bfly", "dense_lds"),
                ((1, 2, 3), "dense_bfly", "dense_lds"),
                ((1, 6, 8, 10, 12), "dense_mfma", "dense_mfma"),
                ((0, 3, 4, 9, 12), "dense_mfma", "dense_mfma"),
                ((0, 1, 3, 7, 10), "dense_mfma", "dense_lds"),
                ((0, 1, 2, 3, 4), "dense_lds", "dense_lds")]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("case", range(len(FAMILY_CASES)))
def test_dense_family_choice(case, dtype):
    hs = _hs()
    qs, fam128, fam64 = FAMILY_CASES[case]
    n = 15
    rng = np.random.default_rng(77 + case)
    U = W.random_unitary(1 << len(qs), rng)
    g = W.Gate("dense", tuple(qs), np.ascontiguousarray(U).view(np.float64).ravel())
    _say(f"family n={n} targets={qs} dtype={dtype}")
    c = hs.circuit_from_gates(n, [g])
    psi0 = W.random_state(n, 5 + case)
    s = hs.sv_create(n, dtype)
    s.set(psi0)
    _, fam = s.apply_timed(c)
    got = s.get()
    s.close()
    assert hs.KERNEL_FAMILY[int(fam[0])] == (fam128 if dtype == "c128" else fam64)
    want = oracle.apply_circuit(psi0, n, [g])
    assert np.max(np.abs(got - want)) <= TOL[dtype]


# 5- and 4-qubit target patterns for both forms of the gate: the matrix-core
# kernel (two lowest targets as lane bits, the others as register bits) and
# the vector kernels (registers, butterflies or the LDS regroup)
DENSE5 = [(5, 6, 7, 8, 9), (0, 1, 5, 7, 9), (0, 4, 5, 6, 8), (2, 3, 4, 6, 8), (1, 3, 4, 5, 8),
          (3, 4, 5, 6, 7), (0, 1, 2, 3, 4), (4, 5, 6, 7, 8),
          (0, 1, 5, 7), (1, 2, 6, 7), (0, 2, 3, 7), (2, 3, 4, 6), (0, 3, 5, 6), (0, 1, 2, 6)]


def _mfma_applies(qs, dtype):
    """The matrix-core form takes 5-qubit gates and 4-qubit gates with two
    targets inside a cache line (at complex64 one or two), when no third
    target is inside it."""
    line_bits = 3 if dtype == "c128" else 4
    q = sorted(qs)
    if len(q) == 5:
        return q[2] >= line_bits
    inside = q[0] if dtype == "c64" else q[1]
    return inside < line_bits <= q[2]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("form", ["mfma", "vector"])
@pytest.mark.parametrize("n", [9, 10, 13])
@pytest.mark.parametrize("case", range(len(DENSE5)))
def test_dense_mfma_forms(case, n, form, dtype):
    hs = _hs()
    qs = [q for q in DENSE5[case]]
    k = len(qs)
    if max(qs) >= n:
        pytest.skip("targets beyond the state")
    rng = np.random.default_rng(900 + 11 * case + n)
    U = W.random_unitary(1 << k, rng)
    perm = rng.permutation(k)
    qs_list = [qs[i] for i in perm]
    g = W.Gate("dense", tuple(qs_list), np.ascontiguousarray(U).view(np.float64).ravel())
    _say(f"dense k={k} n={n} targets={qs_list} form={form} dtype={dtype}")
    psi0 = W.random_state(n, 70 + case + n)
    c = hs.circuit_from_gates(n, [g])
    hs.sv_debug_set_dense_mfma(form == "mfma")
    try:
        s = hs.sv_create(n, dtype)
        s.set(psi0)
        _, fam = s.apply_timed(c)
        got = s.get()
        s.close()
    finally:
        hs.sv_debug_set_dense_mfma(True)
    want_fam = "dense_mfma" if form == "mfma" and _mfma_applies(qs, dtype) and n >= k + 4 else None
    got_fam = hs.KERNEL_FAMILY[int(fam[0])]
    if want_fam:
        assert got_fam == want_fam
    else:
        assert got_fam in ("dense_direct", "dense_bfly", "dense_lds", "dense_small")
    want = oracle.apply_circuit(psi0, n, [g])
    assert np.max(np.abs(got - want)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 3, 7, 12])
def test_diagonal_gate(k, dtype):
    """Diagonal gates of 1..12 targets against the oracle, which applies the
    same diagonal as a dense 2^k x 2^k gate by its group loop."""
    n = 14
    rng = np.random.default_rng(k)
    qs = rng.choice(n, size=k, replace=False).tolist()
    d = np.exp(1j * rng.uniform(0, 2 * np.pi, 1 << k))
    g = W.Gate("dense", tuple(qs), np.ascontiguousarray(np.diag(d)).view(np.float64).ravel())
    gd = W.Gate("diag", tuple(qs), np.ascontiguousarray(d).view(np.float64).ravel())
    psi0 = W.random_state(n, k)
    hs = _hs()
    c = hs.circuit_create(n)
    hs.circuit_add_gate(c, "diag", qs, gd.params)
    s = hs.sv_create(n, dtype)
    s.set(psi0)
    _, fam = s.apply_timed(c)
    got = s.get()
    s.close()
    assert [hs.KERNEL_FAMILY[int(f)] for f in fam] == ["diag"]
    want = oracle.apply_circuit(psi0, n, [g])
    del g
    assert np.max(np.abs(got - want)) <= TOL[dtype]


# --------------------------------------------- HHL-shaped wide gates ---
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("ns,m,seed", [(1, 3, 0), (2, 4, 1), (4, 5, 2), (5, 6, 3), (6, 6, 4), (8, 4, 5)])
def test_wide_gate_circuit(ns, m, seed, dtype):
    n = ns + m + 1
    _say(f"wide-gate circuit ns={ns} m={m} dtype={dtype}")
    gates = W.wide_gate_circuit(ns, m, seed)
    psi0 = W.random_state(n, seed)
    want = oracle.apply_circuit(psi0, n, gates)
    for k in (None, 2, 5):
        got = run_gpu(n, gates, psi0, dtype, k)
        assert np.max(np.abs(got - want)) <= TOL[dtype], k


# -------------------------------------------------------- HHL solves ---
@pytest.mark.parametrize("seed", range(100))
def test_hhl_4bus_unfused_c128(seed):
    """4-bus DC power flow, 2 system + 4 clock + 1 ancilla qubits, unfused."""
    hs = _hs()
    A, b = W.dc_powerflow(4, seed)
    psi_ref, x_ref, xh_ref, info_ref = oracle.hhl_solve(A, b, 4)
    c = hs.circuit_build_hhl(A, b, 4)
    s = hs.sv_create(c.n_qubits, "c128")
    s.apply(c)
    psi = s.get()
    x_hat, info = s.postselect_solution(c, 3)
    assert np.max(np.abs(psi - psi_ref)) <= 1e-12
    assert np.max(np.abs(x_hat - xh_ref)) <= 1e-12
    assert abs(info["p_anc1"] - info_ref["p1"]) <= 1e-12
    assert abs(info["p_anc1_clock0"] - info_ref["p10"]) <= 1e-12
    xs = oracle.ge_solve(A, b)
    fid = float(np.dot(x_hat, xs / np.linalg.norm(xs)) ** 2)
    _say(f"seed={seed} kappa={info_ref['kappa']:.2f} fidelity={fid:.6f}")
    assert fid > 0.5


# The two sides build e^{iAt 2^j} from different eigen-solvers; a phase error
# t 2^j |dlambda| ~ 2 pi 2^9 (few eps) could reach ~1e-12, measured ~5e-14.
HHL64_TOL = {"c128": 1e-12, "c64": 2e-5}


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [None, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("seed", [0, 1])
def test_hhl_64bus(seed, k, dtype):
    hs = _hs()
    A, b = W.dc_powerflow(64, seed)
    psi_ref, x_ref, xh_ref, info_ref = oracle.hhl_solve(A, b, 10)
    c = hs.circuit_build_hhl(A, b, 10)
    run = hs.fuse(c, k) if k else c
    s = hs.sv_create(c.n_qubits, dtype)
    s.apply(run)
    psi = s.get()
    x_hat, info = s.postselect_solution(c, 63)
    err = float(np.max(np.abs(psi - psi_ref)))
    fid = float(np.dot(x_hat, xh_ref) ** 2)
    _say(f"64-bus seed={seed} k={k} {dtype}: max|d amp|={err:.3e} fid_vs_oracle={fid:.12f} "
         f"gates={run.n_gates}")
    assert err <= HHL64_TOL[dtype]
    assert fid >= 0.999


def test_exact_spectrum_gpu():
    hs = _hs()
    A, b, t, _ = W.exact_spectrum_system(3, 6, 11)
    c = hs.circuit_build_hhl(A, b, 6, t)
    s = hs.sv_create(c.n_qubits, "c128")
    s.apply(hs.fuse(c, 4))
    x_hat, info = s.postselect_solution(c, b.size)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(info["scale"] * x_hat - xs) <= 1e-11 * np.linalg.norm(xs)


# ---------------------------------------------------- state utilities ---
def test_norm_gather_reset():
    hs = _hs()
    n = 16
    psi0 = W.random_state(n, 3)
    s = hs.sv_create(n, "c128")
    assert abs(s.norm2() - 1.0) < 1e-15 and s.get_at([0])[0] == 1
    s.set(psi0)
    assert abs(s.norm2() - 1.0) < 1e-13
    idx = np.array([0, 5, (1 << n) - 1, 12345])
    assert np.max(np.abs(s.get_at(idx) - psi0[idx])) == 0
    s.reset()
    out = s.get()
    assert out[0] == 1 and np.count_nonzero(out) == 1


def test_errors_on_gpu_calls():
    hs = _hs()
    s = hs.sv_create(5, "c128")
    c = hs.circuit_create(6)
    with pytest.raises(hs.HHLSVError, match="SHAPE"):
        s.apply(c)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        s.get_at([1 << 5])
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        s.get(30, 10)


# ------------------------------------------------ wide gates, 5..10 targets ---
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k,control", [(5, True), (6, True), (7, False), (7, True), (8, True), (9, True), (10, True), (6, False)])
def test_wide_gate_widths(k, control, dtype):
    n = 14
    rng = np.random.default_rng(50 + k)
    qs = rng.choice(n, size=k + (1 if control else 0), replace=False).tolist()
    U = W.random_unitary(1 << k, rng)
    g = W.Gate("cdense" if control else "dense", tuple(qs), np.ascontiguousarray(U).view(np.float64).ravel())
    psi0 = W.random_state(n, k)
    want = oracle.apply_circuit(psi0, n, [g])
    got = run_gpu(n, [g], psi0, dtype)
    assert np.max(np.abs(got - want)) <= TOL[dtype]
    # contiguous low targets with the control above them: the HHL layout
    qs2 = [k + 1] + list(range(k)) if control else list(range(k))
    g2 = W.Gate(g.kind, tuple(qs2), g.params)
    want2 = oracle.apply_circuit(psi0, n, [g2])
    got2 = run_gpu(n, [g2], psi0, dtype)
    assert np.max(np.abs(got2 - want2)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k,control", [(3, True), (4, True), (5, True), (6, True), (6, False), (4, False),
                                       (7, True), (8, True), (8, False)])
def test_wide_gate_matrix_cores(k, control, dtype):
    """Wide gates that run on the matrix cores: 8..64 columns on states with
    >= 16384 rows per launch, 128 and 256 columns (rows staged in LDS) with
    >= 2048 rows; scattered and contiguous targets."""
    n = k + (15 if k <= 6 else 12) + (1 if control else 0)
    rng = np.random.default_rng(70 + k + (100 if control else 0))
    qs = rng.choice(n, size=k + (1 if control else 0), replace=False).tolist()
    U = W.random_unitary(1 << k, rng)
    g = W.Gate("cdense" if control else "dense", tuple(qs), np.ascontiguousarray(U).view(np.float64).ravel())
    _say(f"wide on matrix cores n={n} qubits={qs} dtype={dtype}")
    psi0 = W.random_state(n, 7 * k)
    want = oracle.apply_circuit(psi0, n, [g])
    got = run_gpu(n, [g], psi0, dtype)
    assert np.max(np.abs(got - want)) <= TOL[dtype]
    qs2 = [n - 1] + list(range(k)) if control else list(range(2, 2 + k))
    g2 = W.Gate(g.kind, tuple(qs2), g.params)
    want2 = oracle.apply_circuit(psi0, n, [g2])
    got2 = run_gpu(n, [g2], psi0, dtype)
    assert np.max(np.abs(got2 - want2)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("r", [2, 3])
@pytest.mark.parametrize("k,n", [(2, 9), (3, 12), (6, 14), (3, 20), (6, 21), (5, 22)])
def test_controlled_gates_as_mux(k, n, r, dtype):
    """r controlled dense gates in a row on the same k targets, fused into
    one MUX op (2^r - 1 matrices by control value), against the oracle's r
    gates: the vector GEMM on small states, the matrix cores from 16384 rows
    ((2^r - 1) 2^(n-k-r)); scattered targets and controls, a single state."""
    rng = np.random.default_rng(300 + 10 * k + n + 1000 * r)
    qs = rng.choice(n, size=k + r, replace=False).tolist()
    gates = [W.Gate("cdense", (qs[l],) + tuple(qs[r:]),
                    np.ascontiguousarray(W.random_unitary(1 << k, rng)).view(np.float64).ravel())
             for l in range(r)]
    hs = _hs()
    fused = hs.fuse(hs.circuit_from_gates(n, gates), 1)
    assert [kind for kind, _, _ in fused.gates()] == [f"mux{r}"]
    _say(f"mux{r} n={n} k={k} qubits={qs} rows={((1 << r) - 1) << (n - k - r)} dtype={dtype}")
    psi0 = W.random_state(n, 11 * k + n)
    want = oracle.apply_circuit(psi0, n, gates)
    got = run_gpu(n, gates, psi0, dtype, k=1)
    assert np.max(np.abs(got - want)) <= TOL[dtype]


# ---------------------------------------------------- hipGraph replays ---
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_graph_replay_matches_eager(dtype):
    """sv_apply on small states replays a captured graph; every replay (with
    eager work and synchronisation in between) must equal the eager run."""
    hs = _hs()
    n = 12
    gates = W.random_circuit(n, 60, 77, kmax=4)
    c = hs.fuse(hs.circuit_from_gates(n, gates), 3)
    psi0 = W.random_state(n, 77)
    eager = hs.sv_create(n, dtype)
    eager.set(psi0)
    eager.apply_timed(c)          # kernel-by-kernel launches
    ref = eager.get()
    s = hs.sv_create(n, dtype)
    for rep in range(4):
        s.reset()
        assert s.norm2() == 1.0
        s.set(psi0)
        s.apply(c)                # graph replay
        out = s.get()
        assert np.array_equal(out, ref), rep
    assert np.max(np.abs(ref - oracle.apply_circuit(psi0, n, gates))) <= TOL[dtype]


# ------------------------------------------- device-built evolution tables ---
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nbus,m,k", [(64, 10, None), (64, 10, 4), (32, 8, 3), (128, 6, 2), (256, 5, 4)])
def test_device_evolutions_match_oracle(nbus, m, k, dtype):
    hs = _hs()
    A, b = W.dc_powerflow(nbus, 8)
    psi_ref, _, xh_ref, info_ref = oracle.hhl_solve(A, b, m)
    c = hs.circuit_build_hhl(A, b, m, device_evolutions=True)
    run = hs.fuse(c, k) if k else c
    s = hs.sv_create(c.n_qubits, dtype)
    s.apply(run)
    err = float(np.max(np.abs(s.get() - psi_ref)))
    x_hat, info = s.postselect_solution(c, nbus - 1)
    _say(f"device evolutions nbus={nbus} m={m} k={k} {dtype}: max|d amp|={err:.3e}")
    assert err <= TOL[dtype]
    assert float(np.dot(x_hat, xh_ref) ** 2) >= 0.999


def test_stream_probe_leaves_state_unchanged():
    """The bandwidth probe reads and writes back every amplitude: the state
    is bitwise the same afterwards, and each launch reports a positive time."""
    hs = _hs()
    n = 16
    psi0 = W.random_state(n, 1616)
    s = hs.sv_create(n, "c128")
    s.set(psi0)
    ms = s.stream_probe(3)
    got = s.get()
    s.close()
    assert ms.shape == (3,) and np.all(ms > 0)
    assert np.array_equal(got, psi0)
    s64 = hs.sv_create(n, "c64")
    with pytest.raises(hs.HHLSVError):
        s64.stream_probe(1)
    s64.close()
