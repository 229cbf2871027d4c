"""CPU tests of libhhlsv's host side: exported symbols, the HHL circuit
builder, the fusion pass and input validation.  No GPU call is made; circuits
are evaluated with the numpy tensor helpers of tests/_ref.py.
"""
import math
import os
import re

import numpy as np
import pytest
import scipy.linalg

import oracle
import paper_2402_08136_amd as hs
import workloads as W
from tests._ref import apply_tensor, apply_ucry_tensor, cmat, max_abs_diff

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = _header_functions()
    assert "sv_create" in names and "fuse" in names
    for nm in names:
        assert hasattr(hs._lib, nm), f"{nm} declared in include/ but not exported"


# ------------------------------------------------------- numpy evaluation ---
def _np_apply_gate(psi, n, kind, qs, ps):
    if kind in ("dense",):
        return apply_tensor(psi, n, qs, cmat(ps, len(qs)))
    if kind == "diag":
        return apply_tensor(psi, n, qs, np.diag(np.asarray(ps).view(np.complex128)))
    if kind == "cdense":
        return apply_tensor(psi, n, qs[1:], cmat(ps, len(qs) - 1), control=qs[0])
    if kind == "ucry":
        return apply_ucry_tensor(psi, n, qs[0], qs[1:], ps)
    if kind in ("mux2", "mux3"):
        # block-diag(I, U_1, ..) over (controls, targets): index v + V r
        r = 2 if kind == "mux2" else 3
        V, K = 1 << r, 1 << (len(qs) - r)
        us = np.asarray(ps).view(np.complex128).reshape(V - 1, K, K)
        M = np.zeros((V * K, V * K), dtype=complex)
        M[0::V, 0::V] = np.eye(K)
        for v in range(1, V):
            M[v::V, v::V] = us[v - 1]
        return apply_tensor(psi, n, qs, M)
    return apply_tensor(psi, n, qs, oracle.gate_matrix(kind, ps))


def np_run(circ: hs.Circuit, psi):
    n = circ.n_qubits
    for kind, qs, ps in circ.gates():
        psi = _np_apply_gate(psi, n, kind, qs, ps)
    return psi


# ------------------------------------------------------------ HHL builder ---
@pytest.mark.parametrize("ns,m", [(2, 4), (6, 10), (3, 7)])
def test_hhl_gate_count(ns, m):
    A, b = W.dc_powerflow(1 << ns, 5)
    c = hs.circuit_build_hhl(A, b, m)
    assert c.n_qubits == ns + m + 1
    assert c.n_gates == ns + 6 * m + m * (m - 1) + 2 * (m // 2) + 1


@pytest.mark.parametrize("nbus,m,seed", [(4, 4, 0), (16, 7, 1), (64, 10, 2), (4, 4, 14)])
def test_hhl_parameters_match_oracle(nbus, m, seed):
    A, b = W.dc_powerflow(nbus, seed)
    info = hs.circuit_build_hhl(A, b, m).info()
    ref = oracle.hhl_params(A, b, m)
    assert info["n_sys"] == ref["ns"] and info["j0"] == ref["j0"]
    for key_l, key_o in [("t", "t"), ("C", "C"), ("lambda_lo", "lambda_lo"),
                         ("lambda_hi", "lambda_hi"), ("kappa", "kappa"), ("b_norm", "beta")]:
        assert abs(info[key_l] - ref[key_o]) <= 1e-12 * abs(ref[key_o]), key_l


@pytest.mark.parametrize("nbus,m,seed", [(4, 4, 3), (32, 8, 4), (64, 10, 5)])
def test_hhl_evolutions_are_matrix_exponentials(nbus, m, seed):
    A, b = W.dc_powerflow(nbus, seed)
    c = hs.circuit_build_hhl(A, b, m)
    info = c.info()
    ns = info["n_sys"]
    D = 1 << ns
    Ap = np.eye(D)
    Ap[: A.shape[0], : A.shape[0]] = A
    cd = [g for g in c.gates() if g[0] == "cdense"]
    assert len(cd) == 2 * m
    for j in range(m):
        want = scipy.linalg.expm(1j * Ap * info["t"] * 2 ** j)
        kind, qs, ps = cd[j]
        assert qs == [ns + j] + list(range(ns))
        U = cmat(ps, ns)
        # phase error grows with t 2^j ||A||; bound from the exponent's size
        tol = 1e-13 * max(1.0, info["t"] * 2 ** j * np.linalg.norm(Ap, 2)) * D
        assert max_abs_diff(U, want) < tol
        assert max_abs_diff(cmat(cd[2 * m - 1 - j][2], ns), want.conj().T) < tol


@pytest.mark.parametrize("ns,seed", [(1, 0), (2, 1), (3, 2), (6, 3)])
def test_state_prep_tree_loads_b(ns, seed):
    """The |b> preparation gates map |0> exactly to b / ||b||."""
    rng = np.random.default_rng(seed)
    N = (1 << ns) - (1 if ns > 1 else 0)
    b = rng.standard_normal(N)
    b[0] = -abs(b[0])                      # signs must survive
    A = np.eye(N) * 2.0
    c = hs.circuit_build_hhl(A, b, 2)
    n = c.n_qubits
    psi = np.zeros(1 << n, dtype=complex)
    psi[0] = 1
    for kind, qs, ps in c.gates()[:ns]:
        assert kind == "ucry"
        psi = _np_apply_gate(psi, n, kind, qs, ps)
    want = np.zeros(1 << n, dtype=complex)
    want[:N] = b / np.linalg.norm(b)
    assert max_abs_diff(psi, want) < 1e-14


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_inverse_qft_gates_closed_form(m):
    ns = 1
    A = np.array([[2.0, 0.5], [0.5, 3.0]])
    c = hs.circuit_build_hhl(A, np.array([1.0, 0.2]), m)
    g = c.gates()
    start = ns + 2 * m
    qft_inv = g[start: start + m + m * (m - 1) // 2 + m // 2]
    n = c.n_qubits
    M = 1 << m
    for x in range(M):
        psi = np.zeros(1 << n, dtype=complex)
        psi[x << ns] = 1
        for kind, qs, ps in qft_inv:
            psi = _np_apply_gate(psi, n, kind, qs, ps)
        e = np.zeros(M, dtype=complex)
        e[x] = 1
        closed = np.fft.fft(e) / math.sqrt(M)    # inverse QFT: e^{-2 pi i x y / M}
        want = np.zeros(1 << n, dtype=complex)
        for y in range(M):
            want[y << ns] = closed[y]
        assert max_abs_diff(psi, want) < 1e-14


def test_hhl_numpy_evaluation_matches_oracle():
    """Library gate list evaluated by numpy equals the oracle's own HHL."""
    A, b = W.dc_powerflow(4, 7)
    c = hs.circuit_build_hhl(A, b, 4)
    n = c.n_qubits
    psi = np.zeros(1 << n, dtype=complex)
    psi[0] = 1
    psi = np_run(c, psi)
    ref, _, _, _ = oracle.hhl_solve(A, b, 4)
    assert max_abs_diff(psi, ref) < 1e-13


# ----------------------------------------------------------------- fusion ---
@pytest.mark.parametrize("n,seed,k", [(4, 0, 1), (5, 1, 2), (6, 2, 3), (7, 3, 4), (8, 4, 5), (8, 5, 2)])
def test_fusion_preserves_unitary(n, seed, k):
    gates = W.random_circuit(n, 60, seed, kmax=3)
    c = hs.circuit_from_gates(n, gates)
    f = hs.fuse(c, k)
    assert f.n_gates <= c.n_gates
    diagonal = ("rz", "p", "cp", "diag")
    wide_in = sum(len(g.qubits) > k and g.kind not in diagonal + ("swap",) for g in gates)
    wide_out = swaps_out = 0
    for kind, qs, ps in f.gates():
        if len(qs) <= k:
            assert kind in ("dense", "diag") and qs == sorted(qs)
        elif kind in diagonal:
            assert len(qs) <= 10    # passed through, or diagonals merged past k_max
        elif kind == "swap":
            swaps_out += 1          # what is left of the relabelling, at the end
        else:
            # too wide to fuse: passed through unchanged (qubits relabelled),
            # or two controlled gates on the same targets as one MUX2
            wide_out += {"mux2": 2, "mux3": 3}.get(kind, 1)
    assert wide_out == wide_in
    assert swaps_out <= min(n - 1, sum(g.kind == "swap" for g in gates))
    psi = W.random_state(n, seed)
    assert max_abs_diff(np_run(f, psi), np_run(c, psi)) < 1e-13


def test_diagonals_merge_past_commuting_gates():
    """Diagonal blocks merge beyond k_max (up to 10 qubits) past gates they
    commute with: gates on other qubits and gates that read the shared
    qubits only as controls; a gate acting on a shared qubit stops them."""
    n, k = 7, 2
    U = W.random_unitary(4, np.random.default_rng(5))
    cd_params = np.stack([U.real, U.imag], -1).ravel()
    gates = [W.Gate("cp", (2, 3), np.array([0.3])),
             W.Gate("h", (5,), np.array([])),
             W.Gate("cdense", (4, 0, 1), cd_params),          # control 4
             W.Gate("cp", (4, 6), np.array([0.5])),
             W.Gate("ucry", (0, 5, 6), np.array([0.1, 0.2, 0.3, 0.4])),   # controls 5, 6
             W.Gate("cp", (5, 6), np.array([0.7])),
             W.Gate("h", (2,), np.array([])),                 # joins cp(2, 3) into a dense block
             W.Gate("cp", (2, 4), np.array([1.1]))]
    c = hs.circuit_from_gates(n, gates)
    f = hs.fuse(c, k)
    diags = [qs for kind, qs, _ in f.gates() if kind == "diag"]
    # cp(5, 6) moves back past the UCRY it only controls and joins cp(4, 6)
    # (3 qubits, above k_max = 2); cp(2, 4) cannot pass the H on qubit 2
    assert diags == [[4, 5, 6], [2, 4]]
    psi = W.random_state(n, 5)
    assert max_abs_diff(np_run(f, psi), np_run(c, psi)) < 1e-13
    g = hs.fuse(c, 5)        # wide enough that the first passes merge more
    psi2 = W.random_state(n, 6)
    assert max_abs_diff(np_run(g, psi2), np_run(c, psi2)) < 1e-13


def test_swaps_become_relabelling():
    """SWAP gates cost no sweep: later gates take the exchanged qubits, and
    the permutation left at the end is undone by as few swaps as it needs
    (none when the swaps cancel, as the two QFT swap layers of HHL do)."""
    n = 5
    rng = np.random.default_rng(9)
    U = W.random_unitary(4, rng)
    gates = [W.Gate("h", (0,), np.array([])), W.Gate("swap", (0, 3), np.array([])),
             W.Gate("dense", (3, 1), np.stack([U.real, U.imag], -1).ravel()),
             W.Gate("swap", (1, 4), np.array([])), W.Gate("cx", (4, 2), np.array([])),
             W.Gate("ry", (1,), np.array([0.4]))]
    c = hs.circuit_from_gates(n, gates)
    for k in (1, 2, 3):
        f = hs.fuse(c, k)
        psi = W.random_state(n, k)
        assert max_abs_diff(np_run(f, psi), np_run(c, psi)) < 1e-13
        # the two swaps form a 3-cycle (0 3)(1 4): two restoring swaps at most
        assert sum(kind == "swap" for kind, _, _ in f.gates()) <= 2
    # h(0), swap(0, 3), rz(3), swap(3, 0): the rz lands on qubit 0 and joins the h
    cancel = gates[:2] + [W.Gate("rz", (3,), np.array([0.2])), W.Gate("swap", (3, 0), np.array([]))]
    cc = hs.circuit_from_gates(n, cancel)
    f = hs.fuse(cc, 1)
    assert [(kind, qs) for kind, qs, _ in f.gates()] == [("dense", [0])]
    psi = W.random_state(n, 4)
    assert max_abs_diff(np_run(f, psi), np_run(cc, psi)) < 1e-13
    A, b = W.dc_powerflow(16, 3)
    hc = hs.circuit_build_hhl(A, b, 6)
    assert any(kind == "swap" for kind, _, _ in hc.gates())
    for k in (2, 5):
        fk = hs.fuse(hc, k)
        assert all(kind != "swap" for kind, _, _ in fk.gates())
        psi = np.zeros(1 << hc.n_qubits, dtype=complex)
        psi[0] = 1
        assert max_abs_diff(np_run(fk, psi), np_run(hc, psi)) < 1e-12


@pytest.mark.parametrize("device_evolutions", [False, True])
@pytest.mark.parametrize("m", [6, 7, 8])
def test_controlled_evolutions_become_mux_gates(device_evolutions, m):
    """Runs of controlled evolutions on the system register merge in threes
    into MUX3 gates (a pair left over into a MUX2, a single one stays):
    U_v is the product of the evolutions set in v, e^{iAt sum 2^j}."""
    ns = 4
    A, b = W.dc_powerflow(1 << ns, 8)
    c = hs.circuit_build_hhl(A, b, m, device_evolutions=device_evolutions)
    ref = hs.circuit_build_hhl(A, b, m)
    f = hs.fuse(c, 3)          # 5-qubit controlled gates stay whole at k_max = 3
    kinds = [kind for kind, _, _ in f.gates()]
    # two runs of m (phase estimation and its inverse)
    assert kinds.count("mux3") == 2 * (m // 3)
    assert kinds.count("mux2") == 2 * (m % 3 == 2) and kinds.count("cdense") == 2 * (m % 3 == 1)
    qs, ps = next((qs, ps) for kind, qs, ps in f.gates() if kind == "mux3")
    assert qs[3:] == list(range(ns)) and len(set(qs[:3])) == 3
    us = np.asarray(ps).view(np.complex128).reshape(7, 1 << ns, 1 << ns)
    assert np.allclose(us[2], us[1] @ us[0], atol=1e-12)                # v = 3
    assert np.allclose(us[6], us[3] @ us[1] @ us[0], atol=1e-12)        # v = 7
    psi = np.zeros(1 << c.n_qubits, dtype=complex)
    psi[0] = 1
    assert max_abs_diff(np_run(f, psi), np_run(ref, psi)) < 1e-12
    # a gate between them, or different targets, keeps them apart
    U = W.random_unitary(4, np.random.default_rng(3))
    up = np.stack([U.real, U.imag], -1).ravel()
    gates = [W.Gate("cdense", (2, 0, 1), up), W.Gate("h", (0,), np.array([])),
             W.Gate("cdense", (3, 0, 1), up), W.Gate("cdense", (4, 1, 0), up)]
    g = hs.fuse(hs.circuit_from_gates(5, gates), 2)
    assert not any(kind.startswith("mux") for kind, _, _ in g.gates())


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_fusion_of_hhl_circuit(k):
    A, b = W.dc_powerflow(4, 2)
    c = hs.circuit_build_hhl(A, b, 4)
    f = hs.fuse(c, k)
    psi = np.zeros(1 << c.n_qubits, dtype=complex)
    psi[0] = 1
    assert max_abs_diff(np_run(f, psi), np_run(c, psi)) < 1e-13
    assert f.info()["C"] == c.info()["C"]


def test_fusion_counts_layered_33q():
    gates = W.layered_circuit(33, 40, 2402)
    assert len(gates) == 40 * (3 * 33 + 16) == 4600
    c = hs.circuit_from_gates(33, gates)
    counts = {k: hs.fuse(c, k).n_gates for k in (1, 2, 3, 4, 5)}
    # k = 1 merges each qubit's 1q run; the idle qubit of a layer also merges
    # into the next layer's run (39 times)
    assert counts[1] == 40 * (33 + 16) - 39
    assert counts[1] > counts[2] > counts[3] >= counts[4] >= counts[5]


def test_fusion_k2_is_the_papers_four_strategies():
    """1q-1q, 1q before/after a 2q gate, and 2q-2q on the same pair all
    collapse into one gate at k_max = 2."""
    n = 3
    gates = [W.Gate("h", (0,), np.array([])), W.Gate("rz", (0,), np.array([0.3])),
             W.Gate("ry", (1,), np.array([0.2])), W.Gate("cx", (0, 1), np.array([])),
             W.Gate("u3", (1,), np.array([0.1, 0.2, 0.3])), W.Gate("cp", (1, 0), np.array([0.7])),
             W.Gate("h", (2,), np.array([]))]
    f = hs.fuse(hs.circuit_from_gates(n, gates), 2)
    assert f.n_gates == 2
    assert sorted(len(qs) for _, qs, _ in f.gates()) == [1, 2]


@pytest.mark.parametrize("k,want", [(1, 6), (2, 3), (3, 2), (4, 2), (5, 2)])
def test_disjoint_gates_share_a_sweep(k, want):
    """A layer of one-qubit gates on distinct qubits fuses into blocks of up
    to k_max qubits (they commute)."""
    n = 6
    gates = [W.Gate("h", (q,), np.array([])) for q in range(n)]
    c = hs.circuit_from_gates(n, gates)
    f = hs.fuse(c, k)
    assert f.n_gates == want
    psi = W.random_state(n, 3)
    assert max_abs_diff(np_run(f, psi), np_run(c, psi)) < 1e-13


def test_disjoint_merge_respects_order():
    """A block moves forward to a disjoint later block only when nothing in
    between touches its qubits; the overlap merges come first."""
    gates = [W.Gate("h", (0,), np.array([])), W.Gate("h", (1,), np.array([])),
             W.Gate("cx", (1, 2), np.array([])), W.Gate("h", (3,), np.array([])),
             W.Gate("ry", (0,), np.array([0.4])), W.Gate("h", (0,), np.array([]))]
    c = hs.circuit_from_gates(4, gates)
    f = hs.fuse(c, 2)
    # {h1, cx12}, then h0 h3 ry0 h0 as one two-qubit block {0, 3}
    assert sorted(tuple(qs) for _, qs, _ in f.gates()) == [(0, 3), (1, 2)]
    psi = W.random_state(4, 9)
    assert max_abs_diff(np_run(f, psi), np_run(c, psi)) < 1e-13
    # a gate between that touches qubit 3 keeps h3 where it is
    gates2 = gates[:4] + [W.Gate("cx", (3, 2), np.array([]))] + gates[4:]
    c2 = hs.circuit_from_gates(4, gates2)
    f2 = hs.fuse(c2, 2)
    psi2 = W.random_state(4, 10)
    assert max_abs_diff(np_run(f2, psi2), np_run(c2, psi2)) < 1e-13


def test_diagonal_runs_stay_diagonal():
    gates = [W.Gate("rz", (0,), np.array([0.3])), W.Gate("cp", (0, 1), np.array([0.5])),
             W.Gate("p", (1,), np.array([0.9]))]
    f = hs.fuse(hs.circuit_from_gates(2, gates), 2)
    assert [g[0] for g in f.gates()] == ["diag"]


# ------------------------------------------------------------- validation ---
def test_validation_errors():
    with pytest.raises(hs.HHLSVError, match="NOT_SYMMETRIC"):
        hs.circuit_build_hhl(np.array([[1.0, 2.0], [0.0, 1.0]]), np.ones(2), 3)
    with pytest.raises(hs.HHLSVError, match="NOT_POSDEF"):
        hs.circuit_build_hhl(np.array([[1.0, 0.0], [0.0, -1.0]]), np.ones(2), 3)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_build_hhl(np.eye(2), np.zeros(2), 3)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_build_hhl(np.eye(2), np.ones(2), 0)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_build_hhl(np.eye(4), np.ones(4), 33)
    c = hs.circuit_create(3)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_add_gate(c, "cx", [0, 0])
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_add_gate(c, "h", [3])
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_add_gate(c, "ry", [0], [])
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_add_gate(c, "dense", [0, 1], np.zeros(8))
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.fuse(c, 6)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_create(35)


def test_qubit_estimate_matches_table1():
    assert hs.sv_qubit_estimate(16, 119.2, True) == (4, 8, 13)
    assert hs.sv_qubit_estimate(32, 492.5, True) == (5, 10, 16)
    assert hs.sv_qubit_estimate(64, 109.3, True) == (6, 8, 15)


def test_sym_eig_against_numpy():
    """The library's eigen-solve (through the circuit parameters) agrees with
    LAPACK's on an ill-conditioned 64-bus system."""
    A, b = W.dc_powerflow(64, 9)
    info = hs.circuit_build_hhl(A, b, 10).info()
    w = np.linalg.eigvalsh(A)
    assert abs(info["lambda_lo"] - w[0]) < 1e-12 * w[-1]
    assert abs(info["lambda_hi"] - w[-1]) < 1e-12 * w[-1]


# ------------------------------------------------ deferred evolution tables ---
@pytest.mark.parametrize("nbus,m", [(4, 4), (32, 6), (64, 8)])
def test_deferred_evolutions_materialise_identically(nbus, m):
    """With the device-evolution flag the host builds the matrices only on
    demand (serialize, fusion into small gates); they equal the eager ones."""
    A, b = W.dc_powerflow(nbus, 4)
    eager = hs.circuit_build_hhl(A, b, m)
    lazy = hs.circuit_build_hhl(A, b, m, device_evolutions=True)
    assert eager.serialize() == lazy.serialize()
    for k in (2, 5):
        assert hs.fuse(eager, k).serialize() == hs.fuse(lazy, k).serialize()
    assert eager.info() == lazy.info()


# ------------------------------------------ dilation and the sign qubit ---
def _general_cases():
    A1, b1, t1, _ = W.signed_spectrum_system(3, 7, 1)
    A2, b2, t2, _ = W.nonsymmetric_exact_system(5, 7, 2)
    A3, b3 = W.general_system(6, 3, kappa=40.0)
    A4, b4 = W.general_system(7, 4, kappa=15.0, symmetric=True)
    A5, b5 = W.dc_powerflow(8, 5)
    A6, b6 = W.dc_powerflow(14, 6)
    return [("signed", A1, b1, 7, t1, oracle.HHL_SIGNED),
            ("dilate", A2, b2, 7, t2, oracle.HHL_DILATE),
            ("dilate", A3, b3, 8, 0.0, oracle.HHL_DILATE),
            ("signed", A4, b4, 6, 0.0, oracle.HHL_SIGNED),
            ("signed", -A5, b5, 7, 0.0, oracle.HHL_SIGNED),
            ("dilate", A5, b5, 6, 0.0, oracle.HHL_DILATE),
            ("gauss_seidel", A6, b6, 6, 0.0, oracle.HHL_GS)]


@pytest.mark.parametrize("case", range(7))
def test_signed_dilated_parameters_match_oracle(case):
    mode, A, b, m, t, oflags = _general_cases()[case]
    info = hs.circuit_build_hhl(A, b, m, t, mode=mode).info()
    ref = oracle.hhl_params(A, b, m, t, flags=oflags)
    assert info["n_sys"] == ref["ns"] and info["j0"] == ref["j0"]
    assert info["x_offset"] == ref["x_off"] and info["sign_qubit"] == ref["sign_qubit"] == 1
    assert info["dilated"] == (mode in ("dilate", "gauss_seidel"))
    assert info["preconditioned"] == (mode == "gauss_seidel")
    assert info["n_total"] == ref["n"]
    for key_l, key_o in [("t", "t"), ("C", "C"), ("lambda_lo", "lambda_lo"),
                         ("lambda_hi", "lambda_hi"), ("kappa", "kappa"), ("b_norm", "beta")]:
        assert abs(info[key_l] - ref[key_o]) <= 1e-11 * abs(ref[key_o]), key_l


@pytest.mark.parametrize("case", [0, 1, 3, 4, 6])
def test_signed_dilated_numpy_evaluation_matches_oracle(case):
    """The library's gate list (signed inversion angles, dilated evolutions)
    evaluated gate by gate with numpy equals the oracle's final state."""
    mode, A, b, m, t, oflags = _general_cases()[case]
    c = hs.circuit_build_hhl(A, b, m, t, mode=mode)
    psi = np.zeros(1 << c.n_qubits, dtype=complex)
    psi[0] = 1
    psi = np_run(c, psi)
    ref, _, _, _ = oracle.hhl_solve(A, b, m, t, flags=oflags)
    assert max_abs_diff(psi, ref) < 1e-12


def test_signed_inversion_angles():
    """Clock value c decodes to c, or c - 2^m for c >= 2^{m-1}; the angle is
    2 asin(clamp(j0 / v)) and negative for negative v."""
    A, b, t, _ = W.signed_spectrum_system(2, 5, 9)
    c = hs.circuit_build_hhl(A, b, 5, t, mode="signed")
    j0 = c.info()["j0"]
    uc = [g for g in c.gates() if g[0] == "ucry" and g[1][0] == c.n_qubits - 1]
    assert len(uc) == 1          # the state-preparation tree targets system qubits
    th = np.asarray(uc[0][2])
    v = np.arange(32)
    v = np.where(v >= 16, v - 32, v)
    want = np.zeros(32)
    nz = v != 0
    want[nz] = 2 * np.arcsin(np.clip(j0 / v[nz], -1, 1))
    assert np.allclose(th, want, rtol=0, atol=1e-15)
    assert th[16] < 0 and th[15] > 0


def test_auto_mode_choices():
    Aspd, b = W.dc_powerflow(8, 1)
    i = hs.circuit_build_hhl(Aspd, b, 6, mode="auto").info()
    assert (i["sign_qubit"], i["dilated"], i["x_offset"]) == (0, 0, 0)
    i = hs.circuit_build_hhl(-Aspd, b, 6, mode="auto").info()
    assert (i["sign_qubit"], i["dilated"]) == (1, 0)
    S, bs = W.general_system(8, 2, kappa=10.0, symmetric=True)
    i = hs.circuit_build_hhl(S, bs, 6, mode="auto").info()
    assert (i["sign_qubit"], i["dilated"]) == (1, 0)
    G, bg = W.general_system(6, 3, kappa=10.0)
    i = hs.circuit_build_hhl(G, bg, 6, mode="auto").info()
    assert (i["sign_qubit"], i["dilated"], i["x_offset"], i["n_sys"]) == (1, 1, 8, 4)


@pytest.mark.parametrize("N", [1, 2, 3, 8, 13, 29])
def test_dilated_register_sizes(N):
    """Pad first (step 1b), then dilate (step 1c): 29 -> 32 -> 64 is the six
    data qubits of the preconditioned 30-bus row of Table I."""
    G, bg = W.general_system(N, N, kappa=5.0)
    c = hs.circuit_build_hhl(G, bg, 5, mode="dilate")
    i = c.info()
    k = math.ceil(math.log2(N)) if N > 1 else 0
    assert i["n_sys"] == k + 1 and i["x_offset"] == 1 << k
    assert c.n_qubits == k + 1 + 5 + 1
    m = 5
    assert c.n_gates == (k + 1) + 6 * m + m * (m - 1) + 2 * (m // 2) + 1


def test_signed_dilated_errors():
    A, b, t, _ = W.signed_spectrum_system(2, 5, 0)
    with pytest.raises(hs.HHLSVError, match="NOT_POSDEF"):
        hs.circuit_build_hhl(A, b, 5)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_build_hhl(A, b, 1, mode="signed")
    with pytest.raises(hs.HHLSVError, match="SINGULAR"):
        hs.circuit_build_hhl(np.diag([1.0, 0.0]), np.ones(2), 4, mode="signed")
    G, bg = W.general_system(5, 0)
    with pytest.raises(hs.HHLSVError, match="NOT_SYMMETRIC"):
        hs.circuit_build_hhl(G, bg, 5, mode="signed")
    with pytest.raises(hs.HHLSVError, match="SINGULAR"):
        hs.circuit_build_hhl(np.array([[0.0, 1.0], [1.0, 2.0]]), np.ones(2), 5, mode="gauss_seidel")
    big = np.eye(2049)
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.circuit_build_hhl(big, np.ones(2049), 4, mode="dilate")
    with pytest.raises(ValueError):
        hs.circuit_build_hhl(A, b, 5, mode="bogus")
    h = hs._vp()
    Ac = np.ascontiguousarray(A)
    rc = hs._lib.circuit_build_hhl_ex(hs._dptr(Ac), hs._dptr(b), b.size, 5, 0.0, 64, hs.ctypes.byref(h))
    assert rc == -1


# ------------------------------------------------- Newton-Raphson power flow ---
@pytest.mark.parametrize("nb,seed", [(5, 0), (14, 1), (30, 2)])
def test_pf_model_matches_oracle(nb, seed):
    """The library's complex-form injections, mismatch and Jacobian equal the
    oracle's polar-form ones at a random operating point."""
    c = W.ac_powerflow_case(nb, seed, pv_frac=0.3)
    rng = np.random.default_rng(seed)
    vm = rng.uniform(0.9, 1.1, nb)
    va = rng.uniform(-0.3, 0.3, nb)
    P, Q, F, J = hs.pf_mismatch_jacobian(c, vm, va)
    Po, Qo, Fo, Jo = oracle.pf_eval(c, vm, va)
    scale = max(1.0, np.abs(Jo).max())
    assert np.abs(P - Po).max() < 1e-12 * scale and np.abs(Q - Qo).max() < 1e-12 * scale
    assert np.abs(F - Fo).max() < 1e-12 * scale
    assert J.shape == Jo.shape and np.abs(J - Jo).max() < 1e-12 * scale


def test_pf_validation():
    c = W.ac_powerflow_case(5, 0)
    bad = dict(c, type=np.zeros(5, np.int32))
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.pf_mismatch_jacobian(bad, np.ones(5), np.zeros(5))
    bad = dict(c, x=np.zeros_like(c["x"]), r=np.zeros_like(c["r"]))
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.pf_mismatch_jacobian(bad, np.ones(5), np.zeros(5))
    bad = dict(c, to=np.array(c["from"]))
    with pytest.raises(hs.HHLSVError, match="INVALID"):
        hs.pf_mismatch_jacobian(bad, np.ones(5), np.zeros(5))
